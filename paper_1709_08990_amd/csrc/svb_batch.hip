// Batched Stream VByte kernels (placeholder until the persistent batched path lands).
#include "svb_internal.hpp"

extern "C" {

int svb_encode_batch(uint32_t, const uint64_t *, const uint64_t *, const uint32_t *, const uint64_t *,
                     uint8_t *, uint64_t *, const uint32_t *, void *) {
    return SVB_ERR_INVALID;
}

int svb_decode_batch(uint32_t, const uint64_t *, const uint64_t *, const uint64_t *, const uint8_t *,
                     const uint64_t *, uint32_t *, const uint32_t *, uint32_t *, void *) {
    return SVB_ERR_INVALID;
}

}  // extern "C"
