// Append without re-encoding (the paper's closing remark on adding integers
// to a stored stream: the data grow at the end and the control stream grows
// with them): the stream of n stored integers followed by k new ones is
// assembled from
//   - the old control bytes, copied, except the last partial one, which takes
//     the first new codes;
//   - the new integers' control bytes, shifted by 2 (n mod 4) bits;
//   - the old data bytes, copied unchanged;
//   - the new integers' data bytes.
// Only the new integers are encoded (by the single-stream encoder, into
// scratch); everything else is a byte copy at whatever alignments the streams
// have.
#include "svb_device.hpp"
#include "svb_internal.hpp"

namespace svb {

namespace {

struct CopyArgs {
    const uint8_t *src;
    uint8_t *dst;
    uint64_t len;             // bytes to copy, unless len_dev is set
    const uint64_t *len_dev;  // device count: *len_dev - len_sub bytes
    uint64_t len_sub;
    uint64_t *size_out;       // if set: receives size_base + the count
    uint64_t size_base;
};

// Copies the bytes [src, src + len) to [dst, dst + len) (no overlap).  Thread c
// writes the 16-byte aligned chunk c of dst's span: one 16-byte store for a
// chunk inside the range, byte stores for the two edge chunks.  Its 16 source
// bytes are cut out of the two aligned 16-byte chunks of src around them, each
// loaded only if it holds a byte of [src, src + len): an aligned chunk never
// straddles a page, so no load can fault.
__global__ __launch_bounds__(kThreads) void copy_bytes_kernel(CopyArgs a) {
    const uint64_t len = a.len_dev ? *a.len_dev - a.len_sub : a.len;
    const uint64_t c = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (c == 0 && a.size_out) *a.size_out = a.size_base + len;
    const uintptr_t d0 = (uintptr_t)a.dst, s0 = (uintptr_t)a.src;
    const uint32_t sh_d = (uint32_t)(d0 & 15u);
    const uint64_t nch = (sh_d + len + 15) >> 4;
    if (len == 0 || c >= nch) return;
    const uintptr_t A = (d0 - sh_d) + 16 * c;        // output chunk [A, A + 16)
    const uintptr_t S = s0 + 16 * c - sh_d;          // its source bytes start at S (may lie below src)
    const uintptr_t Sa = S & ~(uintptr_t)15;
    const uint32_t o = (uint32_t)(S & 15u);
    const uintptr_t s_end = s0 + len;
    u32x4a lo = {0u, 0u, 0u, 0u}, hi = {0u, 0u, 0u, 0u};
    if (Sa < s_end && Sa + 16 > s0) lo = *gptr((const u32x4a *)Sa);
    if (o && Sa + 16 < s_end && Sa + 32 > s0) hi = *gptr((const u32x4a *)(Sa + 16));
    const u32x4a win = shift_window(lo, hi, o);
    const uintptr_t d_end = d0 + len;
    if (A >= d0 && A + 16 <= d_end) {
        *gptr((u32x4a *)A) = win;
    } else {
        const uint32_t wv[4] = {win.x, win.y, win.z, win.w};
#pragma unroll
        for (uint32_t b = 0; b < 16; ++b) {
            const uintptr_t x = A + b;
            if (x >= d0 && x < d_end) gptr((uint8_t *)x)[0] = (uint8_t)(wv[b >> 2] >> (8u * (b & 3u)));
        }
    }
}

struct MergeArgs {
    const uint8_t *old_ctrl;  // the old stream (its control bytes)
    const uint8_t *new_ctrl;  // the new integers' control bytes (ceil(k/4), unused codes 0)
    uint8_t *out;
    uint64_t n, k;
};

// Control bytes floor(n/4) .. ceil((n + k)/4) - 1 of the result: the old
// partial byte's codes (n mod 4 of them) and the new codes shifted by 2 (n mod
// 4) bits.  One thread per byte.
__global__ __launch_bounds__(kThreads) void merge_ctrl_kernel(MergeArgs a) {
    const uint64_t b0 = a.n / 4;
    const uint64_t c_new = (a.n + a.k + 3) / 4, c_k = (a.k + 3) / 4;
    const uint64_t b = b0 + (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (b >= c_new) return;
    const uint32_t r = (uint32_t)(a.n & 3u);
    const uint64_t q = b - b0;  // new control byte holding the codes that land at bits 2r.. of byte b
    const uint32_t cur = q < c_k ? gptr(a.new_ctrl)[q] : 0u;
    uint32_t v;
    if (r == 0) {
        v = cur;
    } else {
        const uint32_t prev = q ? gptr(a.new_ctrl)[q - 1] : 0u;
        v = ((cur << (2 * r)) | (prev >> (8 - 2 * r))) & 0xFFu;
        if (q == 0) v |= gptr(a.old_ctrl)[b0] & ((1u << (2 * r)) - 1u);
    }
    gptr(a.out)[b] = (uint8_t)v;
}

uint32_t grid_for(uint64_t threads) { return (uint32_t)((threads + kThreads - 1) / kThreads); }

}  // namespace

hipError_t launch_copy_bytes(const uint8_t *src, uint8_t *dst, uint64_t len_max, const uint64_t *len_dev,
                             uint64_t len_sub, uint64_t *size_out, uint64_t size_base, hipStream_t s) {
    CopyArgs a = {src, dst, len_max, len_dev, len_sub, size_out, size_base};
    if (len_max == 0 && !size_out) return hipSuccess;
    const uint64_t chunks = len_max ? (15 + len_max + 15) / 16 : 1;  // at most 15 bytes before dst's first chunk
    hipLaunchKernelGGL(copy_bytes_kernel, dim3(grid_for(chunks)), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_merge_ctrl(const uint8_t *old_ctrl, const uint8_t *new_ctrl, uint8_t *out, uint64_t n, uint64_t k,
                             hipStream_t s) {
    const uint64_t bytes = (n + k + 3) / 4 - n / 4;
    if (bytes == 0) return hipSuccess;
    MergeArgs a = {old_ctrl, new_ctrl, out, n, k};
    hipLaunchKernelGGL(merge_ctrl_kernel, dim3(grid_for(bytes)), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace svb
