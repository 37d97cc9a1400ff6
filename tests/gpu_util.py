"""Helpers for the GPU tests: device transfers and case logging (no codec arithmetic)."""
import sys

import numpy as np


def log_case(*parts):
    """Name the case about to run on the GPU (flushed, so a crash still shows it)."""
    sys.stderr.write("[gpu case] " + " ".join(str(p) for p in parts) + "\n")
    sys.stderr.flush()


def to_dev_u32(x):
    import torch
    a = np.ascontiguousarray(x, dtype=np.uint32).view(np.int32)
    return torch.from_numpy(a.copy()).cuda()


def to_dev_u8(s):
    import torch
    return torch.from_numpy(np.ascontiguousarray(s, dtype=np.uint8).copy()).cuda()


def u32_host(t):
    return t.detach().cpu().numpy().view(np.uint32)


def u8_host(t):
    return t.detach().cpu().numpy().astype(np.uint8)
