"""Helpers shared by the GPU parity tests (no method arithmetic here)."""
import numpy as np


def normwise_err(gpu, ref, floor_scale=None):
    """Per-variable max |gpu - ref| / max |ref| (the parity metric for FP64
    fields that can be ~0 at some nodes).  floor_scale replaces a zero or tiny
    max |ref| (e.g. free-stream states)."""
    gpu = np.asarray(gpu)
    ref = np.asarray(ref)
    out = []
    for v in range(ref.shape[0]):
        scale = np.abs(ref[v]).max()
        if floor_scale is not None:
            scale = max(scale, floor_scale)
        if scale == 0.0:
            scale = 1.0
        out.append(np.abs(gpu[v] - ref[v]).max() / scale)
    return np.array(out)


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()
