"""Helpers for GPU tests: pack numpy entries into device tensor buffers."""
import numpy as np


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch


def to_dev(torch, val, res):
    """(int32 values [E], uint32 residues [k, E]) -> int32 device buffer of
    (1 + k) * E words: value plane, then residue planes."""
    val = np.ascontiguousarray(val, dtype=np.int32).reshape(-1)
    res = np.ascontiguousarray(res, dtype=np.uint32).reshape(res.shape[0], val.size)
    host = np.concatenate([val.view(np.int32), res.view(np.int32).reshape(-1)])
    return torch.from_numpy(host).to("cuda")


def from_dev(buf, k, E):
    h = buf.cpu().numpy().astype(np.int32)
    val = h[:E].copy()
    res = h[E:E * (1 + k)].view(np.uint32).reshape(k, E).copy()
    return val, res


def empty_dev(torch, k, E):
    return torch.full(((1 + k) * E,), -7, dtype=torch.int32, device="cuda")
