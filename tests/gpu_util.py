"""Helpers for the GPU parity tests (host-side only)."""
import numpy as np
import pytest
import torch


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def kpa_mod():
    import paper_1901_01328_amd as P
    return P.load()


def u64(t):
    return t.detach().cpu().numpy().view(np.uint64)


def u32(t):
    return t.detach().cpu().numpy().view(np.uint32)


def dev_u64(a, device="cuda"):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.uint64))
    return torch.from_numpy(a.view(np.int64)).to(device)


def dev_u32(a, device="cuda"):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.uint32))
    return torch.from_numpy(a.view(np.int32)).to(device)


def say(msg):
    print(msg, flush=True)
