"""Helpers shared by the GPU parity tests (no arithmetic of the method)."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_cs_0702135_amd._lib as L
    if not os.path.exists(L.LIB_PATH):
        raise RuntimeError("libnbody.so missing: build it before running GPU tests")


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    return t.detach().cpu().numpy()


def rel_vec_err(got, ref):
    """Per-particle |got - ref| / |ref| for (3, n) vectors."""
    num = np.sqrt(((got - ref) ** 2).sum(0))
    den = np.sqrt((ref ** 2).sum(0))
    return num / np.maximum(den, 1e-300)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()
