"""The autotuner only proposes launch shapes the library accepts, and a
tuned table changes launch shapes, never results beyond float32 summation
order: pair sums under every candidate shape of a small block agree with
the oracle."""
import numpy as np
import pytest

from tests.gpu_util import dev, host, need_gpu
from workloads.plummer import plummer, random_active_set

pytestmark = pytest.mark.gpu


def test_every_candidate_shape_is_accepted():
    need_gpu()
    import paper_cs_0702135_amd as nb
    from paper_cs_0702135_amd import autotune
    try:
        for n_i in (16, 1024, 1 << 20):
            for shape in autotune.candidates(n_i, 1 << 20, forms=(0, 1, 2)):
                nb.tune_set(0, 1 << 62, shape)
    finally:
        nb.tune_clear()


def test_candidate_shapes_agree_with_oracle(orc):
    need_gpu()
    import paper_cs_0702135_amd as nb
    import torch
    from paper_cs_0702135_amd import autotune
    n = 3000
    pos, vel, m = plummer(n, 21)
    act = random_active_set(n, 300, 22)
    ra, _, _ = orc.force(pos, vel, m, 1e-4, active=act)
    P, V, M, A = dev(pos), dev(vel), dev(m), dev(act, torch.int32)
    try:
        for shape in autotune.candidates(300, n, forms=(0, 1)):
            nb.tune_set(0, 1 << 62, shape)
            a, _, _ = nb.force(P, V, M, 1e-4, A)
            err = np.linalg.norm(host(a) - ra, axis=0) / np.linalg.norm(ra, axis=0)
            assert err.max() < 1e-5, shape
    finally:
        nb.tune_clear()
