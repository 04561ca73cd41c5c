"""The VALU issue-rate diagnostic (nbody_valu_rates) that states the pair
kernel's issue bound: every kind measured, float32 FMA within the published
float32 peak, float32 arithmetic issuing faster than the float64 adds and the
conversions, and those faster than the reciprocal square root."""
import pytest

pytestmark = pytest.mark.gpu


def test_rates():
    import paper_cs_0702135_amd as nb
    r = nb.valu_rates(8)
    assert list(r) == list(nb.VALU_KINDS)
    assert all(v > 0 for v in r.values())
    # 64 lanes x 2 flops per FMA: within the 157.3 TFLOP/s float32 peak
    assert r["v_fmac_f32"] * 64 * 2 <= 157.3e12 * 1.02
    assert r["v_fmac_f32"] > r["v_add_f64"] > r["v_rsq_f32"]
    assert r["v_mul_f32"] > r["v_cvt_f32_f64"] > r["v_rsq_f32"]


def test_bad_arguments():
    import paper_cs_0702135_amd as nb
    for w in (0, 9):
        with pytest.raises(nb.NBodyError):
            nb.valu_rates(w)
