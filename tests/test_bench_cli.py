"""Host-side behaviour of bench.py that needs no GPU: a run on more than one
GPU is refused with a message (one GPU only; the sharding is a design note),
the description of the host the oracle runs on, and the arithmetic of the
roofline's issue bound are plain host code."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
    assert '"metric"' not in r.stdout


def test_host_cpu_description():
    sys.path.insert(0, ROOT)
    import bench
    h = bench.host_cpu()
    assert set(h) == {"model", "logical_cpus", "usable_cpus"}
    assert h["logical_cpus"] is None or h["logical_cpus"] >= 1


def test_valu_issue_bound_arithmetic(monkeypatch):
    """The bench line's issue bound: the counted wave instructions of each kind
    over that kind's issue rate, summed, and the fraction bound / kernel time
    (rates stubbed: this is host arithmetic)."""
    sys.path.insert(0, ROOT)
    import bench
    import paper_cs_0702135_amd as nb
    rates = {"v_fmac_f32": 1.0e12, "v_mul_f32": 1.0e12, "v_add_f64": 0.5e12,
             "v_cvt_f32_f64": 0.5e12, "v_rsq_f32": 0.25e12}
    monkeypatch.setattr(nb, "valu_rates", lambda waves_per_simd=8, device=None: dict(rates))
    c = {"SQ_INSTS_VALU_FMA_F32": 15e9, "SQ_INSTS_VALU_ADD_F32": 1e9, "SQ_INSTS_VALU_MUL_F32": 6e9,
         "SQ_INSTS_VALU_ADD_F64": 6e9, "SQ_INSTS_VALU_CVT": 6e9, "SQ_INSTS_VALU_TRANS_F32": 1e9}
    out = bench.valu_issue_bound({"counters_per_launch": c}, kernel_ms=50.0)
    # (16 + 6) / 1e12 + (6 + 6) / 0.5e12 + 1 / 0.25e12 seconds = 22 + 24 + 4 ms
    assert out["bound_ms"] == 50.0
    assert out["bound_ms_rsq_coissued"] == 46.0
    assert out["frac"] == 1.0 and out["frac_rsq_coissued"] == 0.92
    assert out["wave_instr_per_launch"]["v_fmac_f32"] == 16e9
