"""The launch tables shipped in paper_cs_0702135_amd/tuned/ hold only shapes the
library accepts (the rules of nbody_tune_set) and planning models it can use,
so installing them can never fail on the GPU."""
import glob
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TUNED = os.path.join(ROOT, "paper_cs_0702135_amd", "tuned")


def _shape_ok(s):
    common = s["tile"] >= 1 and s["min_j_wave"] >= 1 and 1 <= s["target_groups"] <= (1 << 20)
    if s.get("layout", 0) == 1:
        return (common and s["rep"] == 0 and s["i_per_lane"] in (1, 2, 4, 8)
                and s["waves"] in (1, 2, 4))
    return (common and s.get("layout", 0) == 0 and s["rep"] in (0, 1, 2)
            and s["i_per_lane"] in (1, 2, 4) and s["waves"] in (1, 2, 4, 8)
            and not (s["i_per_lane"] == 4 and s["waves"] == 8))


def test_force_tables_hold_accepted_shapes():
    files = glob.glob(os.path.join(TUNED, "*_nj*_*.json"))
    assert files, "no tuned launch table shipped"
    for f in files:
        t = json.load(open(f))
        assert t["mode"] in ("fp32", "ds") and t["n_j"] >= 1
        sizes = [e[0] for e in t["entries"]]
        assert sizes == sorted(sizes) and len(set(sizes)) == len(sizes)
        for n_i, shape, ms in t["entries"]:
            assert n_i >= 1 and ms > 0, f
            assert set(shape) - {"layout"} == {"rep", "i_per_lane", "waves", "tile",
                                               "min_j_wave", "target_groups"}, f
            assert _shape_ok(shape), (f, n_i, shape)


def test_ensemble_models_are_usable():
    files = glob.glob(os.path.join(TUNED, "*_ensemble_*.json"))
    assert files
    for f in files:
        c = json.load(open(f))
        assert c["groups_per_cu"] >= 1 and 1 <= c["max_team"] <= 64
        assert c["group_rate"] > 0 and c["steps_coef"] > 0
        assert c["tile_us"] >= 0 and c["block_coef"] > 0 and 0 <= c["block_exp"] <= 1
        assert c["step_us"] >= 0 and c["barrier_us"] >= 0 and c["barrier_group_us"] >= 0
        # a workgroup shape the library compiles (autotune.ENS_SHAPES)
        from paper_cs_0702135_amd.autotune import ENS_SHAPES
        assert (c["waves"], c["j_tile"], c["i_per_lane"]) in ENS_SHAPES
