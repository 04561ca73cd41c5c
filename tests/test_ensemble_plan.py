"""Host-side team planner of the batched ensemble (nbody_ensemble_plan).

The planner runs on the host only, so these checks need no GPU.  With at
least as many workgroups as clusters every cluster gets a team of its own
and spare groups go to the team with the longest modelled time while that
shortens it; with fewer, clusters are packed onto single-group teams, the
longest first onto the least loaded (LPT), whose makespan is within 4/3 of
the optimum.
"""
import numpy as np
import pytest

from workloads.plummer import CONFIGS, ensemble_members

CFG = {"groups_per_cu": 3, "max_team": 64, "step_us": 30.0, "barrier_us": 15.0,
       "barrier_group_us": 0.5, "group_rate": 2.0e9, "steps_coef": 247.0, "steps_exp": 0.35}


def _model(n, g, t_end=1.0 / 16, c=CFG):
    steps = max(1.0, c["steps_coef"] * n ** c["steps_exp"] * t_end)
    per = c["step_us"] * 1e-6 + (c["barrier_us"] + c["barrier_group_us"] * g) * 1e-6 * (g > 1) \
        + 0.20 * n ** 1.81 / (g * c["group_rate"])
    return steps * per


@pytest.fixture(scope="module")
def nb():
    try:
        import paper_cs_0702135_amd as m
        m._lib.load()
    except Exception as e:  # library not built
        pytest.skip("libnbody.so not built: %s" % e)
    return m


def test_spare_groups_go_to_the_slowest(nb):
    sizes, _, _ = ensemble_members(CONFIGS["ensemble256"])
    G = 768
    team_of, team_size, secs = nb.ensemble_plan(sizes, G, 1.0 / 16, CFG)
    nc = len(sizes)
    # one team per cluster, within the grid, within the team cap
    assert len(team_size) == nc and sorted(team_of) == list(range(nc))
    assert team_size.sum() <= G and team_size.max() <= 64 and team_size.min() >= 1
    g = team_size[team_of]
    # the modelled times are those of the model at the chosen team sizes
    want = np.array([_model(n, k) for n, k in zip(sizes, g)])
    np.testing.assert_allclose(secs, want, rtol=1e-12)
    # the plan shortens the slowest cluster relative to one group each
    assert secs.max() < max(_model(n, 1) for n in sizes)
    # greedy stopping rule: either the groups ran out, or the slowest team
    # cannot be shortened by one more group (or sits at the cap)
    slow = int(np.argmax(secs))
    assert (team_size.sum() == G or g[slow] == 64
            or _model(sizes[slow], g[slow] + 1) >= secs[slow])
    # larger clusters never get fewer groups than clearly smaller ones
    order = np.argsort(sizes)
    assert np.all(np.diff(g[order][::8]) >= -1)


def test_fewer_groups_than_clusters_is_lpt(nb):
    rng = np.random.default_rng(3)
    sizes = rng.integers(200, 5000, 97)
    G = 16
    team_of, team_size, secs = nb.ensemble_plan(sizes, G, 1.0 / 16, CFG)
    assert len(team_size) <= G and np.all(team_size == 1)
    t1 = np.array([_model(n, 1) for n in sizes])
    np.testing.assert_allclose(secs, t1, rtol=1e-12)
    load = np.bincount(team_of, weights=t1, minlength=len(team_size))
    lower = max(t1.sum() / G, t1.max())
    assert load.max() <= 4.0 / 3.0 * lower


def test_single_cluster_and_bad_arguments(nb):
    team_of, team_size, secs = nb.ensemble_plan([8192], 768, 1.0 / 16, CFG)
    assert list(team_of) == [0] and 1 <= team_size[0] <= 64
    with pytest.raises(nb.NBodyError):
        nb.ensemble_plan([100, 0], 8, 1.0 / 16, CFG)
    with pytest.raises(nb.NBodyError):
        nb.ensemble_plan([100], 0, 1.0 / 16, CFG)
    with pytest.raises(nb.NBodyError):
        nb.ensemble_plan([100], 8, 1.0 / 16, dict(CFG, group_rate=0.0))
