"""Host-side team planner of the batched ensemble (nbody_ensemble_plan).

The planner runs on the host only, so these checks need no GPU.  It
minimises the modelled makespan: clusters that one group finishes within the
target share single-group teams, the others get the fewest groups that
finish them within it, the target is the least one whose plan fits the grid,
and spare groups then go to the slowest teams.  The checks: every cluster in
exactly one team, the team cap and the grid respected, the reported times
equal to the model at the chosen team sizes, and a makespan no longer than
that of the simple plan (one team per cluster, spare groups to the slowest)
or, with fewer groups than clusters, within 4/3 of the lower bound.
"""
import numpy as np
import pytest

from workloads.plummer import CONFIGS, ensemble_members

CFG = {"groups_per_cu": 3, "max_team": 64, "step_us": 30.0, "barrier_us": 15.0,
       "barrier_group_us": 0.5, "group_rate": 2.0e9, "steps_coef": 247.0, "steps_exp": 0.35,
       "waves": 4, "j_tile": 256, "i_per_lane": 2, "tile_us": 6.0, "block_coef": 0.9,
       "block_exp": 0.62}


def _pass(n_i, n, g, c):
    from paper_cs_0702135_amd.autotune import ens_tiles
    tiles = ens_tiles(int(np.ceil(n_i)), n, g, 64 * c["i_per_lane"], c["j_tile"])
    return tiles * c["tile_us"] * 1e-6 + n_i * n / (g * c["group_rate"])


def _model(n, g, t_end=1.0 / 16, c=CFG):
    n = int(n)
    steps = max(1.0, c["steps_coef"] * n ** c["steps_exp"] * t_end)
    block = min(n, max(1.0, c["block_coef"] * n ** c["block_exp"]))
    fixed = c["step_us"] * 1e-6 + (c["barrier_us"] + c["barrier_group_us"] * g) * 1e-6 * (g > 1)
    return _pass(n, n, g, c) + steps * (fixed + _pass(block, n, g, c))


@pytest.fixture(scope="module")
def nb():
    try:
        import paper_cs_0702135_amd as m
        m._lib.load()
    except Exception as e:  # library not built
        pytest.skip("libnbody.so not built: %s" % e)
    return m


def _simple_plan_makespan(sizes, G, cap=64):
    """One team per cluster, spare groups one at a time to the slowest team."""
    g = np.ones(len(sizes), dtype=int)
    t = np.array([_model(n, 1) for n in sizes])
    spare = G - len(sizes)
    while spare > 0:
        c = int(np.argmax(t))
        if g[c] >= cap or _model(sizes[c], g[c] + 1) >= t[c]:
            break
        g[c] += 1
        t[c] = _model(sizes[c], g[c])
        spare -= 1
    return t.max()


def _check_plan(sizes, G, team_of, team_size, secs):
    nt = len(team_size)
    assert team_of.min() >= 0 and team_of.max() < nt
    assert len(np.unique(team_of)) == nt  # no empty team
    assert team_size.sum() <= G and team_size.max() <= 64 and team_size.min() >= 1
    g = team_size[team_of]
    want = np.array([_model(n, k) for n, k in zip(sizes, g)])
    np.testing.assert_allclose(secs, want, rtol=1e-12)
    # a team of several clusters runs them one after another on one group
    multi = np.bincount(team_of, minlength=nt) > 1
    assert np.all(team_size[multi] == 1)
    return np.bincount(team_of, weights=secs, minlength=nt)


def test_makespan_plan_on_the_workload(nb):
    sizes, _, _ = ensemble_members(CONFIGS["ensemble256"])
    G = 768
    team_of, team_size, secs = nb.ensemble_plan(sizes, G, 1.0 / 16, CFG)
    load = _check_plan(sizes, G, team_of, team_size, secs)
    makespan = load.max()
    assert makespan <= _simple_plan_makespan(sizes, G) * (1 + 1e-9)
    # small clusters share groups: fewer teams than clusters
    assert len(team_size) < len(sizes)
    # no cluster can finish faster than its best team size allows
    best = max(min(_model(n, k) for k in range(1, 65)) for n in sizes)
    assert makespan >= best * (1 - 1e-12)
    # greedy stopping rule for the spare groups: either they ran out, or the
    # slowest team cannot be shortened by one more group (or sits at the cap)
    slow = int(np.argmax(load))
    on_slow = team_of == slow
    more = sum(_model(n, team_size[slow] + 1) for n in sizes[on_slow])
    assert (team_size.sum() == G or team_size[slow] == 64 or more >= load[slow])


def test_makespan_plan_larger_grids_never_slower(nb):
    sizes, _, _ = ensemble_members(CONFIGS["ensemble256"])
    prev = np.inf
    for G in (256, 512, 768, 1024):
        team_of, team_size, secs = nb.ensemble_plan(sizes, G, 1.0 / 16, CFG)
        m = _check_plan(sizes, G, team_of, team_size, secs).max()
        assert m <= prev * (1 + 1e-6)
        prev = m


def test_fewer_groups_than_clusters(nb):
    rng = np.random.default_rng(3)
    sizes = rng.integers(200, 5000, 97)
    G = 16
    team_of, team_size, secs = nb.ensemble_plan(sizes, G, 1.0 / 16, CFG)
    load = _check_plan(sizes, G, team_of, team_size, secs)
    assert len(team_size) <= G
    t1 = np.array([_model(n, 1) for n in sizes])
    lower = max(t1.sum() / G, max(min(_model(n, k) for k in range(1, 65)) for n in sizes))
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
