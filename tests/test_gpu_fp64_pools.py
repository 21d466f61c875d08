"""FP64 wave pools (MG_SCHED_POOLS_W8 on an FP64 set) against the FP64 lane
schedule and the oracle, through the C ABI.

Every particle consumes the random numbers of its own counters, so the pool
schedule gives the lane schedule's results bit for bit: positions, edges,
alive flags, hit-sequence hashes, hit counts, exit, absorbed and total
counts, histograms and streamed histograms, on graphs with each method
variant (absorbing vertices and the split cap, mirror leaves, cubic
coefficients, Wentzell vertices, semi-infinite edges), across launch chunks.
Against the oracle the bars of the FP64 path hold (hash agreement >= 99.99 %,
|dx| <= 1e-12 on the agreeing particles).
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_02175_amd import binding
    binding.lib()
    return binding


def _graph(case):
    if case == "config2":
        return workloads.config2()[0], 2, 1e-2, 8
    if case == "absorbing":
        g = workloads.star_graph(5, [0.3, 0.5, 0.2, 0.8, 0.4], [-30.0, 5.0, -60.0, 0.0, -10.0],
                                 [0, -2.0, 0, 0, 0], 1.0, b_center=[0.3, 0.1, 0.3, 0.2, 0.1])
        g.vtx_kind[2] = 1
        g.vtx_kind[5] = 1
        return g, 1, 5e-3, 3
    if case == "mirror":
        g, _ = workloads.config2()
        g = workloads.star_graph(g.n_edges, g.length, g.drift_a, g.drift_c, g.sigma,
                                 b_center=np.ones(g.n_edges), leaf_kind=2)
        return g, 2, 1e-2, 8
    if case == "cubic":
        return workloads.double_well_star(16), 2, 2e-3, 8
    if case == "wentzell":
        return workloads.wentzell_star(cubic=True), 1, 2e-3, 4
    if case == "semi_infinite":
        return workloads.paper_star5("quadratic"), 1, 1e-3, 8
    raise ValueError(case)


@pytest.mark.parametrize("case", ["config2", "absorbing", "mirror", "cubic", "wentzell",
                                  "semi_infinite"])
def test_fp64_pools_equal_lanes(B, case):
    g, mode, dt, M = _graph(case)
    n = 30_000
    G = B.mg_graph_create(g)
    out = []
    for sched in (B.MG_SCHED_LANES, B.MG_SCHED_POOLS_W8):
        print(f"fp64 pools vs lanes: {case} schedule={sched}", flush=True)
        p = B.mg_particles_init(G, n, mode, vertex=0, init_seed=3, trace=True, max_splits=M,
                                schedule=sched, steps_per_launch=173)
        B.mg_observe_histogram(p, 16, 7)
        B.mg_simulate(p, 400, dt, 19)
        B.mg_simulate(p, 211, dt, 19)
        out.append((B.mg_particles_read(p, trace=True), B.mg_exit_counts(p),
                    B.mg_observed_histogram(p), B.mg_histogram(p, 32)))
    (ra, ca, oa, ha), (rb, cb, ob, hb) = out
    for f in ("edge", "x", "alive", "seqhash", "hits"):
        assert np.array_equal(ra[f], rb[f]), f
    for x, y in zip(ca, cb):
        assert np.array_equal(x, y)
    assert oa[1] == ob[1] and np.array_equal(oa[0], ob[0])
    assert np.array_equal(ha, hb)
    assert int(ca[2][2]) > 0  # vertex hits happened


def test_fp64_pools_against_oracle(B, orc):
    """Config 2's star at both dt, 20k particles, 2000 steps on the FP64
    pools, particle by particle against the oracle."""
    g, run = workloads.config2()
    G = B.mg_graph_create(g)
    for dt in run["dts"]:
        st = orc.init(g, 20_000, 2, seed=5)
        c = orc.simulate(g, st, 0, 2000, dt, 3)
        p = B.mg_particles_init(G, 20_000, 2, init_seed=5, trace=True,
                                schedule=B.MG_SCHED_POOLS_W8)
        B.mg_simulate(p, 2000, dt, 3)
        r = B.mg_particles_read(p, trace=True)
        same = r["seqhash"] == st.seqhash
        assert same.mean() >= 0.9999, same.mean()
        assert np.array_equal(r["edge"][same], st.edge[same])
        assert np.abs(r["x"][same] - st.x[same]).max() <= 1e-12
        ex, ab, tot = B.mg_exit_counts(p)
        nd = int((~same).sum())
        assert np.abs(ex.astype(np.int64) - c.exit_slot.astype(np.int64)).sum() <= 2 * 2000 * nd
        assert int(tot[2]) == int(r["hits"].astype(np.int64).sum())


def test_fp64_schedule_validation(B):
    """FP64 sets take the lane schedule, the 8-step pools or the automatic
    choice; the FP32-only pool shapes are refused."""
    g, _ = workloads.config1()
    G = B.mg_graph_create(g)
    for sched in (B.MG_SCHED_POOLS, B.MG_SCHED_POOLS256):
        with pytest.raises(B.MgError):
            B.mg_particles_init(G, 100, 1, vertex=0, schedule=sched)
    t = B.mg_autotune(B.mg_particles_init(G, 100, 1, vertex=0), 1e-3)
    assert t["schedule"] in (B.MG_SCHED_LANES, B.MG_SCHED_POOLS_W8)
