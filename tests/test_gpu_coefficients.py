"""General coefficient functions (cubic drift and diffusion, Sec. 2.2)
through the C ABI: the FP64 path against the oracle element by element on a
star and in the batched form, FP32 against FP64 under common random numbers
(lane and pool schedules, alone and batched), and graph validation."""
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


def _check_against_oracle(B, orc, g, p, n, steps, dt, seed, st, c):
    r = B.mg_particles_read(p, trace=True)
    same = r["seqhash"] == st.seqhash
    assert same.mean() >= 0.9999, same.mean()
    assert np.array_equal(r["edge"][same], st.edge[same])
    assert np.array_equal(r["hits"][same], st.hits[same])
    assert np.abs(r["x"][same] - st.x[same]).max() <= 1e-12
    nd = int((~same).sum())
    ex, _, tot = B.mg_exit_counts(p)
    assert np.abs(ex.astype(np.int64) - c.exit_slot.astype(np.int64)).sum() <= 2 * steps * nd
    if nd == 0:
        assert int(tot[1]) == c.substeps and int(tot[2]) == c.hits
    h = B.mg_histogram(p, 32)
    assert np.abs(h.astype(np.int64) - orc.histogram(g, st, 32).astype(np.int64)).sum() <= 2 * nd


def test_double_well_star_fp64_parity(B, orc):
    """The 64-edge double-well star (cubic drift, graded diffusion), 20k
    particles uniform by length, 1000 steps of 1e-2 in three calls: hit
    sequences, edges, positions, counters and bins against the oracle."""
    g = workloads.double_well_star()
    n, steps, dt = 20_000, 1000, 1e-2
    st = orc.init(g, n, orc.INIT_UNIFORM_LENGTH, seed=3)
    c = orc.simulate(g, st, 0, steps, dt, 14)
    G = B.mg_graph_create(g)
    p = B.mg_particles_init(G, n, B.MG_INIT_UNIFORM_LENGTH, init_seed=3,
                            precision=B.MG_FP64, trace=True)
    for k in (1, 499, 500):
        B.mg_simulate(p, k, dt, 14)
    _check_against_oracle(B, orc, g, p, n, steps, dt, 14, st, c)


def test_cubic_segment_and_batch_fp64(B, orc):
    """A segment with cubic drift and diffusion (the oracle's stationary
    pin's coefficients) against the oracle, and a batch of it with an affine
    star equal to the sets run alone."""
    g = workloads.segment(2.0, 12.0, -44.0, 1.0)
    g.drift_c2, g.drift_c3 = [48.0], [-16.0]
    g.sigma_c1, g.sigma_c2, g.sigma_c3 = [0.3], [-0.1], [0.02]
    n, steps, dt = 20_000, 600, 1e-3
    st = orc.init(g, n, orc.INIT_UNIFORM_LENGTH, seed=7)
    c = orc.simulate(g, st, 0, steps, dt, 5)
    G = B.mg_graph_create(g)
    p = B.mg_particles_init(G, n, B.MG_INIT_UNIFORM_LENGTH, init_seed=7,
                            precision=B.MG_FP64, trace=True)
    B.mg_simulate(p, steps, dt, 5)
    _check_against_oracle(B, orc, g, p, n, steps, dt, 5, st, c)
    star = workloads.star_graph(3, [1.0, 2.0, 0.5], [0.5, -1.0, 0.0], [-2.0, 0.3, 1.0], 1.2)
    Gs = B.mg_graph_create(star)
    pa = [B.mg_particles_init(G, 3000, B.MG_INIT_UNIFORM_LENGTH, init_seed=1,
                              precision=B.MG_FP64, trace=True),
          B.mg_particles_init(Gs, 2000, B.MG_INIT_UNIFORM_LENGTH, init_seed=2,
                              precision=B.MG_FP64, trace=True, graph_tag=1)]
    pb = [B.mg_particles_init(G, 3000, B.MG_INIT_UNIFORM_LENGTH, init_seed=1,
                              precision=B.MG_FP64, trace=True),
          B.mg_particles_init(Gs, 2000, B.MG_INIT_UNIFORM_LENGTH, init_seed=2,
                              precision=B.MG_FP64, trace=True, graph_tag=1)]
    b = B.mg_batch_create(pb)
    B.mg_batch_simulate(b, 200, 1e-3, 9)
    for q in pa:
        B.mg_simulate(q, 200, 1e-3, 9)
    for qa, qb in zip(pa, pb):
        ra, rb = B.mg_particles_read(qa, trace=True), B.mg_particles_read(qb, trace=True)
        for f in ("edge", "x", "seqhash", "hits"):
            assert np.array_equal(ra[f], rb[f]), f
        for x, y in zip(B.mg_exit_counts(qa), B.mg_exit_counts(qb)):
            assert np.array_equal(x, y)


def test_cubic_segment_with_mirror_ends(B, orc):
    """Cubic coefficients and mirror vertices together (the mirror branch
    of the cubic step): FP64 against the oracle element by element, FP32
    against FP64 in distribution, FP32 pools equal to FP32 lanes."""
    g = workloads.segment(2.0, 12.0, -44.0, 1.0, end_kind=2)
    g.drift_c2, g.drift_c3 = [48.0], [-16.0]
    g.sigma_c1, g.sigma_c2, g.sigma_c3 = [0.3], [-0.1], [0.02]
    n, steps, dt = 20_000, 600, 1e-3
    st = orc.init(g, n, orc.INIT_UNIFORM_LENGTH, seed=5)
    c = orc.simulate(g, st, 0, steps, dt, 6)
    G = B.mg_graph_create(g)
    p = B.mg_particles_init(G, n, B.MG_INIT_UNIFORM_LENGTH, init_seed=5,
                            precision=B.MG_FP64, trace=True)
    B.mg_simulate(p, steps, dt, 6)
    _check_against_oracle(B, orc, g, p, n, steps, dt, 6, st, c)
    h64 = B.mg_histogram(p, 40)
    res = {}
    for name, sched in (("lanes", B.MG_SCHED_LANES), ("pools_w8", B.MG_SCHED_POOLS_W8)):
        q = B.mg_particles_init(G, n, B.MG_INIT_UNIFORM_LENGTH, init_seed=5,
                                precision=B.MG_FP32, trace=True, schedule=sched)
        B.mg_simulate(q, steps, dt, 6)
        res[name] = (B.mg_histogram(q, 40), B.mg_particles_read(q, trace=True))
    h32, r32 = res["lanes"]
    assert 0.5 * np.abs(h32 / h32.sum() - h64 / h64.sum()).sum() <= 2e-3
    hp, rp = res["pools_w8"]
    assert np.array_equal(hp, h32)
    for f in ("edge", "x", "seqhash", "hits"):
        assert np.array_equal(rp[f], r32[f]), f


def test_double_well_star_fp32_against_fp64(B):
    """FP32 against FP64 on the double-well star under common random numbers:
    binned total variation <= 2e-3, exit probabilities at the centre within
    1e-3, most hit sequences equal; the lane schedule, the pools of 128 with
    8-step windows (AUTO's choice and asked for) and the batched form equal
    each other bit for bit."""
    g = workloads.double_well_star()
    G = B.mg_graph_create(g)
    n, dt, bins = 200_000, 1e-2, 64
    res = {}
    for name, prec, sched in (("fp64", B.MG_FP64, B.MG_SCHED_AUTO),
                              ("auto", B.MG_FP32, B.MG_SCHED_AUTO),
                              ("pools_w8", B.MG_FP32, B.MG_SCHED_POOLS_W8),
                              ("lanes", B.MG_FP32, B.MG_SCHED_LANES)):
        p = B.mg_particles_init(G, n, B.MG_INIT_UNIFORM_LENGTH, init_seed=6,
                                precision=prec, trace=True, schedule=sched)
        if name == "auto":
            assert B.mg_autotune(p, dt)["schedule"] == B.MG_SCHED_POOLS_W8
        for k in (3, 997, 1000):
            B.mg_simulate(p, k, dt, 21)
        res[name] = (B.mg_histogram(p, bins), B.mg_exit_counts(p),
                     B.mg_particles_read(p, trace=True))
    pb = B.mg_particles_init(G, n, B.MG_INIT_UNIFORM_LENGTH, init_seed=6,
                             precision=B.MG_FP32, trace=True)
    seg = workloads.segment(2.0, 12.0, -44.0, 1.0)
    seg.drift_c2, seg.drift_c3 = [48.0], [-16.0]
    other = B.mg_particles_init(B.mg_graph_create(seg), 3000, B.MG_INIT_UNIFORM_LENGTH,
                                init_seed=2, precision=B.MG_FP32, trace=True, graph_tag=1)
    b = B.mg_batch_create([pb, other])
    for k in (3, 997, 1000):
        B.mg_batch_simulate(b, k, dt, 21)
    res["batch"] = (B.mg_histogram(pb, bins), B.mg_exit_counts(pb),
                    B.mg_particles_read(pb, trace=True))
    h64, (e64, _, _), r64 = res["fp64"]
    h32, (e32, _, t32), r32 = res["lanes"]
    tv = 0.5 * np.abs(h32 / h32.sum() - h64 / h64.sum()).sum()
    assert tv <= 2e-3, tv
    c = slice(g.vtx_offsets[0], g.vtx_offsets[1])
    assert np.abs(e64[c] / e64[c].sum() - e32[c] / e32[c].sum()).max() <= 1e-3
    assert (r32["seqhash"] == r64["seqhash"]).mean() > 0.9
    # an FP32 batch cannot mix cubic and affine graphs
    aff = B.mg_particles_init(B.mg_graph_create(workloads.star_graph(3, 1.0)), 100,
                              B.MG_INIT_UNIFORM_LENGTH, precision=B.MG_FP32, trace=True,
                              graph_tag=2)
    with pytest.raises(B.MgError):
        B.mg_batch_create([pb, aff])
    for name in ("auto", "pools_w8", "batch"):
        h, (e, _, t), r = res[name]
        assert np.array_equal(h, h32) and np.array_equal(e, e32) and np.array_equal(t, t32)
        for f in ("edge", "x", "seqhash", "hits"):
            assert np.array_equal(r[f], r32[f]), (name, f)


def test_coefficient_validation(B):
    """FP32 sets on graphs with higher terms refuse the pool schedules other
    than pools of 128 with 8-step windows;
    sigma(x) must stay positive on the whole edge (an interior zero is
    caught); higher terms need finite edges and finite values; zero higher
    terms are affine."""
    g = workloads.double_well_star(8)
    G = B.mg_graph_create(g)
    for sched in (B.MG_SCHED_POOLS, B.MG_SCHED_POOLS256):
        with pytest.raises(B.MgError):
            B.mg_particles_init(G, 100, B.MG_INIT_UNIFORM_LENGTH, precision=B.MG_FP32,
                                schedule=sched)
    for sched in (B.MG_SCHED_LANES, B.MG_SCHED_POOLS_W8, B.MG_SCHED_AUTO):
        B.mg_particles_init(G, 100, B.MG_INIT_UNIFORM_LENGTH, precision=B.MG_FP32,
                            schedule=sched)
    bad = workloads.segment(2.0, 0.0, 0.0, 1.0)
    bad.sigma_c1, bad.sigma_c2 = [-4.0], [4.0]  # (1 - 2x)^2, zero at 0.5
    with pytest.raises(B.MgError):
        B.mg_graph_create(bad)
    bad.sigma_c1, bad.sigma_c2, bad.sigma_c3 = [0.0], [-3.0], [1.0]  # 1 - 3x^2 + x^3 < 0 at 1
    with pytest.raises(B.MgError):
        B.mg_graph_create(bad)
    inf = workloads.from_edges(2, [0], [1], [np.inf], [0.0], [0.0], 1.0, bin_span=2.0)
    inf.drift_c2 = [0.1]
    with pytest.raises(B.MgError):
        B.mg_graph_create(inf)
    nan = workloads.segment(1.0)
    nan.drift_c3 = [np.nan]
    with pytest.raises(B.MgError):
        B.mg_graph_create(nan)
    ok = workloads.segment(1.0)
    ok.drift_c2 = ok.drift_c3 = ok.sigma_c1 = ok.sigma_c2 = ok.sigma_c3 = [0.0]
    B.mg_particles_init(B.mg_graph_create(ok), 100, B.MG_INIT_UNIFORM_LENGTH,
                        precision=B.MG_FP32)


def test_streamed_histogram_with_cubic_coefficients(B, orc):
    """Streamed snapshots on the double-well star: FP64 against the oracle's
    streamed histogram, FP32 pools against FP32 lanes bit for bit."""
    g = workloads.double_well_star(16)
    G = B.mg_graph_create(g)
    n, dt, bins, every = 20_000, 1e-2, 32, 25
    p = B.mg_particles_init(G, n, B.MG_INIT_UNIFORM_LENGTH, init_seed=2,
                            precision=B.MG_FP64, trace=True)
    B.mg_observe_histogram(p, bins, every)
    for k in (7, 293, 200):
        B.mg_simulate(p, k, dt, 5)
    h, snaps = B.mg_observed_histogram(p)
    st = orc.init(g, n, orc.INIT_UNIFORM_LENGTH, seed=2)
    acc, osnaps, _ = orc.observed_histogram(g, st, 0, 500, dt, 5, every, bins)
    r = B.mg_particles_read(p, trace=True)
    nd = int((r["seqhash"] != st.seqhash).sum())
    assert nd <= n // 10_000 + 1, nd          # the bound below uses nd
    assert snaps == osnaps == 20
    assert np.abs(h.astype(np.int64).ravel() - acc.astype(np.int64).ravel()).sum() <= 2 * snaps * nd
    out = {}
    for name, sched in (("lanes", B.MG_SCHED_LANES), ("pools_w8", B.MG_SCHED_POOLS_W8)):
        q = B.mg_particles_init(G, n, B.MG_INIT_UNIFORM_LENGTH, init_seed=2,
                                precision=B.MG_FP32, schedule=sched)
        B.mg_observe_histogram(q, bins, every)
        for k in (7, 293, 200):
            B.mg_simulate(q, k, dt, 5)
        out[name] = B.mg_observed_histogram(q)
    assert out["lanes"][1] == out["pools_w8"][1] == 20
    assert np.array_equal(out["lanes"][0], out["pools_w8"][0])
    tv = 0.5 * np.abs(out["lanes"][0] / out["lanes"][0].sum() - h / h.sum()).sum()
    assert tv <= 2e-3, tv
