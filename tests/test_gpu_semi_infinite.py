"""Semi-infinite edges (Def. 1 allows l_e = inf; the paper's star metric
graphs, Def. 3, have only such edges) through the C ABI: the FP64 path
against the oracle element by element, FP32 against FP64 under common
random numbers, the FP32 schedules against each other bit for bit, and the
calls that need finite edges."""
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


def _graph(potential):
    return workloads.paper_star5(potential, length=np.inf)


@pytest.mark.parametrize("potential", ["linear", "quadratic"])
def test_semi_infinite_star_fp64_parity(B, orc, potential):
    """The paper's 5-edge star with semi-infinite edges, 20k particles from
    the vertex, 1500 steps of 1e-3 (a hit on most steps near the vertex):
    hit sequences, edges, positions, exit counts and binned counts against
    the oracle."""
    g = _graph(potential)
    n, steps, dt = 20_000, 1500, 1e-3
    st = orc.init(g, n, orc.INIT_AT_VERTEX, vertex=0, seed=4)
    c = orc.simulate(g, st, 0, steps, dt, 9)
    G = B.mg_graph_create(g)
    p = B.mg_particles_init(G, n, B.MG_INIT_AT_VERTEX, vertex=0, init_seed=4,
                            precision=B.MG_FP64, trace=True)
    B.mg_simulate(p, steps, dt, 9)
    r = B.mg_particles_read(p, trace=True)
    same = r["seqhash"] == st.seqhash
    assert same.mean() >= 0.9999, same.mean()
    assert np.array_equal(r["edge"][same], st.edge[same])
    assert np.abs(r["x"][same] - st.x[same]).max() <= 1e-12
    assert np.all(np.isfinite(r["x"]))
    nd = int((~same).sum())
    ex, ab, tot = B.mg_exit_counts(p)
    assert np.abs(ex.astype(np.int64) - c.exit_slot.astype(np.int64)).sum() <= 2 * steps * nd
    far = [s for s in range(g.nnz) if g.slot_orient[s] == 1]
    assert int(ex[far].sum()) == 0
    off, up, _ = workloads.csr_bins(g, 0.02, 40)
    h = B.mg_histogram_csr(p, off, up)
    ho = orc.histogram_csr(g, st, off, up)
    assert np.abs(h.astype(np.int64) - ho.astype(np.int64)).sum() <= 2 * nd


def test_semi_infinite_star_fp32_against_fp64(B):
    """FP32 against FP64 on the semi-infinite quadratic star under common
    random numbers: binned total variation <= 2e-3, exit probabilities within
    1e-3, and the pool schedules equal the lane schedule bit for bit."""
    g = _graph("quadratic")
    G = B.mg_graph_create(g)
    n, steps, dt = 200_000, 2000, 1e-3
    off, up, _ = workloads.csr_bins(g, 0.02, 40)
    res = {}
    for name, prec, sched in (("fp64", B.MG_FP64, B.MG_SCHED_AUTO),
                              ("lanes", B.MG_FP32, B.MG_SCHED_LANES),
                              ("pools", B.MG_FP32, B.MG_SCHED_POOLS),
                              ("pools_w8", B.MG_FP32, B.MG_SCHED_POOLS_W8)):
        p = B.mg_particles_init(G, n, B.MG_INIT_AT_VERTEX, vertex=0, init_seed=6,
                                precision=prec, trace=True, schedule=sched)
        for k in (3, 997, 1000):
            B.mg_simulate(p, k, dt, 21)
        res[name] = (B.mg_histogram_csr(p, off, up), B.mg_exit_counts(p)[0],
                     B.mg_particles_read(p, trace=True))
    h64, e64, r64 = res["fp64"]
    h32, e32, r32 = res["lanes"]
    tv = 0.5 * np.abs(h32 / h32.sum() - h64 / h64.sum()).sum()
    assert tv <= 2e-3, tv
    v = np.asarray(g.vtx_offsets)
    for e_a, e_b in ((e32, e64),):
        pa = e_a[v[0]:v[1]] / max(e_a[v[0]:v[1]].sum(), 1)
        pb = e_b[v[0]:v[1]] / max(e_b[v[0]:v[1]].sum(), 1)
        assert np.abs(pa - pb).max() <= 1e-3
    assert (r32["seqhash"] == r64["seqhash"]).mean() > 0.95
    for name in ("pools", "pools_w8"):
        h, e, r = res[name]
        assert np.array_equal(h, h32) and np.array_equal(e, e32), name
        for f in ("edge", "x", "seqhash", "hits"):
            assert np.array_equal(r[f], r32[f]), (name, f)


def test_init_rules_and_uniform_bins_on_a_span(B, orc):
    """Uniform-by-length init and a start on a vertex at infinity are
    rejected; uniform bins (one-off and streamed) cover each edge's bin span
    with everything beyond in the last bin, as the oracle counts them."""
    g = _graph("linear")
    G = B.mg_graph_create(g)
    with pytest.raises(B.MgError):
        B.mg_particles_init(G, 100, B.MG_INIT_UNIFORM_LENGTH)
    with pytest.raises(B.MgError):           # a vertex at infinity
        B.mg_particles_init(G, 100, B.MG_INIT_AT_VERTEX, vertex=1)
    edge, pos = [0, 0, 1, 4, 2], [0.0, 1.99, 2.0, 1e6, 0.5]
    st = orc.init(g, 5, orc.INIT_EXPLICIT, edge=edge, pos=pos)
    for prec in (B.MG_FP64, B.MG_FP32):
        q = B.mg_particles_init(G, 5, B.MG_INIT_EXPLICIT, edge=edge, pos=pos, precision=prec)
        assert np.array_equal(B.mg_histogram(q, 8), orc.histogram(g, st, 8))
    # streamed snapshots on the semi-infinite star against the oracle's
    n, dt, bins = 20_000, 1e-3, 50
    p = B.mg_particles_init(G, n, B.MG_INIT_AT_VERTEX, vertex=0, init_seed=2,
                            precision=B.MG_FP64, trace=True)
    B.mg_observe_histogram(p, bins, 25)
    for k in (7, 293, 200):
        B.mg_simulate(p, k, dt, 5)
    h, snaps = B.mg_observed_histogram(p)
    st = orc.init(g, n, orc.INIT_AT_VERTEX, vertex=0, seed=2)
    acc, osnaps, _ = orc.observed_histogram(g, st, 0, 500, dt, 5, 25, bins)
    r = B.mg_particles_read(p, trace=True)
    nd = int((r["seqhash"] != st.seqhash).sum())
    assert nd <= n // 10_000 + 1, nd          # the bound below uses nd
    assert snaps == osnaps == 20
    assert np.abs(h.astype(np.int64).ravel() - acc.astype(np.int64).ravel()).sum() <= 2 * snaps * nd
    # a semi-infinite edge needs a bin span
    g.bin_span = None
    with pytest.raises(B.MgError):
        B.mg_graph_create(g)
    # a span shorter than a finite edge: the last bin takes the rest
    f = workloads.star_graph(3, [1.0, 2.0, 3.0], sigma=1.0, bin_span=[1.0, 0.5, 3.0])
    Gf = B.mg_graph_create(f)
    st = orc.init(f, 20_000, orc.INIT_UNIFORM_LENGTH, seed=8)
    for prec in (B.MG_FP64, B.MG_FP32):
        q = B.mg_particles_init(Gf, 20_000, B.MG_INIT_UNIFORM_LENGTH, init_seed=8, precision=prec)
        assert np.array_equal(B.mg_histogram(q, 10), orc.histogram(f, st, 10))


def test_semi_infinite_graph_validation(B):
    """A semi-infinite edge's terminal vertex must hold only that edge's end;
    NaN and non-positive lengths are rejected."""
    bad = workloads.from_edges(3, [0, 1], [1, 2], [np.inf, 1.0], bin_span=1.0)  # vertex 1 also starts edge 1
    with pytest.raises(B.MgError):
        B.mg_graph_create(bad)
    for L in (np.nan, -np.inf, 0.0):
        with pytest.raises(B.MgError):
            B.mg_graph_create(workloads.from_edges(2, [0], [1], [L]))
    ok = workloads.from_edges(3, [0, 1], [1, 2], [1.0, np.inf], bin_span=[1.0, 5.0])  # a segment then a half-line
    B.mg_graph_create(ok)
