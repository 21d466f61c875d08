"""Mirror vertices (reflecting leaves: a proposal that leaves the edge
through one takes its mirror image when that lies inside the edge, the
far-end reflection of the paper's star-graph kernel in the appendix) through the C
ABI: the FP64 path against the oracle element by element, FP32 against FP64
under common random numbers, the FP32 schedules and the batched form against
each other bit for bit, the folded-normal law of one FP32 step at full
size, and graph validation."""
import numpy as np
import pytest
from scipy import stats

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


def _mixed_tree():
    """A random tree of 60 edges whose leaves are, in turn, mirror,
    absorbing and standard; quadratic potentials on the edges."""
    rng = np.random.default_rng(12)
    g = workloads.random_tree(60, rng, quadratic=True)
    deg = np.diff(g.vtx_offsets)
    leaves = np.flatnonzero(deg == 1)
    leaves = leaves[leaves != 0]
    g.vtx_kind[leaves[0::3]] = 2
    g.vtx_kind[leaves[1::3]] = 1
    return g


def _mixed_tree_cubic():
    """The mixed tree with a cubic drift term and a graded diffusion."""
    g = _mixed_tree()
    g.drift_c3 = np.full(g.n_edges, -0.2)
    g.sigma_c1 = np.full(g.n_edges, 0.1)
    return g


def _graphs():
    return {
        "brownian_star": workloads.star_graph(3, [0.5, 1.0, 1.5], sigma=1.0, leaf_kind=2),
        "langevin_star64": workloads.star_graph(
            **_config2_kwargs(), leaf_kind=2),
        "mixed_tree": _mixed_tree(),
        "mixed_tree_cubic": _mixed_tree_cubic(),
    }


def _config2_kwargs():
    g, _ = workloads.config2()
    return dict(n_edges=g.n_edges, length=g.length, drift_a=g.drift_a, drift_c=g.drift_c,
                sigma=g.sigma, b_center=np.ones(g.n_edges))


@pytest.mark.parametrize("name", ["brownian_star", "langevin_star64", "mixed_tree",
                                  "mixed_tree_cubic"])
def test_mirror_fp64_parity(B, orc, name):
    """20k particles uniform by length, 1000 steps of 1e-2 (leaves reached
    many times): hit sequences, edges, positions, exit and absorbed counts,
    hits and sub-steps against the oracle."""
    g = _graphs()[name]
    n, steps, dt = 20_000, 1000, 1e-2
    st = orc.init(g, n, orc.INIT_UNIFORM_LENGTH, seed=5)
    c = orc.simulate(g, st, 0, steps, dt, 17)
    G = B.mg_graph_create(g)
    p = B.mg_particles_init(G, n, B.MG_INIT_UNIFORM_LENGTH, init_seed=5,
                            precision=B.MG_FP64, trace=True)
    for k in (1, 499, 500):
        B.mg_simulate(p, k, dt, 17)
    r = B.mg_particles_read(p, trace=True)
    same = r["seqhash"] == st.seqhash
    assert same.mean() >= 0.9999, same.mean()
    assert np.array_equal(r["edge"][same], st.edge[same])
    assert np.array_equal(r["alive"][same], st.alive[same].astype(r["alive"].dtype))
    assert np.array_equal(r["hits"][same], st.hits[same])
    assert np.abs(r["x"][same] - st.x[same]).max() <= 1e-12
    nd = int((~same).sum())
    ex, ab, tot = B.mg_exit_counts(p)
    assert np.abs(ex.astype(np.int64) - c.exit_slot.astype(np.int64)).sum() <= 2 * steps * nd
    assert np.abs(ab.astype(np.int64) - c.absorbed.astype(np.int64)).sum() <= nd
    if not name.startswith("mixed_tree"):
        # on the stars no move is longer than an edge: a mirror leaf never
        # splits, so it records no exit (the tree's short edges do split
        # there now and then, as the oracle does)
        mslots = [g.vtx_offsets[v] for v in np.flatnonzero(g.vtx_kind == 2)]
        assert int(ex[mslots].sum()) == 0 and int(c.exit_slot[mslots].sum()) == 0
    if nd == 0:
        assert int(tot[2]) == c.hits and int(tot[0]) == c.truncations
    h = B.mg_histogram(p, 32)
    assert np.abs(h.astype(np.int64) - orc.histogram(g, st, 32).astype(np.int64)).sum() <= 2 * nd


def test_mirror_fp32_schedules_batch_and_fp64(B):
    """The 64-edge Langevin star with mirror leaves: FP32 against FP64 under
    common random numbers (binned total variation, exit probabilities at the
    centre); the lane, pool and window schedules and the batched form equal
    each other bit for bit."""
    g = workloads.star_graph(**_config2_kwargs(), leaf_kind=2)
    G = B.mg_graph_create(g)
    n, dt, bins = 200_000, 1e-2, 64
    res = {}
    for name, prec, sched in (("fp64", B.MG_FP64, B.MG_SCHED_AUTO),
                              ("lanes", B.MG_FP32, B.MG_SCHED_LANES),
                              ("pools", B.MG_FP32, B.MG_SCHED_POOLS),
                              ("pools256", B.MG_FP32, B.MG_SCHED_POOLS256),
                              ("pools_w8", B.MG_FP32, B.MG_SCHED_POOLS_W8)):
        p = B.mg_particles_init(G, n, B.MG_INIT_UNIFORM_LENGTH, init_seed=6,
                                precision=prec, trace=True, schedule=sched)
        for k in (3, 997, 1000):
            B.mg_simulate(p, k, dt, 21)
        res[name] = (B.mg_histogram(p, bins), B.mg_exit_counts(p),
                     B.mg_particles_read(p, trace=True))
    pb = B.mg_particles_init(G, n, B.MG_INIT_UNIFORM_LENGTH, init_seed=6,
                             precision=B.MG_FP32, trace=True)
    other = B.mg_particles_init(B.mg_graph_create(_mixed_tree()), 5000,
                                B.MG_INIT_UNIFORM_LENGTH, init_seed=2,
                                precision=B.MG_FP32, graph_tag=1, trace=True)
    b = B.mg_batch_create([pb, other])
    for k in (3, 997, 1000):
        B.mg_batch_simulate(b, k, dt, 21)
    res["batch"] = (B.mg_histogram(pb, bins), B.mg_exit_counts(pb),
                    B.mg_particles_read(pb, trace=True))
    h64, (e64, _, _), r64 = res["fp64"]
    h32, (e32, a32, t32), r32 = res["lanes"]
    tv = 0.5 * np.abs(h32 / h32.sum() - h64 / h64.sum()).sum()
    assert tv <= 2e-3, tv
    c = slice(g.vtx_offsets[0], g.vtx_offsets[1])
    p64, p32 = e64[c] / e64[c].sum(), e32[c] / e32[c].sum()
    assert np.abs(p64 - p32).max() <= 1e-3
    assert (r32["seqhash"] == r64["seqhash"]).mean() > 0.9
    # a leaf records an exit only after a move longer than its edge (a
    # normal beyond about 4.7 at the shortest edges): a handful in 4e8 steps
    steps_total = n * 2000
    for e in (e32, e64):
        assert int(e[g.vtx_offsets[1]:].sum()) <= 1e-7 * steps_total
    for name in ("pools", "pools256", "pools_w8", "batch"):
        h, (e, a, t), r = res[name]
        assert np.array_equal(h, h32) and np.array_equal(e, e32), name
        assert np.array_equal(t, t32), name
        for f in ("edge", "x", "seqhash", "hits"):
            assert np.array_equal(r[f], r32[f]), (name, f)


@pytest.mark.parametrize("a,x0", [(-8.0, 0.05), (6.0, 0.9)])
def test_mirror_fp32_one_step_law(B, a, x0):
    """One FP32 step on a segment with mirror ends from x0, 4M particles:
    the folded normal law of x0 + a dt + sigma sqrt(dt) Z on [0, L] (KS),
    no vertex hit, every position strictly inside."""
    L, sig, dt, n = 1.0, 0.5, 0.04, 4_000_000
    g = workloads.segment(L, a, 0.0, sig, end_kind=2)
    G = B.mg_graph_create(g)
    p = B.mg_particles_init(G, n, B.MG_INIT_EXPLICIT, edge=np.zeros(n),
                            pos=np.full(n, x0), precision=B.MG_FP32)
    B.mg_simulate(p, 1, dt, 33)
    x = B.mg_particles_read(p)["x"]
    _, _, tot = B.mg_exit_counts(p)
    assert int(tot[2]) == 0
    assert np.all((x > 0.0) & (x < L))
    m, s = x0 + a * dt, sig * np.sqrt(dt)
    F = stats.norm.cdf
    cdf = lambda y: ((F((y - m) / s) - F(-m / s)) + (F(-m / s) - F((-y - m) / s))
                     + (F((2 * L - m) / s) - F((2 * L - y - m) / s)))
    ks = stats.kstest(x, cdf)
    assert ks.pvalue > 1e-4, ks


def test_mirror_validation(B):
    """A mirror vertex must be a leaf; unknown kinds are rejected (kind 3 is a
    Wentzell vertex, which with a_v = c_v = 0 is a valid standard one)."""
    g = workloads.star_graph(3, 1.0)
    g.vtx_kind[0] = 2
    with pytest.raises(B.MgError):
        B.mg_graph_create(g)
    g.vtx_kind[0] = 4
    with pytest.raises(B.MgError):
        B.mg_graph_create(g)
    g.vtx_kind[0] = 3
    B.mg_graph_create(g)
    g.vtx_kind[0] = 0
    g.vtx_kind[1:] = 2
    B.mg_graph_create(g)
