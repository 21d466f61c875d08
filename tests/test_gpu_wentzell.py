"""GPU Wentzell vertices (Sec. 2.2's general gluing condition: killing a_v
and stickiness c_v), through the C ABI, against the FP64 oracle on the same
seeded inputs.

Bars (as for the standard step):
* FP64 path: hit sequences equal on >= 99.99 % of particles, |dx| <= 1e-12
  on those (positions of particles held on a vertex included: -t or L + t
  for a stay t still owed), edges, alive flags and hit counts equal; exit,
  absorbed, truncation and sub-step counts and the histogram within what
  the differing particles can move.
* FP32 path under common random numbers: histogram TV <= 2e-3 and
  exit-probability error <= 1e-3 against FP64; the fraction of particles
  killed and the fraction held on a vertex within 1e-3; the lane schedule
  and the wave pools bit for bit.
* Batched sets equal the sets run alone; a_v = c_v = 0 equals the standard
  vertex bit for bit.
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


def _tv(h1, h2):
    p, q = h1.astype(np.float64).ravel(), h2.astype(np.float64).ravel()
    return 0.5 * np.abs(p / p.sum() - q / q.sum()).sum()


def _exit_err(ex_a, ex_b, offsets, min_exits=10_000):
    worst = 0.0
    for v in range(offsets.size - 1):
        s0, s1 = offsets[v], offsets[v + 1]
        ta, tb = float(ex_a[s0:s1].sum()), float(ex_b[s0:s1].sum())
        if tb < min_exits:
            continue
        worst = max(worst, float(np.abs(ex_a[s0:s1] / max(ta, 1.0) - ex_b[s0:s1] / tb).max()))
    return worst


def _on_vertex(r, g):
    L = g.length[r["edge"]]
    return (r["x"] <= 0.0) | (r["x"] >= L)


@pytest.mark.parametrize("case", ["affine_uniform", "affine_at_vertex", "cubic_uniform"])
def test_wentzell_fp64_parity(B, orc, case):
    """FP64 particle by particle against the oracle: uniform starts and
    starts on the sticky, killing centre (every particle's first step is a
    visit), affine and cubic coefficients; 20k particles, 600 steps of 2e-3,
    M = 4, launches of 137 steps (a held particle's stay crosses launch
    boundaries)."""
    g = workloads.wentzell_star(cubic=case.startswith("cubic"))
    mode = 1 if case.endswith("at_vertex") else 2
    n, steps, dt, M, bins = 20_000, 600, 2e-3, 4, 32
    print(f"wentzell fp64 parity: {case} n={n} steps={steps}", flush=True)
    st = orc.init(g, n, mode, vertex=0, seed=4)
    c = orc.simulate(g, st, 0, steps, dt, 12, max_splits=M)
    assert c.absorbed.sum() > 0
    held = (st.x <= 0.0) | (st.x >= g.length[st.edge])
    assert (held & (st.alive == 1)).mean() > 0.05
    G = B.mg_graph_create(g)
    p = B.mg_particles_init(G, n, mode, vertex=0, init_seed=4, trace=True, max_splits=M,
                            steps_per_launch=137)
    B.mg_simulate(p, steps, dt, 12)
    r = B.mg_particles_read(p, trace=True)
    same = r["seqhash"] == st.seqhash
    nd = int((~same).sum())
    assert nd <= n // 10_000 + 1, nd
    assert np.array_equal(r["edge"][same], st.edge[same])
    assert np.array_equal(r["alive"][same], st.alive[same])
    assert np.array_equal(r["hits"][same], st.hits[same])
    dx = np.abs(r["x"][same] - st.x[same])
    assert dx.max(initial=0.0) <= 1e-12, dx.max()
    ex, ab, tot = B.mg_exit_counts(p)
    diff = ~same
    assert int(tot[2]) - c.hits == (int(r["hits"][diff].astype(np.int64).sum())
                                    - int(st.hits[diff].astype(np.int64).sum()))
    assert np.abs(ex.astype(np.int64) - c.exit_slot.astype(np.int64)).sum() <= 2 * steps * nd
    assert np.abs(ab.astype(np.int64) - c.absorbed.astype(np.int64)).sum() <= 2 * nd
    assert abs(int(tot[0]) - c.truncations) <= steps * nd
    both = int(r["hits"][diff].astype(np.int64).sum() + st.hits[diff].astype(np.int64).sum())
    assert abs(int(tot[1]) - c.substeps) <= both + steps * nd
    assert int((r["alive"] == 1).sum()) * steps <= int(tot[3]) <= n * steps
    h = B.mg_histogram(p, bins)
    ho = orc.histogram(g, st, bins)
    assert np.abs(h.astype(np.int64) - ho.astype(np.int64)).sum() <= 2 * nd


def test_wentzell_zero_terms_equal_standard_vertex(B):
    """a_v = c_v = 0 at a Wentzell centre gives the standard vertex's paths
    and counts bit for bit (FP64), its vertex-stream draws changing
    nothing."""
    g0 = workloads.config2()[0]
    g1 = workloads.config2()[0]
    g1.vtx_kind[0] = 3
    g1.vtx_kill = np.zeros(g1.n_vertices)
    g1.vtx_sticky = np.zeros(g1.n_vertices)
    out = []
    for g in (g0, g1):
        G = B.mg_graph_create(g)
        p = B.mg_particles_init(G, 30_000, 2, init_seed=3, trace=True)
        B.mg_simulate(p, 400, 1e-2, 11)
        out.append((B.mg_particles_read(p, trace=True), B.mg_exit_counts(p)))
    (ra, ca), (rb, cb) = out
    for f in ("edge", "x", "alive", "seqhash", "hits"):
        assert np.array_equal(ra[f], rb[f]), f
    for x, y in zip(ca, cb):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("cubic", [False, True])
def test_wentzell_fp32_against_fp64(B, cubic):
    """FP32 against FP64 under common random numbers, 1e6 particles, 2000
    steps of 2e-3 from the uniform law."""
    g = workloads.wentzell_star(cubic=cubic)
    n, steps, dt, bins = 1_000_000, 2000, 2e-3, 64
    print(f"wentzell fp32 vs fp64: cubic={cubic} n={n} steps={steps}", flush=True)
    G = B.mg_graph_create(g)
    res = {}
    for prec in (B.MG_FP64, B.MG_FP32):
        p = B.mg_particles_init(G, n, 2, init_seed=6, precision=prec)
        B.mg_simulate(p, steps, dt, 13)
        r = B.mg_particles_read(p)
        res[prec] = (B.mg_histogram(p, bins), B.mg_exit_counts(p), r)
    (h64, (ex64, ab64, _), r64), (h32, (ex32, ab32, _), r32) = res[B.MG_FP64], res[B.MG_FP32]
    assert _tv(h32, h64) <= 2e-3
    assert _exit_err(ex32, ex64, g.vtx_offsets) <= 1e-3
    assert ab64.sum() > 0.05 * n
    assert abs(int(ab32.sum()) - int(ab64.sum())) <= 1e-3 * n
    held64 = (_on_vertex(r64, g) & (r64["alive"] == 1)).mean()
    held32 = (_on_vertex(r32, g) & (r32["alive"] == 1)).mean()
    assert held64 > 0.05 and abs(held32 - held64) <= 1e-3, (held32, held64)
    same_edge = (r32["edge"] == r64["edge"]).mean()
    assert same_edge >= 0.999, same_edge


def test_wentzell_fp32_pools_equal_lanes(B):
    """The FP32 wave pools (128 per wave, 8-step windows: held particles are
    parked and visit in the split passes) give the lane schedule's results
    bit for bit, with the streamed histogram on."""
    g = workloads.wentzell_star(cubic=True)
    G = B.mg_graph_create(g)
    out = []
    for sched in (B.MG_SCHED_LANES, B.MG_SCHED_POOLS_W8, B.MG_SCHED_AUTO):
        p = B.mg_particles_init(G, 50_000, 1, vertex=0, init_seed=2, precision=B.MG_FP32,
                                trace=True, max_splits=3, schedule=sched)
        B.mg_observe_histogram(p, 16, 5)
        B.mg_simulate(p, 500, 2e-3, 21)
        B.mg_simulate(p, 333, 2e-3, 21)
        out.append((B.mg_particles_read(p, trace=True), B.mg_exit_counts(p),
                    B.mg_observed_histogram(p)))
    (ra, ca, oa) = out[0]
    for rb, cb, ob in out[1:]:
        for f in ("edge", "x", "alive", "seqhash", "hits"):
            assert np.array_equal(ra[f], rb[f]), f
        for x, y in zip(ca, cb):
            assert np.array_equal(x, y)
        assert oa[1] == ob[1] and np.array_equal(oa[0], ob[0])
    assert int(ca[1].sum()) > 0


@pytest.mark.parametrize("prec", [0, 1])
def test_wentzell_batch_equals_sets_alone(B, prec):
    """A batch of Wentzell stars (FP64: with a standard star beside them)
    gives each set's results as when it runs alone."""
    graphs = [workloads.wentzell_star(5, seed=7), workloads.wentzell_star(9, seed=8, cubic=True)]
    if prec == 0:
        graphs.append(workloads.config2()[0])
    Gs = [B.mg_graph_create(g) for g in graphs]
    counts = [20_000, 7_000, 9_000][: len(graphs)]

    def make():
        return [B.mg_particles_init(G, c, 2, init_seed=i, precision=prec, trace=True,
                                    graph_tag=i, max_splits=5)
                for i, (G, c) in enumerate(zip(Gs, counts))]
    alone = make()
    for p in alone:
        B.mg_simulate(p, 300, 2e-3, 17)
    batched = make()
    b = B.mg_batch_create(batched)
    B.mg_batch_simulate(b, 300, 2e-3, 17)
    for pa, pb in zip(alone, batched):
        ra, rb = B.mg_particles_read(pa, trace=True), B.mg_particles_read(pb, trace=True)
        for f in ("edge", "x", "alive", "seqhash", "hits"):
            assert np.array_equal(ra[f], rb[f]), f
        for x, y in zip(B.mg_exit_counts(pa), B.mg_exit_counts(pb)):
            assert np.array_equal(x, y)
