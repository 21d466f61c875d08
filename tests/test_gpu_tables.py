"""GPU tabulated coefficient functions (per-edge knot values and slopes of
the drift and diffusion, cubic Hermite interpolants), through the C ABI,
against the FP64 oracle on the same seeded inputs.

Bars: FP64 hit sequences equal the oracle's on >= 99.99 % of particles with
|dx| <= 1e-12 on those (the library evaluates each interval's cubic in
powers of the local coordinate, the oracle the Hermite basis: equal up to
rounding), histogram within what the differing particles move; FP32 against
FP64 under common random numbers within TV 2e-3 and exit-probability error
1e-3; FP32 and FP64 pools equal the lane schedules bit for bit; a table of a
cubic runs the cubic coefficients' paths on the GPU too.
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


@pytest.mark.parametrize("mode", [1, 2])
def test_tables_fp64_parity(B, orc, mode):
    """The periodic star (non-polynomial drift and diffusion tabulated at 16
    intervals per edge): 20k particles, 800 steps of 2e-3 from the centre or
    uniform, FP64 particle by particle against the oracle."""
    g = workloads.periodic_star()
    n, steps, dt, bins = 20_000, 800, 2e-3, 32
    print(f"tables fp64 parity: mode={mode}", flush=True)
    st = orc.init(g, n, mode, vertex=0, seed=2)
    c = orc.simulate(g, st, 0, steps, dt, 4)
    G = B.mg_graph_create(g)
    p = B.mg_particles_init(G, n, mode, vertex=0, init_seed=2, trace=True)
    B.mg_simulate(p, steps, dt, 4)
    r = B.mg_particles_read(p, trace=True)
    same = r["seqhash"] == st.seqhash
    nd = int((~same).sum())
    assert nd <= n // 10_000 + 1, nd
    assert np.array_equal(r["edge"][same], st.edge[same])
    assert np.abs(r["x"][same] - st.x[same]).max() <= 1e-12
    ex, ab, tot = B.mg_exit_counts(p)
    assert np.abs(ex.astype(np.int64) - c.exit_slot.astype(np.int64)).sum() <= 2 * steps * nd
    h = B.mg_histogram(p, bins)
    ho = orc.histogram(g, st, bins)
    assert np.abs(h.astype(np.int64) - ho.astype(np.int64)).sum() <= 2 * nd
    assert c.hits > 0


def test_tables_fp32_against_fp64_and_schedules(B):
    """FP32 against FP64 under common random numbers (1e6 particles, 2000
    steps of 2e-3), and both precisions' pools equal their lane schedules
    bit for bit."""
    g = workloads.periodic_star()
    G = B.mg_graph_create(g)
    n, steps, dt, bins = 1_000_000, 2000, 2e-3, 64
    res = {}
    for prec in (B.MG_FP64, B.MG_FP32):
        p = B.mg_particles_init(G, n, 2, init_seed=6, precision=prec)
        B.mg_simulate(p, steps, dt, 13)
        res[prec] = (B.mg_histogram(p, bins), B.mg_exit_counts(p)[0])
    assert _tv(res[B.MG_FP32][0], res[B.MG_FP64][0]) <= 2e-3
    ex32, ex64 = res[B.MG_FP32][1], res[B.MG_FP64][1]
    s0, s1 = g.vtx_offsets[0], g.vtx_offsets[1]
    p32 = ex32[s0:s1] / ex32[s0:s1].sum()
    p64 = ex64[s0:s1] / ex64[s0:s1].sum()
    assert np.abs(p32 - p64).max() <= 1e-3
    for prec in (B.MG_FP64, B.MG_FP32):
        out = []
        for sched in (B.MG_SCHED_LANES, B.MG_SCHED_POOLS_W8):
            p = B.mg_particles_init(G, 40_000, 1, vertex=0, init_seed=3, precision=prec,
                                    trace=True, schedule=sched)
            B.mg_simulate(p, 500, dt, 17)
            out.append(B.mg_particles_read(p, trace=True))
        for f in ("edge", "x", "alive", "seqhash", "hits"):
            assert np.array_equal(out[0][f], out[1][f]), (prec, f)


def test_table_of_a_cubic_runs_the_cubic_on_the_gpu(B):
    """The double-well star's cubics, tabulated at 3 intervals per edge,
    give the cubic coefficients' FP64 paths (the interpolant of a cubic is
    the cubic): the same hit sequences on >= 99.9 %, positions within 1e-9."""
    gc = workloads.double_well_star(16)
    d = lambda c: (c[1], 2 * c[2], 3 * c[3], np.zeros(16))

    def cubic(e, x, c):
        return c[0][e] + c[1][e] * x + c[2][e] * x ** 2 + c[3][e] * x ** 3
    mu = (gc.drift_a, gc.drift_c, gc.drift_c2, gc.drift_c3)
    sg = (gc.sigma, gc.sigma_c1, np.zeros(16), np.zeros(16))
    gt = workloads.double_well_star(16)
    gt.drift_c2 = gt.drift_c3 = gt.sigma_c1 = None
    workloads.tabulate(gt, 3, lambda e, x: cubic(e, x, mu), lambda e, x: cubic(e, x, d(mu)),
                       lambda e, x: cubic(e, x, sg), lambda e, x: cubic(e, x, d(sg)))
    out = []
    for g in (gc, gt):
        G = B.mg_graph_create(g)
        p = B.mg_particles_init(G, 50_000, 2, init_seed=8, trace=True)
        B.mg_simulate(p, 600, 2e-3, 5)
        out.append(B.mg_particles_read(p, trace=True))
    a, b = out
    same = a["seqhash"] == b["seqhash"]
    assert same.mean() >= 0.999
    assert np.abs(a["x"][same] - b["x"][same]).max() < 1e-9


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_of_cubic_tabulated_and_wentzell_graphs_equals_sets_alone(B, prec):
    """A batch runs the kernels of its most general graph: a cubic-coefficient
    star (run alone by the cubic instantiation) batched with a tabulated star
    and a Wentzell star (the full general one) gives each set's results as
    when it runs alone, in both precisions."""
    graphs = [workloads.double_well_star(16), workloads.periodic_star(),
              workloads.wentzell_star(5, seed=7)]
    Gs = [B.mg_graph_create(g) for g in graphs]
    counts = [30_000, 12_000, 9_000]

    def make():
        return [B.mg_particles_init(G, c, 2, init_seed=i, precision=prec, trace=True,
                                    graph_tag=i, max_splits=5)
                for i, (G, c) in enumerate(zip(Gs, counts))]
    print(f"level batch: precision={prec}", flush=True)
    alone = make()
    for p in alone:
        B.mg_simulate(p, 400, 2e-3, 23)
    batched = make()
    b = B.mg_batch_create(batched)
    B.mg_batch_simulate(b, 400, 2e-3, 23)
    for pa, pb in zip(alone, batched):
        ra, rb = B.mg_particles_read(pa, trace=True), B.mg_particles_read(pb, trace=True)
        for f in ("edge", "x", "alive", "seqhash", "hits"):
            assert np.array_equal(ra[f], rb[f]), f
        for x, y in zip(B.mg_exit_counts(pa), B.mg_exit_counts(pb)):
            assert np.array_equal(x, y)
        assert int(B.mg_exit_counts(pa)[2][2]) > 0
