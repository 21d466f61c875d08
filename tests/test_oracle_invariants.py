"""Exact invariants of the oracle: decomposition independence (the random
numbers are keyed by particle, step and hit, not by schedule), mass
conservation, histogram definition, initial laws."""
import numpy as np
from scipy import stats

import workloads


def _c2_small(orc, n=4000, seed=0):
    g, run = workloads.config2()
    st = orc.init(g, n, orc.INIT_UNIFORM_LENGTH, seed=seed)
    return g, st


def test_split_run_equals_single_run(orc):
    g, st = _c2_small(orc)
    a = st.copy()
    b = st.copy()
    ca = orc.simulate(g, a, 0, 1000, 1e-2, 17)
    cb = orc.simulate(g, b, 0, 500, 1e-2, 17)
    cb = orc.simulate(g, b, 500, 300, 1e-2, 17, counts=cb)
    cb = orc.simulate(g, b, 800, 200, 1e-2, 17, counts=cb)
    for f in ("edge", "x", "alive", "seqhash", "hits"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
    assert np.array_equal(ca.exit_slot, cb.exit_slot)
    assert (ca.substeps, ca.hits, ca.truncations) == (cb.substeps, cb.hits, cb.truncations)


def test_subset_and_thread_count_independence(orc):
    g, st = _c2_small(orc)
    full = st.copy()
    orc.simulate(g, full, 0, 300, 1e-2, 5, threads=8)
    idx = np.array([0, 7, 123, 3999, 2500])
    sub = st.take(idx)
    orc.simulate(g, sub, 0, 300, 1e-2, 5, threads=1)
    for f in ("edge", "x", "alive", "seqhash", "hits"):
        assert np.array_equal(getattr(full, f)[idx], getattr(sub, f)), f
    # the init stream is keyed by particle index too
    sub0 = orc.init(g, 4000, orc.INIT_UNIFORM_LENGTH, seed=0, pids=idx)
    assert np.array_equal(sub0.edge, st.edge[idx]) and np.array_equal(sub0.x, st.x[idx])


def test_seed_and_tag_change_the_paths(orc):
    g, st = _c2_small(orc, n=500)
    a, b, c = st.copy(), st.copy(), st.copy()
    orc.simulate(g, a, 0, 100, 1e-2, 1)
    orc.simulate(g, b, 0, 100, 1e-2, 2)
    orc.simulate(g, c, 0, 100, 1e-2, 1, tag=3)
    assert np.mean(a.x == b.x) < 0.01 and np.mean(a.x == c.x) < 0.01


def test_mass_histogram_and_hits_consistency(orc):
    # a graph with absorbing vertices: a star whose leaves 1 and 2 absorb
    g = workloads.star_graph(4, [1.0, 0.5, 2.0, 1.5], [0.5, -1.0, 0.0, 2.0], [0, 0, -1.0, 0], 1.0,
                             b_center=[0.4, 0.1, 0.3, 0.2])
    g.vtx_kind[1] = 1
    g.vtx_kind[2] = 1
    N = 50_000
    st = orc.init(g, N, orc.INIT_AT_VERTEX, vertex=0, seed=4)
    c = orc.simulate(g, st, 0, 400, 2e-3, 6)
    alive = int(st.alive.sum())
    assert alive + int(c.absorbed.sum()) == N
    assert c.absorbed[0] == 0 and c.absorbed[3] == 0 and c.absorbed[4] == 0
    assert c.absorbed[1] > 0 and c.absorbed[2] > 0
    h = orc.histogram(g, st, 37)
    assert int(h.sum()) == alive
    assert int(st.hits.sum()) == c.hits
    # substeps = steps of alive-at-start particles + continuations; every
    # hit either ends the step (absorbed, zero time left, cap) or continues
    assert c.substeps >= N
    # histogram against the plain definition: bins of width L/nb
    for e in range(g.n_edges):
        sel = (st.edge == e) & (st.alive == 1)
        L = g.length[e]
        ref = np.histogram(st.x[sel], np.linspace(0, L, 38))[0]
        # floor(x nb / L) and comparison with k L / nb can differ only for x
        # within an ulp of a bin edge
        assert np.abs(ref.astype(np.int64) - h[e].astype(np.int64)).sum() <= 2


def test_init_laws(orc):
    # uniform by length: edge frequencies proportional to L, positions U[0, L]
    g, run = workloads.config2()
    N = 400_000
    st = orc.init(g, N, orc.INIT_UNIFORM_LENGTH, seed=9)
    p = g.length / g.length.sum()
    cnt = np.bincount(st.edge, minlength=g.n_edges)
    chi2 = ((cnt - p * N) ** 2 / (p * N)).sum()
    assert stats.chi2.sf(chi2, g.n_edges - 1) > 1e-4
    u = st.x / g.length[st.edge]
    assert stats.kstest(u, "uniform").pvalue > 1e-4
    assert np.all((st.x > 0) & (st.x < g.length[st.edge]))
    # on a vertex: edge drawn from b, particle on the chosen end
    b = np.array([0.2, 0.5, 0.3])
    g3 = workloads.from_edges(2, [0, 1, 0], [1, 0, 1], [1.0, 2.0, 3.0], weight_init=[2, 1, 3], weight_term=[1, 5, 1])
    st = orc.init(g3, 100_000, orc.INIT_AT_VERTEX, vertex=0, seed=1)
    # vertex 0: slots (e0 init, w=2), (e1 term, w=5), (e2 init, w=3)
    cnt = np.bincount(st.edge, minlength=3) / 100_000
    assert np.all(np.abs(cnt - b) < 5 * np.sqrt(b * (1 - b) / 100_000))
    assert np.all(st.x[st.edge == 1] == 2.0) and np.all(st.x[st.edge != 1] == 0.0)
