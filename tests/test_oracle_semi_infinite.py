"""Pins of the oracle on semi-infinite edges (Def. 1 allows l_e = inf; the
paper's star metric graphs, Def. 3, have only such edges) against what the
paper and the mathematics fix."""
import numpy as np
import pytest
from scipy import special, stats

import workloads
from workloads import stationary


def _paper_quadratic_masses(off, true_up, D):
    """Bin masses of the quadratic-potential steady state in the paper's own
    closed form (Sec. 4.1 and its appendix of normalisers): on edge i,
    B exp(-(10 i) x^2 / (2D)) on [0, inf) with B = sqrt(2/(D pi)) /
    sum_i 1/sqrt(10 i), written out here from those formulas."""
    i = np.arange(1, 6, dtype=np.float64)
    B = np.sqrt(2.0 / (D * np.pi)) / np.sum(1.0 / np.sqrt(10.0 * i))
    out = []
    for e in range(5):
        a = 10.0 * (e + 1) / (2.0 * D)
        edges = np.concatenate([[0.0], true_up[off[e]:off[e + 1]]])
        out.append(B * np.diff(0.5 * np.sqrt(np.pi / a) * special.erf(np.sqrt(a) * edges)))
    return np.concatenate(out)


def test_closed_form_module_matches_the_paper_quadratic_star():
    """The stationary module's bin masses on the paper's semi-infinite
    quadratic star equal the paper's printed closed form."""
    g = workloads.paper_star5("quadratic", length=np.inf)
    off, up, tu = workloads.csr_bins(g, 0.05, 12)
    m = stationary.star_csr_masses(g, off, tu)
    p = _paper_quadratic_masses(off, tu, 0.5)
    assert abs(p.sum() - 1.0) < 1e-14
    np.testing.assert_allclose(m, p, rtol=1e-12, atol=1e-15)


def test_semi_infinite_star_stationary_law(orc):
    """The oracle on the paper's semi-infinite quadratic star reaches the
    paper's Gaussian steady state: time-averaged bin masses within the
    Monte-Carlo and time-step error of the closed form (total variation),
    and every leg's mass within 4 standard errors of B sqrt(pi D / (20 i))."""
    g = workloads.paper_star5("quadratic", length=np.inf)
    off, up, tu = workloads.csr_bins(g, 0.05, 12)
    exact = _paper_quadratic_masses(off, tu, 0.5)
    N, dt = 20_000, 1e-3
    st = orc.init(g, N, orc.INIT_AT_VERTEX, vertex=0, seed=3)
    c = orc.simulate(g, st, 0, 1000, dt, 11)
    acc = np.zeros(off[-1])
    n0, snaps = 1000, 6
    for _ in range(snaps):
        orc.simulate(g, st, n0, 200, dt, 11, counts=c)
        n0 += 200
        acc += orc.histogram_csr(g, st, off, up).astype(np.float64)
    emp = acc / acc.sum()
    tv = 0.5 * np.abs(emp - exact).sum()
    assert tv < 0.02, tv
    # nothing reaches the vertices at infinity; positions stay finite
    assert np.all(np.isfinite(st.x)) and np.all(st.x >= 0.0)
    far = [s for s in range(g.nnz) if g.slot_orient[s] == 1]
    assert c.exit_slot[far].sum() == 0
    legs_emp = np.array([emp[off[e]:off[e + 1]].sum() for e in range(5)])
    legs = np.array([exact[off[e]:off[e + 1]].sum() for e in range(5)])
    se = np.sqrt(legs * (1 - legs) / (N * snaps / 2))  # snapshots half-correlated at most
    assert np.all(np.abs(legs_emp - legs) < 4 * se + 2e-3), (legs_emp, legs)


def test_far_start_moves_as_plain_euler_maruyama(orc):
    """A particle far out on a semi-infinite edge with constant drift never
    reaches the vertex within a short run: its moves are plain EM increments,
    so its mean and variance over many particles follow x0 + a t and
    sigma^2 t exactly (normal law, any dt)."""
    g = workloads.from_edges(2, [0], [1], [np.inf], [1.5], [0.0], 0.8, bin_span=100.0)
    N, dt, steps, x0 = 40_000, 0.01, 50, 40.0
    st = orc.init(g, N, orc.INIT_EXPLICIT, edge=np.zeros(N), pos=np.full(N, x0))
    c = orc.simulate(g, st, 0, steps, dt, 7)
    assert c.hits == 0
    t = steps * dt
    z = (st.x - (x0 + 1.5 * t)) / (0.8 * np.sqrt(t))
    assert abs(z.mean()) < 4 / np.sqrt(N)
    assert abs(z.var() - 1.0) < 4 * np.sqrt(2.0 / N)
    assert stats.kstest(z, "norm").pvalue > 1e-4


def test_uniform_init_needs_finite_edges_and_bins_a_span(orc):
    """Uniform-by-length init is undefined with an infinite edge; uniform
    bins cover the edge's bin span, the last bin taking everything beyond,
    and a semi-infinite edge must have a span."""
    g = workloads.paper_star5("linear", length=np.inf, bin_span=2.0)
    with pytest.raises(ValueError):
        orc.init(g, 10, orc.INIT_UNIFORM_LENGTH)
    st = orc.init(g, 4, orc.INIT_EXPLICIT, edge=[0, 0, 1, 4], pos=[0.0, 1.99, 2.0, 1e9])
    h = orc.histogram(g, st, 8)
    assert h[0, 0] == 1 and h[0, 7] == 1 and h[1, 7] == 1 and h[4, 7] == 1
    assert h.sum() == 4
    g.bin_span = None
    with pytest.raises(ValueError):
        orc.init(g, 10, orc.INIT_AT_VERTEX, vertex=0)
