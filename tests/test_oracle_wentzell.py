"""Pins of the oracle's Wentzell vertices (partial killing a_v, stickiness c_v).

Sec. 2.2 gives the general gluing condition a_v f(v) - sum_e b_ve f'_e(v) +
c_v (L f)(v) = 0 with a_v + sum_e b_ve + c_v = 1, but no scheme for it.  The
oracle's per-visit rule (killing with probability 1 - exp(-kappa l) and a
stay of gamma l on the vertex, l the visit's local time) is checked here
against closed forms of the continuous process that do not depend on the
scheme: the Robin-boundary survival on a segment (eigen-expansion), the
killed and sticky laws on a half-line from the vertex (excursion theory),
and the stationary atom of a sticky star.  Bars: 4 Monte-Carlo standard
errors plus an allowance for the scheme's error next to a vertex, which
falls like sqrt(dt) (measured: about 0.4 sqrt(dt) on the sticky atom, below
0.1 sqrt(dt) on killing alone); an error in kappa, gamma or sigma_v by a
factor moves these laws by far more.  A Wentzell vertex with a_v = c_v = 0
is a standard vertex, bit for bit.
"""
import numpy as np
import pytest

import closed_forms as cf
import workloads


def _wentzell_segment(a, c, length=1.0, sigma=1.0):
    """One edge from Wentzell vertex 0 to a standard leaf (length inf: a
    half-line, its far end a vertex at infinity)."""
    g = workloads.segment(length if np.isfinite(length) else 1.0, 0.0, 0.0, sigma)
    if not np.isfinite(length):
        g.length[:] = np.inf
        g.bin_span = np.array([4.0])
    g.vtx_kind[0] = 3
    g.slot_jump_prob[g.vtx_offsets[0]] = 1.0 - a - c
    g.vtx_kill = np.array([a, 0.0])
    g.vtx_sticky = np.array([c, 0.0])
    return g


def _se(p, n):
    return np.sqrt(max(p * (1 - p), 1e-12) / n)


def test_robin_segment_survival(orc):
    """Killing only (a = 0.6, b = 0.4: kappa = 1.5), uniform start on [0, 1],
    reflecting far end: survival at t = 0.5 against the eigen-expansion of
    u_t = u_xx / 2 with u_x(0) = kappa u(0)."""
    n, dt, T = 100_000, 1e-3, 0.5
    g = _wentzell_segment(0.6, 0.0)
    st = orc.init(g, n, orc.INIT_UNIFORM_LENGTH, seed=1)
    orc.simulate(g, st, 0, int(round(T / dt)), dt, 3)
    exact = cf.robin_segment_survival(T, 1.0, 1.0, 1.5)
    got = st.alive.mean()
    assert abs(got - exact) <= 4 * _se(exact, n) + 0.1 * np.sqrt(dt), (got, exact)


def test_killing_halfline_from_vertex(orc):
    """Killing only on a half-line (sigma = sqrt 2, kappa = 0.3 / 0.7), start
    on the vertex: P(alive at 1) = erfcx(kappa sigma sqrt(t / 2))."""
    n, dt, T = 100_000, 1e-3, 1.0
    sig = np.sqrt(2.0)
    g = _wentzell_segment(0.3, 0.0, np.inf, sig)
    st = orc.init(g, n, orc.INIT_AT_VERTEX, vertex=0, seed=2)
    orc.simulate(g, st, 0, int(round(T / dt)), dt, 4)
    exact = cf.killing_halfline_alive(T, sig, 0.3 / 0.7)
    got = st.alive.mean()
    assert abs(got - exact) <= 4 * _se(exact, n) + 0.1 * np.sqrt(dt), (got, exact)


@pytest.mark.parametrize("a,c,sig", [(0.0, 0.5, 1.0), (0.2, 0.5, np.sqrt(2.0))])
def test_sticky_halfline_from_vertex(orc, a, c, sig):
    """Sticky (and killing) vertex on a half-line, start on it: P(on v and
    alive at t = 1) and P(alive at 1) against the inverse Laplace transforms
    of the excursion-theory resolvent.  A particle owing a stay sits on v."""
    n, dt, T = 100_000, 1e-3, 1.0
    g = _wentzell_segment(a, c, np.inf, sig)
    beta = 1.0 - a - c
    gam, kap = c / beta, a / beta
    st = orc.init(g, n, orc.INIT_AT_VERTEX, vertex=0, seed=5)
    orc.simulate(g, st, 0, int(round(T / dt)), dt, 7)
    on_v = ((st.x <= 0.0) & (st.alive == 1)).mean()
    ex_v = cf.sticky_halfline_at_vertex(T, sig, gam, kap)
    assert abs(on_v - ex_v) <= 4 * _se(ex_v, n) + 0.6 * np.sqrt(dt), (on_v, ex_v)
    ex_a = cf.sticky_halfline_alive(T, sig, gam, kap)
    alive = st.alive.mean()
    assert abs(alive - ex_a) <= 4 * _se(ex_a, n) + 0.3 * np.sqrt(dt), (alive, ex_a)


def test_sticky_star_stationary_atom(orc):
    """Three-edge star (lengths 0.5, 1, 1.5), sticky centre c = 0.25 with
    b-hat = (0.2, 0.3, 0.5), reflecting leaves, sigma = 1: after six
    relaxation times from the uniform law, the atom on the centre and the
    edge masses equal the stationary law (density C b_e / D on edge e, atom
    gamma C)."""
    n, dt, T = 40_000, 1e-3, 6.0
    b_hat = np.array([0.2, 0.3, 0.5])
    c = 0.25
    g = workloads.star_graph(3, [0.5, 1.0, 1.5], None, None, 1.0, b_center=b_hat)
    s0, s1 = g.vtx_offsets[0], g.vtx_offsets[1]
    g.slot_jump_prob[s0:s1] = (1.0 - c) * b_hat
    g.vtx_kind[0] = 3
    g.vtx_kill = np.zeros(4)
    g.vtx_sticky = np.array([c, 0.0, 0.0, 0.0])
    st = orc.init(g, n, orc.INIT_UNIFORM_LENGTH, seed=8)
    orc.simulate(g, st, 0, int(round(T / dt)), dt, 9)
    atom, masses = cf.sticky_star_stationary([0.5, 1.0, 1.5], b_hat, 1.0, c / (1.0 - c))
    on_v = (st.x <= 0.0).mean()
    tol = lambda p: 4 * _se(p, n) + 0.6 * np.sqrt(dt)
    assert abs(on_v - atom) <= tol(atom), (on_v, atom)
    for e in range(3):
        m = ((st.edge == e) & (st.x > 0.0)).mean()
        assert abs(m - masses[e]) <= tol(masses[e]), (e, m, masses[e])


def test_zero_wentzell_is_standard(orc):
    """a_v = c_v = 0 is the standard gluing condition: a Wentzell vertex with
    both zero gives the standard vertex's paths bit for bit (its vertex-stream
    draws change nothing)."""
    g0 = workloads.config2()[0]
    g1 = workloads.config2()[0]
    g1.vtx_kind[0] = 3
    g1.vtx_kill = np.zeros(g1.n_vertices)
    g1.vtx_sticky = np.zeros(g1.n_vertices)
    out = []
    for g in (g0, g1):
        st = orc.init(g, 3000, orc.INIT_UNIFORM_LENGTH, seed=3)
        c = orc.simulate(g, st, 0, 300, 1e-2, 11)
        out.append((st, c))
    (a, ca), (b, cb) = out
    assert np.array_equal(a.seqhash, b.seqhash) and np.array_equal(a.x, b.x)
    assert np.array_equal(ca.exit_slot, cb.exit_slot)
    assert ca.substeps == cb.substeps and ca.hits == cb.hits
