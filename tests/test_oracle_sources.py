"""Pins of the oracle's injection at source vertices (the inlets of the
tracer problem, Sec. 4.2) and of the steady state that a pulse's streamed
histogram gives, against what the mathematics fixes."""
import numpy as np
import pytest
from scipy import stats

import workloads


def test_sources_law(orc):
    """Sources are drawn in proportion to their rates (zero rate: never),
    the edge from the vertex's b, and the particle sits on the vertex."""
    g = workloads.star_graph(4, [1.0, 2.0, 0.5, 1.5], b_center=[0.1, 0.2, 0.3, 0.4])
    verts = np.array([0, 2, 3, 4])          # centre and three leaves
    rates = np.array([3.0, 1.0, 0.0, 2.0])
    n = 60_000
    st = orc.init_sources(g, n, verts, rates, seed=11)
    at_centre = st.x == 0.0
    # a leaf source puts the particle at the far end of its own edge
    leaf_of_edge = {1: 2, 2: 3, 3: 4}
    src = np.where(at_centre, 0, [leaf_of_edge.get(int(e), -1) for e in st.edge])
    assert not np.any(src == 3), "a zero-rate source was drawn"
    cnt = np.array([(src == v).sum() for v in (0, 2, 4)])
    p = np.array([3.0, 1.0, 2.0]) / 6.0
    chi = ((cnt - n * p) ** 2 / (n * p)).sum()
    assert stats.chi2.sf(chi, 2) > 1e-4, cnt
    # from the centre the edge follows b
    ce = np.bincount(st.edge[at_centre], minlength=4)
    b = np.array([0.1, 0.2, 0.3, 0.4])
    chi = ((ce - ce.sum() * b) ** 2 / (ce.sum() * b)).sum()
    assert stats.chi2.sf(chi, 3) > 1e-4, ce
    L = np.asarray(g.length)
    assert np.all(st.x[~at_centre] == L[st.edge[~at_centre]])


def test_sources_reject_bad_input(orc):
    g = workloads.star_graph(3, 1.0)
    with pytest.raises(ValueError):
        orc.init_sources(g, 10, [0, 1], [0.0, 0.0])
    with pytest.raises(ValueError):
        orc.init_sources(g, 10, [7], [1.0])


def test_pulse_occupation_is_steady_state(orc):
    """Drift-diffusion on [0, L] (velocity u > 0, D = sigma^2/2) injected at
    the reflecting end and absorbed at the other: a steady injection of rate
    r has the constant flux u c - D c' = r and c(L) = 0, so
    c(x) = (r/u)(1 - exp(-u (L - x) / D)).  A unit pulse's occupation density
    (the time-summed histogram times the snapshot interval, per particle)
    must match c/r bin by bin, and its total is the mean absorption time.
    Away from the absorbing end the match is within a few per cent; next to
    it the discrete scheme, which sees a crossing only at a sub-step's end,
    keeps particles a little longer (the usual O(sqrt(dt)) layer of killed
    diffusions), so the last bin gets only an absolute bound."""
    L, u, sig, dt, every = 1.0, 2.0, 1.0, 5e-4, 4
    D = 0.5 * sig * sig
    g = workloads.segment(L, u, 0.0, sig)
    g.vtx_kind[1] = 1
    n, steps, bins = 20_000, 8_000, 10
    st = orc.init_sources(g, n, [0], [1.0], seed=2)
    acc, snaps, c = orc.observed_histogram(g, st, 0, steps, dt, 3, every, bins)
    assert int(st.alive.sum()) < n * 1e-3      # (almost) all absorbed
    occ = acc[0] * (every * dt) / n
    edges = np.linspace(0.0, L, bins + 1)
    prim = lambda x: x / u - (D / u ** 2) * np.exp(-u * (L - x) / D)
    want = np.diff(prim(edges))
    tau = L / u - (D / u ** 2) * (1 - np.exp(-u * L / D))
    assert occ.sum() == pytest.approx(tau, rel=0.04)
    np.testing.assert_allclose(occ[:8], want[:8], rtol=0.05)
    np.testing.assert_allclose(occ, want, rtol=0, atol=0.004)
