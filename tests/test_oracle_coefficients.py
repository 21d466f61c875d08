"""Pins of the oracle's general coefficient functions (Sec. 2.2 allows any
C^1 drift and diffusion; the scheme freezes both at each sub-step's start,
Alg. 2): cubic drift mu_e(x) and cubic diffusion sigma_e(x)."""
import numpy as np
import pytest
from scipy import integrate, stats

import workloads

# mu(x) = -V'(x) for V = 4 ((x - 0.5)(x - 1.5))^2, wells at 0.5 and 1.5
MU = (12.0, -44.0, 48.0, -16.0)
# sigma(x) = 1 + 0.3 x - 0.1 x^2 + 0.02 x^3 (>= 1 on [0, 2])
SIG = (1.0, 0.3, -0.1, 0.02)
TV_TOL = 0.02


def _power(coef, x):
    """sum_j coef[j] x^j written out as powers (not Horner's rule)."""
    return sum(c * x ** j for j, c in enumerate(coef))


def _segment(L, mu, sig, end_kind=0):
    g = workloads.segment(L, mu[0], mu[1], sig[0], end_kind=end_kind)
    g.drift_c2, g.drift_c3 = [mu[2]], [mu[3]]
    g.sigma_c1, g.sigma_c2, g.sigma_c3 = [sig[1]], [sig[2]], [sig[3]]
    return g


@pytest.mark.parametrize("x0", [2.0, 5.0])
def test_one_step_gaussian_with_frozen_coefficients(orc, x0):
    """Far from the vertices one step is x0 + mu(x0) dt + sigma(x0) sqrt(dt)
    Z exactly: KS against that normal law, with mu and sigma summed as plain
    powers.  Every term moves the law by several KS critical values."""
    mu = (0.3, -0.5, 0.2, -0.05)
    sig = (1.0, 0.1, 0.05, -0.004)
    g = _segment(100.0, mu, sig)
    N, dt = 200_000, 0.05
    st = orc.init(g, N, orc.INIT_EXPLICIT, edge=np.zeros(N), pos=np.full(N, x0))
    c = orc.simulate(g, st, 0, 1, dt, 3)
    assert c.hits == 0
    m = x0 + _power(mu, x0) * dt
    s = _power(sig, x0) * np.sqrt(dt)
    ks = stats.kstest(st.x, stats.norm(m, s).cdf)
    assert ks.pvalue > 1e-4, ks
    # the pinned moments, as a sharper check of the same law
    assert abs(st.x.mean() - m) < 5 * s / np.sqrt(N)
    assert abs(st.x.std() / s - 1.0) < 5 / np.sqrt(2 * N)


@pytest.mark.parametrize("end_kind", [0, 2])
def test_stationary_law_with_cubic_drift_and_diffusion(orc, end_kind):
    """A segment [0, 2] with reflecting ends (plain leaves, or mirror
    vertices), double-well drift and a cubic diffusion: the Ito diffusion's
    stationary density is exp(int_0^x 2 mu / sigma^2) / sigma^2 (zero flux),
    integrated here by quadrature.  Started from that law, time-averaged bin
    masses stay within the Monte-Carlo and time-step error (total
    variation)."""
    L, nb = 2.0, 40
    g = _segment(L, MU, SIG, end_kind)

    def dens(x):
        phi = integrate.quad(lambda y: 2 * _power(MU, y) / _power(SIG, y) ** 2, 0, x)[0]
        return np.exp(phi) / _power(SIG, x) ** 2
    edges = np.linspace(0, L, nb + 1)
    mass = np.array([integrate.quad(dens, a, b)[0] for a, b in zip(edges[:-1], edges[1:])])
    mass /= mass.sum()
    # initial positions drawn from that law (inverse CDF on a fine grid)
    grid = np.linspace(0, L, 4001)
    pdf = np.array([dens(x) for x in grid])
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (pdf[1:] + pdf[:-1]) * np.diff(grid))])
    cdf /= cdf[-1]
    N = 20_000
    u = np.random.default_rng(4).uniform(size=N)
    x0 = np.interp(u, cdf, grid)
    st = orc.init(g, N, orc.INIT_EXPLICIT, edge=np.zeros(N), pos=x0)
    dt, n0 = 1e-3, 0
    acc = np.zeros(nb)
    for _ in range(6):
        orc.simulate(g, st, n0, 300, dt, 8)
        n0 += 300
        acc += orc.histogram(g, st, nb).astype(np.float64).ravel()
    emp = acc / acc.sum()
    tv = 0.5 * np.abs(emp - mass).sum()
    # (dropping sigma's linear term moves the law by TV 0.14, a constant
    # sigma by 0.066; the cubic terms are pinned by the one-step law)
    assert tv < TV_TOL, tv


def test_zero_higher_terms_are_the_affine_step(orc):
    """Explicit zero higher terms give bit for bit the run without them
    (the cubics collapse to fma(c, x, a) and sigma)."""
    g0 = workloads.star_graph(3, [1.0, 2.0, 0.5], [0.5, -1.0, 0.0], [-2.0, 0.3, 1.0], 1.2)
    g1 = workloads.star_graph(3, [1.0, 2.0, 0.5], [0.5, -1.0, 0.0], [-2.0, 0.3, 1.0], 1.2)
    z = np.zeros(3)
    g1.drift_c2 = g1.drift_c3 = g1.sigma_c1 = g1.sigma_c2 = g1.sigma_c3 = z
    out = []
    for g in (g0, g1):
        st = orc.init(g, 5000, orc.INIT_UNIFORM_LENGTH, seed=1)
        orc.simulate(g, st, 0, 300, 1e-2, 2)
        out.append(st)
    assert np.array_equal(out[0].x, out[1].x)
    assert np.array_equal(out[0].seqhash, out[1].seqhash)


# ------------------------------------------------ tabulated coefficients --

def _table_of(g, knots, mu, sig):
    """Tables of the cubics mu and sig (coefficients a0..a3) at the knots:
    values and derivatives."""
    d = lambda c: (c[1], 2 * c[2], 3 * c[3], 0.0)
    return workloads.tabulate(g, knots,
                              lambda e, x: _power(mu, x), lambda e, x: _power(d(mu), x),
                              lambda e, x: _power(sig, x), lambda e, x: _power(d(sig), x))


@pytest.mark.parametrize("knots", [1, 3, 8])
def test_table_of_a_cubic_is_the_cubic(orc, knots):
    """Cubic Hermite interpolation reproduces a cubic exactly, so a table of
    the double-well drift and the cubic diffusion (values and derivatives at
    1, 3 or 8 intervals) runs the same paths as the cubic coefficients, up
    to rounding: the same hit sequences, positions within 1e-9 after 600
    steps on a reflecting segment.  A wrong interval, a wrong local
    coordinate or a derivative not scaled by the interval width breaks the
    exactness by far more."""
    L = 2.0
    g_cubic = _segment(L, MU, SIG)
    g_tab = _table_of(_segment(L, (0.0,) * 4, (1.0, 0.0, 0.0, 0.0)), knots, MU, SIG)
    out = []
    for g in (g_cubic, g_tab):
        st = orc.init(g, 20_000, orc.INIT_UNIFORM_LENGTH, seed=5)
        orc.simulate(g, st, 0, 600, 1e-3, 6)
        out.append(st)
    a, b = out
    assert (a.seqhash == b.seqhash).mean() >= 0.999
    same = a.seqhash == b.seqhash
    assert np.abs(a.x[same] - b.x[same]).max() < 1e-9


def test_table_stationary_law_of_non_polynomial_coefficients(orc):
    """A segment [0, 1.5] with reflecting ends, drift -V' of the periodic
    potential V = 1.2 (1 - cos(4 pi x / L)) and diffusion 1 + 0.4 sin(pi x /
    L), tabulated at 16 intervals: the time-averaged bin masses match the
    stationary density exp(int 2 mu / sigma^2) / sigma^2 of the exact
    functions (the interpolation error at 16 intervals is below 1e-5)
    within TV 0.02; a constant sigma would be off by more."""
    L, nb = 1.5, 30
    w = 4 * np.pi / L
    mu = lambda x: -1.2 * w * np.sin(w * x)
    dmu = lambda x: -1.2 * w * w * np.cos(w * x)
    sig = lambda x: 1.0 + 0.4 * np.sin(np.pi * x / L)
    dsig = lambda x: 0.4 * (np.pi / L) * np.cos(np.pi * x / L)
    g = workloads.tabulate(workloads.segment(L, 0.0, 0.0, 1.0), 16,
                           lambda e, x: mu(x), lambda e, x: dmu(x),
                           lambda e, x: sig(x), lambda e, x: dsig(x))

    def dens(x, s=sig):
        phi = integrate.quad(lambda y: 2 * mu(y) / s(y) ** 2, 0, x)[0]
        return np.exp(phi) / s(x) ** 2
    edges = np.linspace(0, L, nb + 1)

    def masses(s):
        m = np.array([integrate.quad(lambda x: dens(x, s), a, b)[0]
                      for a, b in zip(edges[:-1], edges[1:])])
        return m / m.sum()
    mass = masses(sig)
    grid = np.linspace(0, L, 4001)
    pdf = np.array([dens(x) for x in grid])
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (pdf[1:] + pdf[:-1]) * np.diff(grid))])
    cdf /= cdf[-1]
    N = 20_000
    x0 = np.interp(np.random.default_rng(7).uniform(size=N), cdf, grid)
    st = orc.init(g, N, orc.INIT_EXPLICIT, edge=np.zeros(N), pos=x0)
    n0, acc = 0, np.zeros(nb)
    for _ in range(6):
        orc.simulate(g, st, n0, 300, 1e-3, 9)
        n0 += 300
        acc += orc.histogram(g, st, nb).astype(np.float64).ravel()
    emp = acc / acc.sum()
    tv = 0.5 * np.abs(emp - mass).sum()
    assert tv < TV_TOL, tv
    # the diffusion's shape matters at this tolerance
    flat = masses(lambda x: 1.0 + 0.0 * x)
    assert 0.5 * np.abs(flat - mass).sum() > 2 * TV_TOL
