"""Pins of the oracle's streamed (time-summed) histogram and of the
empirical L2 density error (Sec. 4.1's accuracy measurement), against what
the mathematics fixes."""
import numpy as np
import pytest
from scipy import stats

import closed_forms as cf
import workloads


def test_streamed_histogram_snapshot_times_closed_form(orc):
    """No-hit moves with constant coefficients are exact Gaussians at any dt,
    so the expected sum of snapshots at step counts every, 2 every, ... is
    N sum_j P(N(x0 + a t_j, sigma^2 t_j) in bin).  The drift moves the mean by
    a dt every step, so a snapshot taken one step early or late (or a missing
    or extra snapshot) fails the chi-square test."""
    a, sig, dt, every, steps = 3.0, 0.4, 0.5, 2, 8
    L, bins = 100.0, 100
    g = workloads.segment(L, a, 0.0, sig)
    N = 40_000
    st = orc.init(g, N, orc.INIT_EXPLICIT, edge=np.zeros(N), pos=np.full(N, 40.0))
    acc, snaps, c = orc.observed_histogram(g, st, 0, steps, dt, 5, every, bins)
    assert snaps == steps // every and c.hits == 0
    edges = np.linspace(0.0, L, bins + 1)
    exp = np.zeros(bins)
    for j in range(1, snaps + 1):
        t = j * every * dt
        exp += np.diff(stats.norm.cdf(edges, 40.0 + a * t, sig * np.sqrt(t)))
    exp *= N
    obs = acc[0].astype(np.float64)
    assert obs.sum() == N * snaps
    m = exp > 5
    chi = ((obs[m] - exp[m]) ** 2 / exp[m]).sum()
    # snapshots are correlated through the shared paths; the per-bin
    # variance is at most snaps times the multinomial one
    assert chi / snaps < stats.chi2.ppf(0.999, m.sum()), chi


def test_streamed_histogram_offsets_and_conservation(orc):
    """Snapshots follow the step counter, not the call: a run that starts at
    an offset counter and is cut anywhere takes the snapshots at the
    multiples of `every` only; without absorption each snapshot holds every
    particle."""
    g, run = workloads.config1()
    N = 3000
    st = orc.init(g, N, orc.INIT_AT_VERTEX, vertex=0, seed=1)
    acc, snaps, _ = orc.observed_histogram(g, st, 7, 100, 1e-3, 2, 10, 20)
    assert snaps == 10  # counters 10, 20, ..., 100 lie in (7, 107]
    assert int(acc.sum()) == N * snaps
    st2 = orc.init(g, N, orc.INIT_AT_VERTEX, vertex=0, seed=1)
    a1, s1, _ = orc.observed_histogram(g, st2, 7, 38, 1e-3, 2, 10, 20)
    a2, s2, _ = orc.observed_histogram(g, st2, 45, 62, 1e-3, 2, 10, 20)
    assert s1 + s2 == snaps and np.array_equal(a1 + a2, acc)
    assert np.array_equal(st2.x, st.x)


def test_density_l2_hand_example(orc):
    """One edge of length 2, two bins (width 1): counts (3, 1) estimate the
    density (0.75, 0.25); against the uniform 0.5 the distance is
    sqrt(1 * 0.25^2 + 1 * 0.25^2)."""
    assert orc.density_l2([2.0], 2, [3, 1], [0.5, 0.5]) == pytest.approx(np.sqrt(0.125),
                                                                         rel=1e-15)
    # with an explicit mass of 8 the estimate is (0.375, 0.125)
    v = np.sqrt((0.375 - 0.5) ** 2 + (0.125 - 0.5) ** 2)
    assert orc.density_l2([2.0], 2, [3, 1], [0.5, 0.5], mass=8) == pytest.approx(v,
                                                                                 rel=1e-15)


def test_density_l2_zero_on_exact_counts_and_bin_widths(orc):
    """Counts exactly proportional to the reference mass of each bin give 0,
    on edges of different lengths (the bin width enters the estimate)."""
    L = np.array([1.0, 4.0, 0.5])
    bins = 4
    rng = np.random.default_rng(0)
    mass = rng.integers(1, 50, size=(3, bins)).astype(np.float64)
    tot = mass.sum()
    ref = mass / tot / (L / bins)[:, None]
    assert orc.density_l2(L, bins, mass.astype(np.uint64), ref) == pytest.approx(0.0,
                                                                                abs=1e-14)


def test_density_l2_multinomial_floor(orc):
    """For N samples from bin masses p_k the expected squared distance is
    sum_k p_k (1 - p_k) / (N w_k): the Monte-Carlo floor of the error
    measure, checked by averaging over repeated multinomial draws."""
    L = np.array([2.0, 1.0])
    bins = 5
    rng = np.random.default_rng(1)
    p = rng.dirichlet(np.ones(L.size * bins))
    w = np.repeat(L / bins, bins)
    ref = p / w
    N, reps = 2000, 4000
    sq = [orc.density_l2(L, bins, rng.multinomial(N, p), ref, mass=N) ** 2
          for _ in range(reps)]
    expect = float(np.sum(p * (1 - p) / (N * w)))
    se = np.std(sq) / np.sqrt(reps)
    assert abs(np.mean(sq) - expect) < 4 * se, (np.mean(sq), expect, se)


@pytest.mark.parametrize("which", ["linear", "quadratic", "config2", "flat"])
def test_stationary_bin_means_match_quadrature(which):
    """The closed-form bin averages the density-error measurement compares
    against: total mass one, and agreement with a fine trapezoid quadrature of
    pi_e(x) = C b_e / D exp(-(V_e(x) - V_e(0)) / D) on every bin."""
    from workloads import stationary
    if which in ("linear", "quadratic"):
        g = workloads.paper_star5(which)
    elif which == "config2":
        g = workloads.config2()[0]
    else:
        g = workloads.star_graph(3, [1.0, 2.0, 0.5], b_center=[0.2, 0.5, 0.3])
    bins = 16
    ref = stationary.star_bin_means(g, bins)
    w = np.asarray(g.length)[:, None] / bins
    assert (ref * w).sum() == pytest.approx(1.0, abs=1e-12)
    D = 0.5 * float(g.sigma[0]) ** 2
    b = np.zeros(g.n_edges)
    b[g.slot_edge[: g.vtx_offsets[1]]] = g.slot_jump_prob[: g.vtx_offsets[1]]
    Vs = [lambda x, a=float(g.drift_a[e]), c=float(g.drift_c[e]): -a * x - 0.5 * c * x * x
          for e in range(g.n_edges)]
    masses, xs, ds = cf.star_stationary(g.length, Vs, b, g.sigma[0], grid=400_001)
    quad = np.array([cf.binned(xs[e], ds[e], np.linspace(0, g.length[e], bins + 1))
                     for e in range(g.n_edges)]) / w
    np.testing.assert_allclose(ref, quad, rtol=1e-6, atol=1e-9 * ref.max())


def test_histogram_csr_hand_example(orc):
    """Uneven bins on two edges: upper boundaries (0.1, 0.5, 2.0) on edge 0
    and (1.0,) on edge 1; a particle on a boundary goes to the bin below it,
    the edge's ends to its first and last bins, dead particles nowhere."""
    g = workloads.from_edges(3, [0, 0], [1, 2], [2.0, 1.0], sigma=1.0)
    st = orc.init(g, 7, orc.INIT_EXPLICIT, edge=np.array([0, 0, 0, 0, 0, 1, 1]),
                  pos=np.array([0.0, 0.1, 0.3, 0.5, 2.0, 0.0, 1.0]))
    st.alive[6] = 0
    h = orc.histogram_csr(g, st, [0, 3, 4], [0.1, 0.5, 2.0, 1.0])
    assert h.tolist() == [2, 2, 1, 1]


def test_histogram_csr_matches_uniform_and_search(orc):
    """With uniform bins it is the uniform histogram (positions off the
    interior boundaries), and in general a binary search for the first
    upper boundary >= x."""
    g, _ = workloads.config2()
    st = orc.init(g, 20_000, orc.INIT_UNIFORM_LENGTH, seed=3)
    nb = 16
    off = np.arange(g.n_edges + 1) * nb
    up = np.concatenate([np.arange(1, nb + 1) * (L / nb) for L in g.length])
    assert np.array_equal(orc.histogram_csr(g, st, off, up), orc.histogram(g, st, nb).ravel())
    rng = np.random.default_rng(4)
    counts = rng.integers(1, 9, size=g.n_edges)
    off = np.concatenate([[0], np.cumsum(counts)])
    up = np.concatenate([np.sort(rng.uniform(0, L, c - 1)).tolist() + [L]
                         for L, c in zip(g.length, counts)])
    h = orc.histogram_csr(g, st, off, up)
    want = np.zeros(off[-1], np.uint64)
    for e, x in zip(st.edge, st.x):
        k = np.searchsorted(up[off[e]:off[e + 1]], x, side="left")
        want[off[e] + min(k, counts[e] - 1)] += 1
    assert np.array_equal(h, want) and int(h.sum()) == st.pid.size
