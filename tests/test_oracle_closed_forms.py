"""The oracle against what the mathematics fixes (no second implementation of
the scheme is used anywhere here).

Each test states its Monte-Carlo floor; tolerances are a few standard errors
plus, where the scheme has a discretisation bias, an allowance that the test
also shows shrinking with dt.
"""
import numpy as np
import pytest
from scipy import stats

import closed_forms as cf
import workloads


def _chi2_pvalue(counts, probs):
    counts = np.asarray(counts, np.float64)
    exp = probs * counts.sum()
    return stats.chi2.sf(((counts - exp) ** 2 / exp).sum(), counts.size - 1)


# ------------------------------------------------------------ no-hit moves

def test_constant_drift_move_is_exact_gaussian(orc):
    """Away from vertices EM with constant coefficients is exact in law:
    x_T ~ N(x0 + a T, sigma^2 T) at any dt (the EM update, Sec. 3)."""
    a, sig, dt, n = 0.7, 1.3, 0.01, 100
    g = workloads.segment(100.0, a, 0.0, sig)
    N = 200_000
    st = orc.init(g, N, orc.INIT_EXPLICIT, edge=np.zeros(N), pos=np.full(N, 50.0))
    c = orc.simulate(g, st, 0, n, dt, 21)
    assert c.hits == 0 and c.substeps == N * n
    T = n * dt
    z = (st.x - (50.0 + a * T)) / (sig * np.sqrt(T))
    assert stats.kstest(z, "norm").pvalue > 1e-3


def test_linear_drift_ar1_law(orc):
    """With mu(x) = a + c x the EM chain is the Gaussian AR(1)
    x' = (1 + c h) x + a h + sigma sqrt(h) W: mean and variance follow
    m' = (1 + c h) m + a h, v' = (1 + c h)^2 v + sigma^2 h."""
    a, c, sig, h, n = 100.0, -2.0, 0.9, 0.05, 40
    g = workloads.segment(100.0, a, c, sig)
    N = 200_000
    x0 = 40.0
    st = orc.init(g, N, orc.INIT_EXPLICIT, edge=np.zeros(N), pos=np.full(N, x0))
    orc.simulate(g, st, 0, n, h, 22)
    m, v = x0, 0.0
    for _ in range(n):
        m, v = (1 + c * h) * m + a * h, (1 + c * h) ** 2 * v + sig * sig * h
    z = (st.x - m) / np.sqrt(v)
    assert stats.kstest(z, "norm").pvalue > 1e-3


# ------------------------------------------------------ star 3, config 1

def test_config1_exchangeable_masses_and_exits(orc):
    """Config 1 (3 identical edges, uniform b, started at the centre): by
    symmetry the edge occupancy and the exit slots at the centre are exactly
    uniform at any dt; no drift means no truncation."""
    g, run = workloads.config1()
    st = orc.init(g, run["n_particles"], orc.INIT_AT_VERTEX, vertex=0, seed=run["seed"])
    c = orc.simulate(g, st, 0, run["n_steps"], run["dt"], run["seed"],
                     max_splits=run["max_splits"])
    assert c.truncations == 0
    occ = np.bincount(st.edge, minlength=3)
    assert _chi2_pvalue(occ, np.full(3, 1 / 3)) > 1e-3
    centre = c.exit_slot[g.vtx_offsets[0]:g.vtx_offsets[1]]
    # exits of one particle are correlated in time, so test the mean only
    frac = centre / centre.sum()
    assert np.all(np.abs(frac - 1 / 3) < 0.02)
    hist = orc.histogram(g, st, run["bins"])
    assert hist.sum() == run["n_particles"]


def _radial_tv(orc, dt, T=0.25, N=100_000, nbins=20, seed=0):
    g = workloads.star_graph(3, 1.0, None, None, 1.0)
    st = orc.init(g, N, orc.INIT_AT_VERTEX, vertex=0, seed=seed)
    orc.simulate(g, st, 0, int(round(T / dt)), dt, seed + 1)
    edges = np.linspace(0, 1, nbins + 1)
    emp = np.histogram(st.x, edges)[0] / N
    ref = cf.reflected_segment_bin_probs(edges, 0.0, 1.0, np.sqrt(T))
    return 0.5 * np.abs(emp - ref).sum(), ref


def test_radial_reflected_heat_kernel_converges(orc):
    """From the centre of config 1's star the distance to the centre is
    Brownian motion on [0, 1] reflected at both ends (method of images).  The
    binned total-variation distance falls with dt and is at the Monte-Carlo
    floor at dt = 1e-4."""
    tvs = []
    for dt in (1e-2, 1e-3, 1e-4):
        tv, ref = _radial_tv(orc, dt)
        tvs.append(tv)
    N = 100_000
    floor = 0.5 * np.sum(np.sqrt(ref * (1 - ref) / N)) * np.sqrt(2 / np.pi)
    assert tvs[0] > tvs[2]
    assert tvs[2] < 1.5 * floor + 1e-3, (tvs, floor)


def test_path_graph_with_terminal_entries(orc):
    """Two edges meeting at their terminal ends (both entered at x = L) with
    b = (1/2, 1/2) form Brownian motion on one segment of length L0 + L1,
    reflected at both ends.  Checks the entry orientation of the CSR table."""
    L0, L1 = 0.6, 0.4
    g = workloads.from_edges(3, [0, 2], [1, 1], [L0, L1], sigma=1.0)
    N, T, dt = 100_000, 0.15, 1e-4
    st = orc.init(g, N, orc.INIT_EXPLICIT, edge=np.zeros(N), pos=np.full(N, 0.3))
    orc.simulate(g, st, 0, int(round(T / dt)), dt, 5)
    z = np.where(st.edge == 0, st.x, L0 + (L1 - st.x))
    edges = np.linspace(0, L0 + L1, 21)
    emp = np.histogram(z, edges)[0] / N
    ref = cf.reflected_segment_bin_probs(edges, 0.3, L0 + L1, np.sqrt(T))
    tv = 0.5 * np.abs(emp - ref).sum()
    floor = 0.5 * np.sum(np.sqrt(ref * (1 - ref) / N)) * np.sqrt(2 / np.pi)
    assert tv < 1.5 * floor + 1.5e-3, (tv, floor)


# ---------------------------------------------------------- stationarity

STAR4 = dict(L=np.array([1.0, 1.5, 0.8, 2.0]), k=np.array([1.0, 2.0, 3.0, 0.5]),
             m=np.array([0.3, 1.4, 0.4, 1.0]), b=np.array([0.1, 0.2, 0.3, 0.4]))


def _star4_graph():
    L, k, m, b = STAR4["L"], STAR4["k"], STAR4["m"], STAR4["b"]
    return workloads.star_graph(4, L, 2 * k * m, -2 * k, np.sqrt(2.0), b_center=b)


def _star4_stationary():
    L, k, m, b = STAR4["L"], STAR4["k"], STAR4["m"], STAR4["b"]
    pots = [lambda x, kk=kk, mm=mm: kk * (x - mm) ** 2 for kk, mm in zip(k, m)]
    return cf.star_stationary(L, pots, b, np.sqrt(2.0))


def _stationary_run(orc, dt, N=200_000, T=0.5, seed=0):
    g = _star4_graph()
    mass, xs, dens = _star4_stationary()
    rng = np.random.default_rng(seed)
    e0 = rng.choice(4, size=N, p=mass)
    x0 = np.empty(N)
    for e in range(4):
        sel = e0 == e
        x0[sel] = cf.sample_from_density(rng, xs[e], dens[e], int(sel.sum()))
    st = orc.init(g, N, orc.INIT_EXPLICIT, edge=e0, pos=x0)
    c = orc.simulate(g, st, 0, int(round(T / dt)), dt, seed + 7, max_splits=32)
    return st, c, mass, xs, dens


def test_star_quadratic_potential_stays_stationary(orc):
    """Started from the exact stationary law of a 4-edge star with quadratic
    potentials, non-uniform b and drift pushing into both ends of edges, the
    oracle keeps that law: per-edge masses and 10-bin densities per edge.
    Stationary law: pi_e(x) proportional to (b_e / D) exp(-(V_e(x) - V_e(0)) / D)."""
    st, c, mass, xs, dens = _stationary_run(orc, 1e-3)
    N = st.x.size
    occ = np.bincount(st.edge, minlength=4) / N
    assert np.all(np.abs(occ - mass) < 4 * np.sqrt(mass * (1 - mass) / N) + 1.5e-3), (occ, mass)
    tv = 0.0
    floor = 0.0
    for e in range(4):
        edges = np.linspace(0, STAR4["L"][e], 11)
        ref = cf.binned(xs[e], dens[e], edges)
        emp = np.histogram(st.x[st.edge == e], edges)[0] / N
        tv += 0.5 * np.abs(emp - ref).sum()
        floor += 0.5 * np.sum(np.sqrt(ref * (1 - ref) / N)) * np.sqrt(2 / np.pi)
    assert tv < 1.5 * floor + 2e-3, (tv, floor)


# ------------------------------------------------------------- absorbing

def test_absorbing_vertex_survival(orc):
    """Segment reflected at 0 and absorbing at 1, started at 0.5.  The alive
    fraction follows the eigenfunction series once the absorbing end is
    moved out by the continuity correction of discretely monitored Brownian
    motion, beta sigma sqrt(dt) with beta = -zeta(1/2)/sqrt(2 pi) = 0.5826
    (Broadie, Glasserman & Kou 1997); mass is conserved exactly."""
    N, T = 100_000, 0.3
    beta = 0.5826
    for dt in (1e-3, 1e-4):
        g = workloads.segment(1.0, 0.0, 0.0, 1.0)
        g.vtx_kind[1] = 1
        st = orc.init(g, N, orc.INIT_EXPLICIT, edge=np.zeros(N), pos=np.full(N, 0.5))
        c = orc.simulate(g, st, 0, int(round(T / dt)), dt, 3)
        alive = int(st.alive.sum())
        assert alive + int(c.absorbed.sum()) == N
        assert c.absorbed[0] == 0
        S = cf.survival_reflect_absorb(T, 0.5, 1.0 + beta * np.sqrt(dt), 1.0)
        se = np.sqrt(S * (1 - S) / N)
        assert abs(alive / N - S) < 4 * se + 1e-3, (dt, alive / N, S)
    # and the uncorrected limit is approached from above
    assert alive / N > cf.survival_reflect_absorb(T, 0.5, 1.0, 1.0)


# ------------------------------------------------------ exit law at vertex

EXIT = dict(b=[0.5, 0.3, 0.2], c=[10.0, 20.0, 30.0], sigma=np.sqrt(2.0))


def _exit_run(orc, dt, N, M=64, seed=1):
    g = workloads.star_graph(3, 10.0, -np.array(EXIT["c"]), None, EXIT["sigma"],
                             b_center=EXIT["b"])
    st = orc.init(g, N, orc.INIT_AT_VERTEX, vertex=0, seed=seed)
    c = orc.simulate(g, st, 0, 1, dt, seed + 4, max_splits=M)
    return g, st, c


def test_first_vertex_substep_closed_form(orc):
    """P(no hit in the first sub-step from the vertex) =
    sum_e b_e 2 (1 - Phi(c_e sqrt(dt) / sigma)) exactly at any dt."""
    N = 1_000_000
    for dt in (2e-3, 2e-2):
        g, st, c = _exit_run(orc, dt, N)
        p = cf.p_no_hit_first_vertex_substep(EXIT["b"], EXIT["c"], EXIT["sigma"], dt)
        emp = float((st.hits == 0).mean())
        assert abs(emp - p) < 5 * np.sqrt(p * (1 - p) / N), (dt, emp, p)


def test_exit_law_matches_renewal_equation(orc):
    """The edge after one step from the vertex follows the renewal equation's
    law (finite dt); the exit counters record it for particles that hit."""
    N, dt = 1_000_000, 2e-3
    G = cf.exit_law_one_step(EXIT["b"], EXIT["c"], EXIT["sigma"], dt)
    g, st, c = _exit_run(orc, dt, N)
    occ = np.bincount(st.edge, minlength=3) / N
    assert np.all(np.abs(occ - G) < 5 * np.sqrt(G * (1 - G) / N)), (occ, G)
    # exit counters: one record per particle that hit, on its final slot
    hit = st.hits > 0
    centre = c.exit_slot[g.vtx_offsets[0]:g.vtx_offsets[1]]
    assert np.array_equal(centre, np.bincount(st.edge[hit], minlength=3).astype(np.uint64))
    assert c.exit_slot[g.vtx_offsets[1]:].sum() == 0


def test_exit_probabilities_tend_to_b(orc):
    """Corollary 1: as dt -> 0 the exit law tends to b."""
    N = 400_000
    devs = []
    for dt in (2e-2, 2e-4, 2e-6):
        g, st, c = _exit_run(orc, dt, N, M=256)
        occ = np.bincount(st.edge, minlength=3) / N
        devs.append(np.abs(occ - np.array(EXIT["b"])).max())
    assert devs[0] > devs[1] > 0 or devs[1] < 5e-3
    assert devs[2] < 5 * np.sqrt(0.25 / N) + 2e-3, devs


def test_theorem2_bound_on_vertex_substeps(orc):
    """Theorem 2: with gamma = dt max mu^2 / sigma^2, the number M of vertex
    sub-steps of a step started on the vertex obeys
    P(M <= k) >= 1 - exp(-(k - gamma)^2 / (4k)).  Here M = hits + 1."""
    N = 300_000
    for dt in (2e-3, 2e-2):
        g, st, c = _exit_run(orc, dt, N, M=1000)
        gamma = dt * max(EXIT["c"]) ** 2 / EXIT["sigma"] ** 2
        Msub = st.hits.astype(np.int64) + 1
        ks = np.arange(1, 60)
        emp = np.array([(Msub <= k).mean() for k in ks])
        bound = cf.theorem2_bound(ks, gamma)
        assert np.all(emp >= bound - 5 * np.sqrt(0.25 / N)), (dt, emp, bound)
        assert c.truncations == 0


def test_truncation_zero_without_drift_and_counted_with_it(orc):
    """No drift: a vertex sub-step always leaves the vertex, so with M = 2 a
    step (one hit from inside the edge, then a move off the vertex) never
    reaches the split cap; with M = 1 every hit leaving time over is cut.  Strong inward drift with M = 2: every particle whose
    second hit leaves time over is counted once."""
    g, run = workloads.config1()
    st = orc.init(g, 20_000, orc.INIT_AT_VERTEX, vertex=0, seed=2)
    st1 = st.copy()
    c = orc.simulate(g, st, 0, 200, 1e-3, 2, max_splits=2)
    assert c.truncations == 0 and c.hits > 0
    c1 = orc.simulate(g, st1, 0, 200, 1e-3, 2, max_splits=1)
    assert c1.truncations == c1.hits
    N = 200_000
    g, st, c = _exit_run(orc, 2e-2, N, M=2)
    assert c.truncations == int((st.hits >= 2).sum())
    assert int(st.hits.max()) == 2
