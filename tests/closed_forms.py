"""Closed forms that pin the oracle (and, through the oracle, the GPU path).

Everything here is derived from the mathematics of the diffusion, not from
the discrete scheme:

* reflected heat kernel on a segment (method of images);
* survival of Brownian motion on [0, l] reflected at 0 and absorbed at l
  (eigenfunction expansion);
* stationary densities on a star with the standard gluing conditions: on
  edge e, pi_e(x) = C (b_e / D_e) exp(-(V_e(x) - V_e(0)) / D_e) with
  D = sigma^2 / 2 and mu = -V' (zero flux on every edge, and the vertex
  condition D_e pi_e(0) proportional to b_e from the adjoint of the
  generator under sum_e b_e f'_e(v) = 0);
* the exit law of one EM step started on a vertex with constant inward
  drift, from its renewal equation (the law of the time a vertex sub-step
  consumes, sigma^2 W^2 / c^2, is explicit);
* P(no hit in the first vertex sub-step) = sum_e b_e 2 (1 - Phi(c_e sqrt(dt) / sigma))
  (the event behind Theorem 3).
"""
import numpy as np
from scipy import integrate, special, stats


def reflected_segment_bin_probs(edges, z0, length, s, n_images=12):
    """P(Z in [edges[i], edges[i+1]]) for Brownian motion with variance s^2
    started at z0, reflected at 0 and at ``length``."""
    edges = np.asarray(edges, np.float64)
    cdf = np.zeros_like(edges)
    for n in range(-n_images, n_images + 1):
        cdf += stats.norm.cdf((edges - z0 - 2 * n * length) / s)
        cdf += stats.norm.cdf((edges + z0 - 2 * n * length) / s)
    return np.diff(cdf)


def survival_reflect_absorb(t, x0, length, sigma, n_terms=400):
    """P(not absorbed by t) for Brownian motion (diffusivity sigma^2/2) from x0
    on [0, length], reflected at 0 and absorbed at ``length``."""
    D = 0.5 * sigma * sigma
    n = np.arange(n_terms)
    k = (2 * n + 1) * np.pi / (2 * length)
    terms = 4 * (-1.0) ** n / ((2 * n + 1) * np.pi) * np.cos(k * x0) * np.exp(-D * k * k * t)
    return float(terms.sum())


def star_stationary(lengths, potentials, b, sigma, grid=20001):
    """Stationary law on a finite star (centre at x = 0 of every edge,
    reflecting leaves).  ``potentials[e](x)`` is V_e.  Returns per-edge masses
    and, per edge, (x grid, density) normalised to total mass 1."""
    D = 0.5 * np.asarray(sigma, np.float64) ** 2 * np.ones(len(lengths))
    xs, dens, mass = [], [], []
    for e, L in enumerate(lengths):
        x = np.linspace(0.0, L, grid)
        V = potentials[e](x)
        p = b[e] / D[e] * np.exp(-(V - V[0]) / D[e])
        xs.append(x)
        dens.append(p)
        mass.append(integrate.trapezoid(p, x))
    tot = float(np.sum(mass))
    return np.array(mass) / tot, xs, [d / tot for d in dens]


def sample_from_density(rng, x, d, n):
    """Inverse-CDF samples from a tabulated density on the grid x."""
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (d[1:] + d[:-1]) * np.diff(x))])
    cdf /= cdf[-1]
    return np.interp(rng.random(n), cdf, x)


def binned(x, d, edges):
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (d[1:] + d[:-1]) * np.diff(x))])
    return np.diff(np.interp(edges, x, cdf))


def p_no_hit_first_vertex_substep(b, c, sigma, dt):
    """P(the first sub-step from a vertex stays inside the edge) when the
    edge is drawn from b and the drift on edge e is the constant -c_e
    (towards the vertex): the move c_e dt must be beaten by sigma sqrt(dt)|W|."""
    a = np.asarray(c, np.float64) / sigma
    return float(np.sum(np.asarray(b) * 2 * stats.norm.sf(a * np.sqrt(dt))))


def exit_law_one_step(b, c, sigma, dt, n_grid=600, n_gl=96, n_iter=200):
    """Law of the edge a particle is on after one EM step started on a vertex
    (edge drawn from b, constant drift -c_e towards the vertex, edges long
    enough never to reach their far end).

    A vertex sub-step on edge i with time h either leaves the vertex (prob.
    q_i(h) = 2(1 - Phi(a_i sqrt h)), a_i = c_i / sigma) or returns to it
    after consuming s = sigma^2 W^2 / c_i^2, whose density on (0, h) is
    a_i phi(a_i sqrt s) / sqrt s; then a fresh edge is drawn from b.  So
        G_e(h) = b_e q_e(h) + sum_i b_i int_0^h a_i phi(a_i sqrt s) s^-1/2 G_e(h - s) ds.
    Solved by fixed-point iteration (the kernel mass is P(return) < 1) on a
    grid uniform in sqrt(h), with s = t^2 removing the singularity."""
    b = np.asarray(b, np.float64)
    a = np.asarray(c, np.float64) / sigma
    r = np.linspace(0.0, np.sqrt(dt), n_grid)    # grid in sqrt(h)
    h = r * r
    tg, wg = np.polynomial.legendre.leggauss(n_gl)
    E = b.size
    G = np.tile(b[:, None], (1, n_grid))           # initial guess
    q = 2 * stats.norm.sf(a[:, None] * np.sqrt(h)[None, :])   # [E, grid]
    for _ in range(n_iter):
        newG = b[:, None] * q
        for j in range(1, n_grid):
            hj = h[j]
            T = np.sqrt(hj)
            t = 0.5 * T * (tg + 1.0)
            w = 0.5 * T * wg
            rem = np.sqrt(np.maximum(hj - t * t, 0.0))
            Gi = np.stack([np.interp(rem, r, G[e]) for e in range(E)])   # [E, n_gl]
            # int_0^sqrt(h) 2 a_i phi(a_i t) G(h - t^2) dt
            ker = (b[:, None] * 2 * a[:, None] * stats.norm.pdf(a[:, None] * t[None, :]))  # [E_i, n_gl]
            newG[:, j] += (Gi * (ker.sum(axis=0) * w)[None, :]).sum(axis=1)
        if np.max(np.abs(newG - G)) < 1e-14:
            G = newG
            break
        G = newG
    return G[:, -1]


def theorem2_bound(k, gamma):
    """Theorem 2: P(M <= k) >= 1 - exp(-(k - gamma)^2 / (4k)) for k > gamma,
    with M the number of vertex sub-steps of one step started on the vertex."""
    k = np.asarray(k, np.float64)
    return np.where(k > gamma, 1 - np.exp(-(k - gamma) ** 2 / (4 * k)), 0.0)


def norm_sf(x):
    return 0.5 * special.erfc(x / np.sqrt(2))


# ------------------------------------------------------- Wentzell vertices
# A vertex with the general gluing condition a f(v) - sum_e b_e f'_e(v) +
# c (L f)(v) = 0 (beta = sum_e b_e): killing at rate kappa = a / beta per
# unit of local time at v (local time in units of length, the reflection
# term of the distance to v), and gamma = c / beta units of time spent on v
# per unit of local time.  For zero drift and diffusion sigma the density u
# on an edge then satisfies u_x(v) = kappa u(v) (mass is lost at the rate
# kappa times the local-time rate sigma^2 u(v) / 2), and the resolvent of
# the process started on v follows from excursion theory: the inverse local
# time of reflected Brownian motion has Laplace exponent sqrt(2 lambda) /
# sigma, so E_v int e^{-lambda t} 1{X_t = v} dt =
# gamma / (sqrt(2 lambda) / sigma + gamma lambda + kappa).


def robin_segment_survival(t, length, sigma, kappa, n_terms=400):
    """P(alive at t) on [0, length] from the uniform law, killing rate kappa
    per unit local time at 0 (u_x(0) = kappa u(0)), reflecting at length.
    Eigenfunctions cos(k (length - x)) with k tan(k length) = kappa."""
    from scipy import optimize
    D = 0.5 * sigma * sigma
    ks = []
    for n in range(n_terms):
        lo, hi = n * np.pi / length, (n + 0.5) * np.pi / length
        ks.append(optimize.brentq(lambda k: k * np.tan(k * length) - kappa,
                                  lo + 1e-12 / length, hi - 1e-12 / length))
    k = np.array(ks)
    integral = np.sin(k * length) / k
    norm = length / 2 + np.sin(2 * k * length) / (4 * k)
    return float((integral ** 2 / norm / length * np.exp(-D * k * k * t)).sum())


def _sticky_roots(sigma, gamma, kappa):
    """Roots r of s^2 + a s + kappa / gamma, a = sqrt(2) / (gamma sigma):
    the atom's resolvent is 1 / ((sqrt(lambda) - r1)(sqrt(lambda) - r2))."""
    a = np.sqrt(2.0) / (gamma * sigma)
    disc = np.sqrt(complex(a * a - 4.0 * kappa / gamma))
    return (-a + disc) / 2.0, (-a - disc) / 2.0


def sticky_halfline_at_vertex(t, sigma, gamma, kappa=0.0):
    """P(X_t = v, alive) for the process started on v on a half-line [0, inf)
    (one edge, zero drift).  The inverse Laplace transform of
    1 / ((sqrt(l) - r1)(sqrt(l) - r2)) is
    (r1 erfcx(-r1 sqrt t) - r2 erfcx(-r2 sqrt t)) / (r1 - r2); with kappa = 0
    it is erfcx(sqrt(2 t) / (gamma sigma))."""
    from scipy import special
    if kappa == 0.0:
        return float(special.erfcx(np.sqrt(2.0 * t) / (gamma * sigma)))
    r1, r2 = _sticky_roots(sigma, gamma, kappa)
    st = np.sqrt(t)
    v = (r1 * special.erfcx(-r1 * st) - r2 * special.erfcx(-r2 * st)) / (r1 - r2)
    return float(np.real(v))


def sticky_halfline_alive(t, sigma, gamma, kappa):
    """P(alive at t) from v on the half-line: mass is lost at kappa times the
    local-time rate, and the time on v is gamma times the local time, so
    d/dt P(alive) = -(kappa / gamma) P(X_t = v)."""
    from scipy import integrate
    if kappa == 0.0:
        return 1.0
    val, _ = integrate.quad(lambda u: sticky_halfline_at_vertex(u, sigma, gamma, kappa),
                            0.0, t, limit=200)
    return 1.0 - kappa / gamma * val


def killing_halfline_alive(t, sigma, kappa):
    """P(alive at t) from v on a half-line with killing only: E exp(-kappa l_t)
    with l_t distributed as |sigma B_t| (Levy), i.e. erfcx(kappa sigma
    sqrt(t / 2))."""
    from scipy import special
    return float(special.erfcx(kappa * sigma * np.sqrt(t / 2.0)))


def sticky_star_stationary(lengths, b_hat, sigma, gamma):
    """Stationary law on a finite star with zero drift, constant sigma,
    reflecting leaves and a sticky centre: density C b_e / D on edge e
    (D = sigma^2 / 2) and an atom gamma C on the centre (gamma times the
    local-time rate D sum_e pi_e(0) = C).  Returns (atom, per-edge masses)."""
    lengths = np.asarray(lengths, np.float64)
    b_hat = np.asarray(b_hat, np.float64)
    D = 0.5 * sigma * sigma
    C = 1.0 / (float((b_hat * lengths).sum()) / D + gamma)
    return gamma * C, C * b_hat * lengths / D
