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
