"""Closed-form stationary laws of the diffusion on a finite star: the
analytic targets of the density-error measurement (Sec. 4.1).  This is the
mathematics of the limit process, not the scheme: neither the oracle nor the
library uses it.

On a star whose edges all start at the centre vertex (x = 0), with constant
sigma, drift mu_e(x) = a_e + c_e x = -V_e'(x) and reflecting leaves, the
stationary density under the standard gluing conditions is
pi_e(x) = C b_e / D exp(-(V_e(x) - V_e(0)) / D), D = sigma^2 / 2: zero flux
on every edge, and D pi_e(0) / b_e equal on all edges at the vertex.  The
paper's 5-edge forms (linear and quadratic potentials) are the cases
c = 0 and a = 0, truncated to finite edges.
"""
from __future__ import annotations

import numpy as np
from scipy import special


def _bin_integrals(a: float, c: float, D: float, edges: np.ndarray) -> np.ndarray:
    """Integrals of exp(-(V(x) - V(0)) / D) over consecutive bin edges, with
    V(x) = -a x - c x^2 / 2."""
    if c == 0.0 and a == 0.0:
        return np.diff(edges)
    if c == 0.0:
        # exp(a x / D): exact antiderivative, written so it never overflows
        # for inward drift (a < 0)
        r = a / D
        return (np.expm1(r * edges[1:]) - np.expm1(r * edges[:-1])) / r
    if c < 0.0:
        # exp(-(|c| / 2D) (x - m)^2 + |c| m^2 / 2D), m = -a / c
        s = -c / (2.0 * D)
        m = -a / c
        z = np.sqrt(s) * (edges - m)
        scale = 0.5 * np.sqrt(np.pi / s) * np.exp(s * m * m)
        # erf differences lose digits far in one tail; use erfc there
        lo, hi = z[:-1], z[1:]
        right = lo > 0
        out = np.where(right,
                       special.erfc(lo) - special.erfc(hi),
                       special.erf(hi) - special.erf(lo))
        return scale * out
    raise ValueError("c > 0 (a confining-free potential) is not supported")


def star_csr_masses(g, bin_offsets, true_upper) -> np.ndarray:
    """Stationary mass of each bin of a ``csr_bins`` table on a star (finite
    or semi-infinite edges; every edge starts at vertex 0), total mass 1.
    ``true_upper`` holds the real upper bounds (inf for a semi-infinite
    edge's tail bin)."""
    E = int(g.n_edges)
    if not np.all(np.asarray(g.edge_init) == 0):
        raise ValueError("not a star centred at vertex 0")
    sig = np.asarray(g.sigma, np.float64)
    if not np.all(sig == sig[0]):
        raise ValueError("sigma must be constant")
    D = 0.5 * float(sig[0]) ** 2
    b = np.zeros(E)
    for s in range(int(g.vtx_offsets[0]), int(g.vtx_offsets[1])):
        b[int(g.slot_edge[s])] += float(g.slot_jump_prob[s])
    off = np.asarray(bin_offsets, np.int64)
    up = np.asarray(true_upper, np.float64)
    out = np.zeros(int(off[-1]))
    for e in range(E):
        edges = np.concatenate([[0.0], up[off[e]:off[e + 1]]])
        out[off[e]:off[e + 1]] = b[e] / D * _bin_integrals(
            float(g.drift_a[e]), float(g.drift_c[e]), D, edges)
    return out / out.sum()


def star_bin_means(g, bins: int) -> np.ndarray:
    """Bin averages [E, bins] of the stationary density of a star built like
    ``workloads.star_graph`` (every edge starts at vertex 0), normalised to
    total mass 1 over the graph.  The bins of edge e cover its binned length
    (``bin_span``, default the length); the last one also holds the mass
    beyond, as the histograms count it."""
    E = int(g.n_edges)
    if not np.all(np.asarray(g.edge_init) == 0):
        raise ValueError("not a star centred at vertex 0")
    sig = np.asarray(g.sigma, np.float64)
    if not np.all(sig == sig[0]):
        raise ValueError("sigma must be constant")
    D = 0.5 * float(sig[0]) ** 2
    b = np.zeros(E)
    for s in range(int(g.vtx_offsets[0]), int(g.vtx_offsets[1])):
        b[int(g.slot_edge[s])] += float(g.slot_jump_prob[s])
    span = np.asarray(g.length if getattr(g, "bin_span", None) is None else g.bin_span,
                      np.float64)
    out = np.zeros((E, bins))
    for e in range(E):
        edges = np.linspace(0.0, float(span[e]), bins + 1)
        edges[-1] = float(g.length[e])  # the last bin runs to the edge's end
        out[e] = b[e] / D * _bin_integrals(float(g.drift_a[e]), float(g.drift_c[e]), D, edges)
    out /= out.sum()
    width = span[:, None] / bins
    return out / width
