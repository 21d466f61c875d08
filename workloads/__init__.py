"""Seeded synthetic inputs for the metric-graph particle step.

This module only builds inputs: graph tables (edges, lengths, drift and
diffusion coefficients, vertex-edge jump probabilities in CSR form) and run
settings.  It holds none of the method's arithmetic, so both the FP64 CPU
oracle and the GPU library read the same inputs from here without sharing
any code with each other.

Graph description (same fields as the C-ABI ``mg_graph_desc``):

* ``edge_init[e]``, ``edge_term[e]``: the two vertices of edge e; positions
  on e are measured from ``edge_init[e]`` (x in [0, length[e]]).
* ``drift_a[e] + drift_c[e] * x``: the drift mu_e(x) in that coordinate.
* ``sigma[e]``: the diffusion coefficient on e.
* ``vtx_offsets``/``slot_edge``/``slot_orient``/``slot_jump_prob``: per
  vertex v, slots ``vtx_offsets[v] .. vtx_offsets[v+1]-1`` list the incident
  edge ends; orient 0 means v is the edge's initial vertex (a particle enters
  at x = 0), 1 means its terminal vertex (enters at x = L).  The jump
  probabilities b_{v,e} of the standard gluing conditions sum to 1 per vertex.
* ``vtx_kind[v]``: 0 standard vertex, 1 absorbing vertex, 2 mirror vertex
  (a leaf that reflects a proposal leaving through it into the edge), 3
  Wentzell vertex with ``vtx_kill[v]`` = a_v and ``vtx_sticky[v]`` = c_v; its
  jump probabilities then sum to 1 - a_v - c_v.
* A semi-infinite edge has ``length`` = inf; its terminal vertex is a vertex
  at infinity of its own (one slot, never reached).
* ``bin_span[e]`` (optional): the length of e the uniform histograms cover
  (default the edge length; required for a semi-infinite edge).
* ``drift_c2``, ``drift_c3``, ``sigma_c1``, ``sigma_c2``, ``sigma_c3``
  (optional): higher terms of the coefficient functions, mu_e(x) = a + c x +
  c2 x^2 + c3 x^3 and sigma_e(x) = sigma + s1 x + s2 x^2 + s3 x^3.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "GraphDesc", "from_edges", "star_graph", "segment", "random_tree",
    "config1", "config2", "config3", "config4", "config5", "paper_star5",
    "csr_bins",
]


@dataclass
class GraphDesc:
    n_vertices: int
    n_edges: int
    edge_init: np.ndarray
    edge_term: np.ndarray
    length: np.ndarray
    drift_a: np.ndarray
    drift_c: np.ndarray
    sigma: np.ndarray
    vtx_offsets: np.ndarray
    slot_edge: np.ndarray
    slot_orient: np.ndarray
    slot_jump_prob: np.ndarray
    vtx_kind: np.ndarray
    bin_span: np.ndarray | None = None
    meta: dict = field(default_factory=dict)
    # higher coefficient terms (None: zero): mu = a + c x + c2 x^2 + c3 x^3,
    # sigma(x) = sigma + s1 x + s2 x^2 + s3 x^3
    drift_c2: np.ndarray | None = None
    drift_c3: np.ndarray | None = None
    sigma_c1: np.ndarray | None = None
    sigma_c2: np.ndarray | None = None
    sigma_c3: np.ndarray | None = None
    # Wentzell vertices (vtx_kind 3): a_v (killing) and c_v (stickiness) per
    # vertex, with a_v + sum_e b_ve + c_v = 1 (None: zero)
    vtx_kill: np.ndarray | None = None
    vtx_sticky: np.ndarray | None = None
    # tabulated coefficients (None: no tables): [E+1] knot offsets; edge e
    # with K + 1 >= 2 knots has drift and diffusion values and derivatives
    # at x_j = j L_e / K, interpolated by cubic Hermite polynomials
    table_offsets: np.ndarray | None = None
    table_mu: np.ndarray | None = None
    table_dmu: np.ndarray | None = None
    table_sigma: np.ndarray | None = None
    table_dsigma: np.ndarray | None = None

    @property
    def nnz(self) -> int:
        return int(self.vtx_offsets[-1])


def from_edges(n_vertices, edge_init, edge_term, length, drift_a=None,
               drift_c=None, sigma=1.0, weight_init=None, weight_term=None,
               vtx_kind=None, meta=None, bin_span=None) -> GraphDesc:
    """Build the CSR slot table from an edge list.

    ``weight_init[e]``/``weight_term[e]`` are nonnegative weights of edge e at
    its initial/terminal vertex; they are divided by their per-vertex sum to
    give the jump probabilities (all ones = uniform jump probabilities).
    Slots of a vertex are ordered by edge id, the initial end before the
    terminal end for a self-loop.
    """
    ei = np.asarray(edge_init, dtype=np.int32)
    et = np.asarray(edge_term, dtype=np.int32)
    E = int(ei.shape[0])
    V = int(n_vertices)
    L = np.broadcast_to(np.asarray(length, dtype=np.float64), (E,)).copy()
    a = np.zeros(E) if drift_a is None else np.broadcast_to(np.asarray(drift_a, np.float64), (E,)).copy()
    c = np.zeros(E) if drift_c is None else np.broadcast_to(np.asarray(drift_c, np.float64), (E,)).copy()
    s = np.broadcast_to(np.asarray(sigma, dtype=np.float64), (E,)).copy()
    wi = np.ones(E) if weight_init is None else np.asarray(weight_init, np.float64)
    wt = np.ones(E) if weight_term is None else np.asarray(weight_term, np.float64)
    kind = np.zeros(V, np.uint8) if vtx_kind is None else np.asarray(vtx_kind, np.uint8).copy()

    # (vertex, edge, end) triples sorted by vertex, then edge, then end.
    verts = np.concatenate([ei, et])
    edges = np.concatenate([np.arange(E), np.arange(E)]).astype(np.int32)
    ends = np.concatenate([np.zeros(E, np.uint8), np.ones(E, np.uint8)])
    w = np.concatenate([wi, wt])
    order = np.lexsort((ends, edges, verts))
    verts, edges, ends, w = verts[order], edges[order], ends[order], w[order]
    counts = np.bincount(verts, minlength=V)
    offsets = np.zeros(V + 1, np.int32)
    np.cumsum(counts, out=offsets[1:])
    tot = np.bincount(verts, weights=w, minlength=V)
    b = np.where(tot[verts] > 0, w / np.where(tot[verts] > 0, tot[verts], 1.0), 0.0)
    span = None if bin_span is None else np.broadcast_to(
        np.asarray(bin_span, np.float64), (E,)).copy()
    return GraphDesc(V, E, ei, et, L, a, c, s, offsets, edges.astype(np.int32),
                     ends.astype(np.uint8), b.astype(np.float64), kind, span,
                     dict(meta or {}))


def star_graph(n_edges, length=1.0, drift_a=None, drift_c=None, sigma=1.0,
               b_center=None, meta=None, bin_span=None, leaf_kind=0) -> GraphDesc:
    """Finite star: centre vertex 0, leaf vertex i+1 at the far end of edge i.

    Edge i runs from the centre (x = 0) to leaf i+1 (x = L_i); each leaf is a
    degree-1 vertex (jump probability 1, i.e. reflecting by a split there), or
    with ``leaf_kind`` = 2 a mirror vertex (reflecting by the mirror image)."""
    E = int(n_edges)
    ei = np.zeros(E, np.int32)
    et = np.arange(1, E + 1, dtype=np.int32)
    wi = np.ones(E) if b_center is None else np.asarray(b_center, np.float64)
    kind = np.zeros(E + 1, np.uint8)
    kind[1:] = leaf_kind
    return from_edges(E + 1, ei, et, length, drift_a, drift_c, sigma,
                      weight_init=wi, meta=meta, bin_span=bin_span, vtx_kind=kind)


def segment(length=1.0, drift_a=0.0, drift_c=0.0, sigma=1.0, end_kind=0) -> GraphDesc:
    """One edge between two degree-1 vertices: reflecting by a split there,
    or with ``end_kind`` = 2 mirror vertices."""
    return from_edges(2, [0], [1], [length], [drift_a], [drift_c], sigma,
                      vtx_kind=[end_kind, end_kind])


def random_tree(n_edges, rng, length_range=(0.2, 3.0), sigma=np.sqrt(2.0),
                quadratic=False, meta=None) -> GraphDesc:
    """Random recursive tree: vertex i >= 1 hangs from a uniform earlier vertex.

    With ``quadratic`` each edge carries the potential k (x - m)^2
    (k ~ U[0.5, 4], m ~ U[0, L]), i.e. drift 2 k m - 2 k x; otherwise no drift.
    Jump probabilities are uniform per vertex."""
    E = int(n_edges)
    parents = np.array([rng.integers(0, i) for i in range(1, E + 1)], np.int32)
    ei = parents
    et = np.arange(1, E + 1, dtype=np.int32)
    L = rng.uniform(*length_range, size=E)
    a = c = None
    if quadratic:
        k = rng.uniform(0.5, 4.0, size=E)
        m = rng.uniform(0.0, 1.0, size=E) * L
        a, c = 2.0 * k * m, -2.0 * k
    return from_edges(E + 1, ei, et, L, a, c, sigma, meta=meta)


# ----------------------------------------------------------------- configs

def config1() -> tuple[GraphDesc, dict]:
    """Plain EM on a 3-edge star: lengths 1, no drift, sigma 1, b = 1/3;
    1e4 particles start at the centre; dt 1e-3, 1000 steps, 8 splits per step
    at most, Philox seed 0, 100 bins per edge."""
    g = star_graph(3, 1.0, None, None, 1.0, meta={"name": "star3"})
    run = dict(n_particles=10_000, init="vertex", vertex=0, dt=1e-3,
               n_steps=1000, max_splits=8, seed=0, bins=100)
    return g, run


def config2(seed: int = 2) -> tuple[GraphDesc, dict]:
    """Langevin on a 64-edge star: L ~ U[0.5, 2], potential
    V_e(x) = k_e (x - m_e)^2 with k_e ~ U[0.5, 4], m_e ~ U[0, L_e], sigma =
    sqrt(2) (so the stationary law is exp(-V) up to the vertex weights), jump
    probabilities proportional to the diffusivity (all equal: 1/64); 1e7
    particles uniform by length, dt in {1e-2, 1e-3}, 1e4 steps, 256 bins."""
    rng = np.random.default_rng(seed)
    E = 64
    L = rng.uniform(0.5, 2.0, size=E)
    k = rng.uniform(0.5, 4.0, size=E)
    m = rng.uniform(0.0, 1.0, size=E) * L
    sig = np.sqrt(2.0)
    diff = np.full(E, 0.5 * sig * sig)
    g = star_graph(E, L, 2.0 * k * m, -2.0 * k, sig, b_center=diff,
                   meta={"name": "langevin_star64", "k": k, "m": m})
    run = dict(n_particles=10_000_000, init="uniform", dts=(1e-2, 1e-3),
               n_steps=10_000, max_splits=8, seed=0, bins=256)
    return g, run


def paper_star5(potential: str = "linear", length: float = 2.0,
                sigma: float = 1.0, bin_span: float = 2.0,
                leaf_kind: int = 0) -> GraphDesc:
    """The 5-edge star of the paper's experiments (Sec. 4): mu_i = -10 i
    (linear potential) or mu_i = -10 i x (quadratic potential), uniform
    b = 1/5.  ``length`` = inf gives the paper's star metric graph (Def. 3:
    one vertex, semi-infinite edges; here each edge's far end is a vertex at
    infinity of its own); a finite length truncates the edges with
    reflecting leaves.  Uniform histograms cover [0, min(length, bin_span)]
    of every edge.  ``leaf_kind`` = 2 makes the leaves of a finite star
    mirror vertices, as the paper's star kernel reflects at far ends."""
    i = np.arange(1, 6, dtype=np.float64)
    if potential == "linear":
        a, c = -10.0 * i, np.zeros(5)
    elif potential == "quadratic":
        a, c = np.zeros(5), -10.0 * i
    else:
        raise ValueError(potential)
    return star_graph(5, length, a, c, sigma,
                      meta={"name": f"paper_star5_{potential}"},
                      bin_span=min(float(length), float(bin_span)),
                      leaf_kind=leaf_kind)


def double_well_star(n_edges: int = 64, seed: int = 6) -> GraphDesc:
    """Star with non-affine coefficients on every edge: L ~ U[0.5, 2], a
    double-well potential V_e(x) = h_e ((x - p_e)(x - q_e))^2 / L_e^4 with
    wells at p_e = L/4 and q_e = 3L/4 and h_e ~ U[1, 4], drift mu_e = -V_e'
    (a cubic), and a graded diffusion sigma_e(x) = sqrt(2) (1 + g_e x / L_e)
    with g_e ~ U[-0.3, 0.5]; uniform jump probabilities at the centre."""
    rng = np.random.default_rng(seed)
    E = int(n_edges)
    L = rng.uniform(0.5, 2.0, size=E)
    h = rng.uniform(1.0, 4.0, size=E)
    gr = rng.uniform(-0.3, 0.5, size=E)
    p, q = 0.25 * L, 0.75 * L
    # V = h/L^4 (x^2 - s x + t)^2 with s = p + q, t = p q, so
    # -V' = -(2h/L^4)(x^2 - s x + t)(2x - s)
    k = 2.0 * h / L ** 4
    sm, t = p + q, p * q
    c3 = -k * 2.0
    c2 = -k * (-3.0 * sm)
    c1 = -k * (2.0 * t + sm * sm)
    c0 = -k * (-sm * t)
    sig = np.sqrt(2.0)
    g = star_graph(E, L, c0, c1, sig, meta={"name": f"double_well_star{E}"})
    g.drift_c2, g.drift_c3 = c2, c3
    g.sigma_c1 = sig * gr / L
    return g


def wentzell_star(n_edges: int = 5, seed: int = 7, cubic: bool = False) -> GraphDesc:
    """Star whose centre and some leaves are Wentzell vertices (Sec. 2.2's
    general gluing condition): L ~ U[0.2, 0.8], drift a_e ~ U[-6, 2] toward
    or away from the centre, sigma 1 (with ``cubic``: a graded diffusion
    sigma_e(x) = 1 + g_e x / L_e, g_e ~ U[-0.3, 0.5], and a cubic drift term
    c3_e ~ U[-4, 4]); the centre kills (a = 0.05) and is sticky (c = 0.15)
    with b-hat ~ U[0.5, 1.5] normalised; leaf 1 kills (a = 0.3, c = 0.2),
    leaf 2 is sticky only (c = 0.5), leaf 3 kills only (a = 0.4), the other
    leaves are standard.  b = (1 - a - c) b-hat at each Wentzell vertex."""
    rng = np.random.default_rng(seed)
    E = int(n_edges)
    L = rng.uniform(0.2, 0.8, size=E)
    a = rng.uniform(-6.0, 2.0, size=E)
    bh = rng.uniform(0.5, 1.5, size=E)
    bh = bh / bh.sum()
    g = star_graph(E, L, a, None, 1.0, b_center=bh,
                   meta={"name": f"wentzell_star{E}{'_cubic' if cubic else ''}"})
    if cubic:
        gr = rng.uniform(-0.3, 0.5, size=E)
        g.sigma_c1 = gr / L
        g.drift_c3 = rng.uniform(-4.0, 4.0, size=E)
    kill = np.zeros(E + 1)
    sticky = np.zeros(E + 1)
    kill[0], sticky[0] = 0.05, 0.15
    kill[1], sticky[1] = 0.3, 0.2
    sticky[2] = 0.5
    kill[3] = 0.4
    for v in (0, 1, 2, 3):
        g.vtx_kind[v] = 3
        s0, s1 = g.vtx_offsets[v], g.vtx_offsets[v + 1]
        g.slot_jump_prob[s0:s1] *= 1.0 - kill[v] - sticky[v]
    g.vtx_kill, g.vtx_sticky = kill, sticky
    return g


def tabulate(g: GraphDesc, knots, mu, dmu, sigma, dsigma, edges=None) -> GraphDesc:
    """Give edges (all, or the listed ones) tabulated coefficients: K_e + 1
    equally spaced knots x_j = j L_e / K_e (``knots`` per edge, or one count
    for all), with drift and diffusion values and derivatives from the
    functions mu(e, x), dmu(e, x), sigma(e, x), dsigma(e, x) (numpy-vectorised
    in x).  Edges without a table keep their affine or cubic coefficients."""
    E = g.n_edges
    sel = set(range(E) if edges is None else edges)
    k = np.broadcast_to(np.asarray(knots, np.int64), (E,))
    off = np.zeros(E + 1, np.int32)
    cols = {n: [] for n in ("table_mu", "table_dmu", "table_sigma", "table_dsigma")}
    for e in range(E):
        if e not in sel:
            off[e + 1] = off[e]
            continue
        K = int(k[e])
        x = np.arange(K + 1) * (g.length[e] / K)
        for n, f in (("table_mu", mu), ("table_dmu", dmu), ("table_sigma", sigma),
                     ("table_dsigma", dsigma)):
            cols[n].append(np.asarray(f(e, x), np.float64) * np.ones(K + 1))
        off[e + 1] = off[e] + K + 1
    g.table_offsets = off
    for n, v in cols.items():
        setattr(g, n, np.concatenate(v) if v else np.zeros(0))
    return g


def periodic_star(n_edges: int = 8, seed: int = 9, knots: int = 16) -> GraphDesc:
    """Star whose coefficients are not polynomials, given as tables: on edge
    e (L ~ U[0.5, 1.5]) the potential V_e(x) = A_e (1 - cos(2 pi f_e x / L_e))
    (A_e ~ U[0.5, 2], f_e in {1, 2}) gives the drift mu = -V', and the
    diffusion is sigma_e(x) = 1 + g_e sin(pi x / L_e) (g_e ~ U[-0.3, 0.5]);
    both tabulated at ``knots`` + 1 equally spaced points per edge (values
    and derivatives), uniform jump probabilities at the centre."""
    rng = np.random.default_rng(seed)
    E = int(n_edges)
    L = rng.uniform(0.5, 1.5, size=E)
    A = rng.uniform(0.5, 2.0, size=E)
    f = rng.integers(1, 3, size=E).astype(np.float64)
    gr = rng.uniform(-0.3, 0.5, size=E)
    g = star_graph(E, L, 0.0, 0.0, 1.0, meta={"name": f"periodic_star{E}"})
    w = 2.0 * np.pi * f / L

    def mu(e, x):
        return -A[e] * w[e] * np.sin(w[e] * x)

    def dmu(e, x):
        return -A[e] * w[e] ** 2 * np.cos(w[e] * x)

    def sig(e, x):
        return 1.0 + gr[e] * np.sin(np.pi * x / L[e])

    def dsig(e, x):
        return gr[e] * (np.pi / L[e]) * np.cos(np.pi * x / L[e])
    g.meta["coef"] = (mu, dmu, sig, dsig)
    return tabulate(g, knots, mu, dmu, sig, dsig)


def csr_bins(g: GraphDesc, width: float, n_finite: int):
    """Per-edge bins for ``histogram_csr``: on each edge ``n_finite`` bins of
    ``width`` from x = 0 (clipped to the edge's length), then, on an edge
    longer than that, one more bin whose upper boundary is the edge's length
    (or, on a semi-infinite edge, that takes every position beyond).
    Returns (bin_offsets [E+1], bin_upper [nnz bins], true upper bounds
    including inf)."""
    off = [0]
    up, true_up = [], []
    for e in range(int(g.n_edges)):
        L = float(g.length[e])
        k = 0
        for k in range(1, n_finite + 1):
            u = k * width
            if u >= L:
                break
            up.append(u)
            true_up.append(u)
        else:
            k = n_finite + 1
        if np.isinf(L):
            # the tail bin: its stored boundary is any finite value above the
            # previous one; positions beyond it land there as well
            up.append((n_finite + 1) * width)
            true_up.append(np.inf)
        else:
            up.append(L)
            true_up.append(L)
        off.append(len(up))
    return (np.asarray(off, np.int32), np.asarray(up, np.float64),
            np.asarray(true_up, np.float64))


def _vascular_topology(rng, n_vertices, n_edges, n_leaves, side):
    """Connected spatial graph with degree 3 at internal vertices and degree 1
    at leaves: a degree-capped nearest-neighbour spanning tree of the internal
    points, leaves hung on the nearest internal vertex with a free stub, then
    the remaining stubs paired with nearby vertices (each such pair closes one
    independent cycle)."""
    from scipy.spatial import cKDTree
    import heapq

    n_int = n_vertices - n_leaves
    pts = rng.uniform(0.0, side, size=(n_vertices, 3))
    ip = pts[:n_int]
    tree = cKDTree(ip)
    deg = np.zeros(n_vertices, np.int64)
    adj = [set() for _ in range(n_vertices)]
    edges = []

    def add(u, v):
        edges.append((u, v))
        adj[u].add(v)
        adj[v].add(u)
        deg[u] += 1
        deg[v] += 1

    # 1. spanning tree of internal vertices, tree degree <= 3 (Prim order).
    in_tree = np.zeros(n_int, bool)
    heap = []
    knn = 10

    def push(u):
        d, nb = tree.query(ip[u], k=knn)
        for dd, v in zip(np.atleast_1d(d), np.atleast_1d(nb)):
            if v != u and not in_tree[v]:
                heapq.heappush(heap, (float(dd), int(u), int(v)))

    in_tree[0] = True
    push(0)
    n_in = 1
    while n_in < n_int:
        while heap:
            d, u, v = heapq.heappop(heap)
            if in_tree[v] or deg[u] >= 3:
                continue
            add(u, v)
            in_tree[v] = True
            n_in += 1
            push(v)
        if n_in < n_int:
            # restart: nearest free-capacity tree vertex for some outsider
            out = np.flatnonzero(~in_tree)
            cap = np.flatnonzero(in_tree & (deg[:n_int] < 2))
            ct = cKDTree(ip[cap])
            d, j = ct.query(ip[out[0]])
            add(int(cap[j]), int(out[0]))
            in_tree[out[0]] = True
            n_in += 1
            push(int(out[0]))
    # 2. leaves hang on the nearest internal vertex with a free stub.
    for lf in range(n_int, n_vertices):
        k = 8
        while True:
            d, nb = tree.query(pts[lf], k=min(k, n_int))
            cand = [int(v) for v in np.atleast_1d(nb) if deg[v] < 3]
            if cand:
                add(cand[0], lf)
                break
            k *= 4
    # 3. pair the remaining internal stubs with nearby free vertices.
    free = [v for v in rng.permutation(n_int) for _ in range(3 - deg[v])]
    pending = set(int(v) for v in free)
    for u in free:
        u = int(u)
        if deg[u] >= 3:
            continue
        d, nb = tree.query(ip[u], k=24)
        for v in np.atleast_1d(nb):
            v = int(v)
            if v != u and deg[v] < 3 and v not in adj[u]:
                add(u, v)
                break
    left = [v for v in range(n_int) for _ in range(3 - deg[v])]
    cycle_edges = [i for i, (u, v) in enumerate(edges) if u < n_int and v < n_int]
    while left:
        u = left.pop()
        partner = None
        for j, v in enumerate(left):
            if v != u and v not in adj[u]:
                partner = j
                break
        if partner is not None:
            v = left.pop(partner)
            add(u, v)
            continue
        # u holds the last free stub(s): trade an existing edge (c, d) for
        # (u, c) and (u, d); needs two free stubs on u.
        left.remove(u) if u in left else None
        while True:
            i = int(rng.integers(len(edges)))
            c, d = edges[i]
            if c >= n_int or d >= n_int or u in (c, d) or c in adj[u] or d in adj[u]:
                continue
            edges.pop(i)
            adj[c].discard(d)
            adj[d].discard(c)
            deg[c] -= 1
            deg[d] -= 1
            add(u, c)
            add(u, d)
            break
    del pending, cycle_edges
    return pts, np.array(edges, dtype=np.int64)


def config3(seed: int = 3) -> tuple[GraphDesc, dict]:
    """Synthetic stand-in for a cortical microvascular network (tracer
    transport, Sec. 4.2 of the paper): 20k vertices / 26k edges in a cube,
    degree 3 inside and 1 at the 4k boundary vertices; lengths lognormal
    (median 40 um, sigma_log 0.6); radii lognormal (median 4 um, sigma_log
    0.3); Poiseuille flow under random boundary pressures; drift = mean
    velocity Q/(pi r^2) scaled to a median speed of 1 mm/s; diffusivity
    1e-9 m^2/s; jump probabilities proportional to the cross-section pi r^2;
    inflow boundary vertices reflect, outflow ones absorb.  Units are
    made dimensionless with L0 = 40 um and T0 = L0^2 / D, so sigma = sqrt(2).
    dt is ten times the upwind finite-volume CFL limit with 64 cells per
    edge; 1e8 particles uniform by length, 1e4 steps, 64 bins per edge."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla

    rng = np.random.default_rng(seed)
    V, E, n_leaf = 20_000, 26_000, 4_000
    pts, edges = _vascular_topology(rng, V, E, n_leaf, side=1.2e-3)
    assert edges.shape[0] == E
    flip = rng.random(E) < 0.5
    ei = np.where(flip, edges[:, 1], edges[:, 0]).astype(np.int32)
    et = np.where(flip, edges[:, 0], edges[:, 1]).astype(np.int32)
    L0, D, eta = 40e-6, 1e-9, 3.5e-3
    T0 = L0 * L0 / D
    Lm = 40e-6 * np.exp(0.6 * rng.standard_normal(E))
    r = 4e-6 * np.exp(0.3 * rng.standard_normal(E))
    G = np.pi * r ** 4 / (8.0 * eta * Lm)
    deg = np.bincount(np.concatenate([ei, et]), minlength=V)
    leaf = deg == 1
    p = np.zeros(V)
    p[leaf] = rng.uniform(0.0, 1.0, size=int(leaf.sum()))
    # Kirchhoff: sum_e G_e (p_v - p_w) = 0 at internal vertices.
    lap = sp.coo_matrix((np.concatenate([G, G, -G, -G]),
                         (np.concatenate([ei, et, ei, et]),
                          np.concatenate([ei, et, et, ei]))), shape=(V, V)).tocsr()
    inner = np.flatnonzero(~leaf)
    bnd = np.flatnonzero(leaf)
    A = lap[inner][:, inner].tocsc()
    rhs = -(lap[inner][:, bnd] @ p[bnd])
    p[inner] = spla.spsolve(A, rhs)
    Q = G * (p[ei] - p[et])              # > 0: flow from init to term
    u = Q / (np.pi * r * r)
    u *= 1e-3 / np.median(np.abs(u))
    # boundary vertices: inflow (reflecting) or outflow (absorbing)
    kind = np.zeros(V, np.uint8)
    for lf in bnd:
        e = int(np.flatnonzero((ei == lf) | (et == lf))[0])
        out_flow = (ei[e] == lf and Q[e] < 0) or (et[e] == lf and Q[e] > 0)
        kind[lf] = 1 if out_flow else 0
    area = np.pi * r * r
    Lh = Lm / L0
    mu = u * T0 / L0
    sig = np.sqrt(2.0)
    dx = Lh / 64.0
    dt_cfl = np.min(1.0 / (np.abs(mu) / dx + 2.0 * (0.5 * sig * sig) / (dx * dx)))
    # inlets: inflow boundary vertices, with the inflow rate |Q| of their edge
    inlets, inflow = [], []
    for lf in bnd:
        if kind[lf] == 0:
            e = int(np.flatnonzero((ei == lf) | (et == lf))[0])
            inlets.append(int(lf))
            inflow.append(float(abs(Q[e])))
    g = from_edges(V, ei, et, Lh, mu, None, sig, weight_init=area,
                   weight_term=area, vtx_kind=kind,
                   meta={"name": "vascular20k", "T0": T0, "L0": L0,
                         "dt_cfl": float(dt_cfl), "inlets": np.array(inlets, np.int32),
                         "inflow": np.array(inflow)})
    run = dict(n_particles=100_000_000, init="uniform", dt=10.0 * float(dt_cfl),
               n_steps=10_000, max_splits=8, seed=0, bins=64)
    return g, run


def config4(seed: int = 4) -> tuple[list, list, dict]:
    """512 independent graphs of uneven size: even ids stars, odd ids random
    recursive trees; edges round(loguniform[3, 4096]); L ~ U[0.2, 3];
    particle counts loguniform[1e4, 1e6]; even graphs without drift, odd
    graphs with per-edge quadratic potentials (Langevin); sigma = sqrt(2);
    uniform jump probabilities; dt 1e-3, 1000 steps, 64 bins per edge."""
    rng = np.random.default_rng(seed)
    graphs, counts = [], []
    for gi in range(512):
        E = int(np.rint(np.exp(rng.uniform(np.log(3), np.log(4096)))))
        quad = gi % 2 == 1
        if gi % 4 < 2:
            L = rng.uniform(0.2, 3.0, size=E)
            a = c = None
            if quad:
                k = rng.uniform(0.5, 4.0, size=E)
                m = rng.uniform(0.0, 1.0, size=E) * L
                a, c = 2.0 * k * m, -2.0 * k
            g = star_graph(E, L, a, c, np.sqrt(2.0), meta={"name": f"batch{gi}"})
        else:
            g = random_tree(E, rng, quadratic=quad, meta={"name": f"batch{gi}"})
        graphs.append(g)
        counts.append(int(np.rint(np.exp(rng.uniform(np.log(1e4), np.log(1e6))))))
    run = dict(init="uniform", dt=1e-3, n_steps=1000, max_splits=8, seed=0,
               bins=64)
    return graphs, counts, run


def config5() -> tuple[list, list, dict]:
    """Accuracy sweep: config 3's network plus 128 config-2-style stars
    (seeds 5000..5127), advanced together as one batch at each dt in
    {1e-2, 3e-3, 1e-3, 3e-4} over a fixed horizon (stars T = 2, network
    T = 0.05 in its diffusive time unit); 1e8 particles on the network and
    1e8 split evenly over the stars per dt."""
    net, run3 = config3()
    stars = [config2(seed)[0] for seed in range(5000, 5128)]
    graphs = [net] + stars
    counts = [100_000_000] + [100_000_000 // 128] * 128
    run = dict(dts=(1e-2, 3e-3, 1e-3, 3e-4), horizons=[0.05] + [2.0] * 128,
               init="uniform", max_splits=8, seed=0, bins=[64] + [256] * 128)
    return graphs, counts, run
