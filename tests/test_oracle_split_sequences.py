"""Brute-force pin of multi-split steps: the exact law of the sequence of
slots a particle draws within one step, for sequences of up to three vertex
hits, against one-step oracle trials.

A particle on the centre of a star (edge drawn from b, constant drift c_e
towards the vertex, edges too long to reach the far end) proposes, on edge
e with remaining time h, the move -c_e h + sigma sqrt(h) |W|.  It stays in
the edge with probability q_e(h) = 2 (1 - Phi(c_e sqrt(h) / sigma));
otherwise the crossing root is u = sigma |W| / (c_e sqrt(h)), the sub-step
consumes u^2 h = sigma^2 W^2 / c_e^2, and a new edge is drawn from b
(Alg. 2 with Alg. 1's fold at the vertex).  So, with w the half-normal
|W| of each returning sub-step,
    P(slots s1..sk, then inside) = sum_e0 b_e0 b_s1 .. b_sk
        E[ 1{returns on e0, s1, .., s(k-1)} q_sk(h - consumed) ],
a k-fold integral over the w's, evaluated by Gauss-Legendre quadrature in
w (the integrand is smooth there).  The oracle's per-particle hash of
(step, slot) words identifies each particle's sequence."""
import itertools

import numpy as np
from scipy import stats

import workloads

B_ = np.array([0.5, 0.3, 0.2])
C_ = np.array([10.0, 20.0, 30.0])
SIG = np.sqrt(2.0)


def _q(e, h):
    return 2.0 * stats.norm.sf(C_[e] * np.sqrt(np.maximum(h, 0.0)) / SIG)


def _seq_probs(dt, kmax=3, n_gl=48):
    """Exact probabilities of the hit-slot sequences of length 0..kmax."""
    tg, wg = np.polynomial.legendre.leggauss(n_gl)

    def expect(edges, h):
        """E over the half-normal w of each return on edges[:-1] (each must
        fit in the time left) of q_{edges[-1]}(time left); h is an array of
        starting times, vectorised."""
        if len(edges) == 1:
            return _q(edges[0], h)
        e = edges[0]
        wmax = C_[e] * np.sqrt(h) / SIG               # return iff w <= wmax
        w = 0.5 * wmax[..., None] * (tg + 1.0)         # [.., n_gl]
        ww = 0.5 * wmax[..., None] * wg
        rest = h[..., None] - (SIG * w / C_[e]) ** 2
        inner = expect(edges[1:], rest)
        return np.sum(ww * 2.0 * stats.norm.pdf(w) * inner, axis=-1)

    probs = {(): float(np.sum(B_ * np.array([_q(e, dt) for e in range(3)])))}
    for k in range(1, kmax + 1):
        for seq in itertools.product(range(3), repeat=k):
            p = 0.0
            for e0 in range(3):
                p += B_[e0] * np.prod(B_[list(seq)]) * float(
                    expect([e0, *seq], np.array(dt)))
            probs[seq] = p
    return probs


def _fnv(words):
    h = 0xcbf29ce484222325
    for w in words:
        h = ((h ^ w) * 0x100000001b3) & 0xFFFFFFFFFFFFFFFF
    return h


def test_split_sequences_match_exact_law(orc):
    dt, N = 2e-3, 2_000_000
    probs = _seq_probs(dt)
    assert 0.99 < sum(probs.values()) <= 1.0
    g = workloads.star_graph(3, 10.0, -C_, None, SIG, b_center=B_)
    st = orc.init(g, N, orc.INIT_AT_VERTEX, vertex=0, seed=3)
    orc.simulate(g, st, 0, 1, dt, 17, max_splits=64)
    slot_of_edge = {int(g.slot_edge[s]): s for s in range(g.vtx_offsets[0], g.vtx_offsets[1])}
    code = {}
    for seq in probs:
        words = []
        for e in seq:
            words += [0, slot_of_edge[e]]
        code[_fnv(words)] = seq
    keys, cnt = np.unique(st.seqhash, return_counts=True)
    obs = {seq: 0 for seq in probs}
    other = 0
    for k, n in zip(keys.tolist(), cnt.tolist()):
        if k in code:
            obs[code[k]] += n
        else:
            other += n
    exp = np.array([probs[s] * N for s in probs] + [(1.0 - sum(probs.values())) * N])
    o = np.array([obs[s] for s in probs] + [other], np.float64)
    m = exp > 20
    chi = float(((o[m] - exp[m]) ** 2 / exp[m]).sum())
    assert stats.chi2.sf(chi, int(m.sum()) - 1) > 1e-4, (chi, int(m.sum()))
    # the multi-hit classes carry real weight: the test sees them
    assert sum(probs[s] for s in probs if len(s) >= 2) > 0.05
