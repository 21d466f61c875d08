"""The FP64 oracle against a 50-digit re-execution of the same paths.

The step (Alg. 2 with Alg. 1's vertex rule: EM move, interior test, crossing
root in the frame of the hit vertex, remaining time, slot draw) is replayed
in mpmath from the same Philox integers (the generator itself is pinned to
rocRAND elsewhere), with normals, drift, roots and times evaluated to 50
significant digits.  Over 1000 steps the FP64 oracle must take the same
vertex hits and slots and end within 1e-13 of the high-precision position:
FP64 rounding never flips a branch on these paths.  This checks the
oracle's floating-point faithfulness, not its formulas (those are pinned by
the closed forms)."""
import numpy as np
import pytest

import workloads

mp = pytest.importorskip("mpmath")


def _words(orc, p, c1, c2, seed, tag):
    return [int(v) for v in orc.philox(np.array([[p, c1, c2, tag]], np.uint32), seed)[0]]


def _normal_pair(a, b):
    u1 = (mp.mpf(a) + mp.mpf("0.5")) / mp.mpf(2) ** 32
    u2 = (mp.mpf(b) + mp.mpf("0.5")) / mp.mpf(2) ** 32
    r = mp.sqrt(-2 * mp.log(u1))
    return r * mp.cos(2 * mp.pi * u2), r * mp.sin(2 * mp.pi * u2)


def _root(A, B, C):
    """Smallest u in (0, 1] with C + B u + A u^2 = 0 (C >= 0), clamped."""
    if C == 0:
        if A == 0:
            return mp.mpf(0)
        u = -B / A
    elif A == 0:
        u = -C / B
    else:
        disc = max(B * B - 4 * A * C, mp.mpf(0))
        q = -(B + (1 if B >= 0 else -1) * mp.sqrt(disc)) / 2
        r = sorted([q / A, C / q])
        u = r[0] if r[0] > 0 else r[1]
        if not u > 0:
            u = mp.mpf(1)
    return min(max(u, mp.mpf(0)), mp.mpf(1))


def _replay(orc, g, thr, pid, e, x, n_steps, dt, seed, M=8, tag=0):
    """Returns (edge, x, [(step, slot), ...]) of one particle, 50 digits."""
    mp.mp.dps = 50
    L = [mp.mpf(float(v)) for v in g.length]
    a = [mp.mpf(float(v)) for v in g.drift_a]
    c = [mp.mpf(float(v)) for v in g.drift_c]
    sg = [mp.mpf(float(v)) for v in g.sigma]
    x = mp.mpf(float(x))
    hits = []
    normals = {}
    for n in range(n_steps):
        grp = n >> 2
        if grp not in normals:
            w = _words(orc, pid, grp, 0, seed, tag)
            normals = {grp: _normal_pair(w[0], w[1]) + _normal_pair(w[2], w[3])}
        W = normals[grp][n & 3]
        h = mp.mpf(dt)
        k = 0
        while True:
            if x == 0:
                W = abs(W)
            elif x == L[e]:
                W = -abs(W)
            mu = a[e] + c[e] * x
            gg = sg[e] * mp.sqrt(h)
            xt = x + mu * h + gg * W
            if 0 < xt < L[e]:
                x = xt
                break
            at_init = xt <= 0
            v = int(g.edge_init[e] if at_init else g.edge_term[e])
            d = x if at_init else L[e] - x
            s = 1 if at_init else -1
            u = _root(s * mu * h, s * gg * W, d)
            h = h - u * u * h
            k += 1
            if g.vtx_kind[v] == 1:
                return e, None, hits + [(n, -1 - v)]
            w = _words(orc, pid, n, k, seed, tag)
            s0, s1 = int(g.vtx_offsets[v]), int(g.vtx_offsets[v + 1])
            slot = next((j for j in range(s0, s1) if w[0] < int(thr[j])), s1 - 1)
            hits.append((n, slot))
            e = int(g.slot_edge[slot])
            x = L[e] if g.slot_orient[slot] else mp.mpf(0)
            if h < mp.mpf(10) ** -40 or k == M:
                break
            W = _normal_pair(w[1], w[2])[0]
    return e, x, hits


@pytest.mark.parametrize("case", ["config1", "paper_star_linear", "config2"])
def test_fp64_oracle_matches_50_digit_replay(orc, case):
    if case == "config1":
        g, mode, dt, kw = workloads.config1()[0], orc.INIT_AT_VERTEX, 1e-3, dict(vertex=0)
    elif case == "paper_star_linear":
        g, mode, dt, kw = workloads.paper_star5("linear"), orc.INIT_AT_VERTEX, 1e-3, dict(vertex=0)
    else:
        g, mode, dt, kw = workloads.config2()[0], orc.INIT_UNIFORM_LENGTH, 1e-2, {}
    thr = orc.thresholds(g)
    n_steps, seed = 1000, 21
    for pid in (3, 40):
        st = orc.init(g, 64, mode, seed=5, pids=np.array([pid]), **kw)
        e0, x0 = int(st.edge[0]), float(st.x[0])
        tr, _ = orc.simulate_traced(g, st, 0, 0, n_steps, dt, seed)
        e, x, hits = _replay(orc, g, thr, pid, e0, x0, n_steps, dt, seed)
        ours = list(zip(tr["step"].tolist(), tr["slot"].tolist()))
        want = [(s_, sl) for s_, sl in hits if sl >= 0]
        assert ours == want, (case, pid, len(ours), len(want))
        assert len(want) > 0
        assert int(st.edge[0]) == e
        assert abs(float(st.x[0]) - float(x)) <= 1e-13, (case, pid, float(st.x[0]) - float(x))
