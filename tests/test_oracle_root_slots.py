"""Pins of the crossing-time solver and of the slot draw.

Crossing time: the oracle's u must be the smallest root in (0, 1] of
C + B u + A u^2 (C >= 0), checked against 60-digit roots from mpmath.
Slot draw: over all 2^32 values of the 32-bit draw, slot s must be chosen
for exactly T_s - T_{s-1} of them, within one draw of b_s 2^32, and a slot
with b = 0 never.
"""
import mpmath as mp
import numpy as np

import workloads


def _smallest_root_mp(A, B, C):
    mp.mp.dps = 60
    A, B, C = mp.mpf(A), mp.mpf(B), mp.mpf(C)
    if A == 0:
        roots = [-C / B] if B != 0 else []
    else:
        disc = B * B - 4 * A * C
        if disc < 0:
            disc = mp.mpf(0)
        s = mp.sqrt(disc)
        roots = [(-B - s) / (2 * A), (-B + s) / (2 * A)]
    good = [r for r in roots if 0 < r <= 1]
    return min(good) if good else None


def test_root_random_well_conditioned(orc):
    rng = np.random.default_rng(5)
    n = 4000
    ustar = rng.uniform(0.01, 1.0, n)
    A = rng.normal(0, 1, n) * 10.0 ** rng.uniform(-3, 1, n)
    Cc = rng.uniform(0, 1, n) * 10.0 ** rng.uniform(-4, 0, n)
    B = -(Cc + A * ustar ** 2) / ustar      # u* is a root
    u = orc.first_root(A, B, Cc)
    bad = 0
    for i in range(n):
        r = _smallest_root_mp(A[i], B[i], Cc[i])
        assert r is not None
        # the quadratic's condition number at the root bounds the error
        deriv = abs(B[i] + 2 * A[i] * float(r))
        scale = abs(Cc[i]) + abs(B[i]) * float(r) + abs(A[i]) * float(r) ** 2
        tol = 8e-16 * scale / max(deriv, 1e-300) + 4e-16 * float(r)
        if abs(u[i] - float(r)) > max(tol, 1e-15):
            bad += 1
    assert bad == 0


def test_root_at_vertex_and_edge_cases(orc):
    # C == 0: roots 0 and -B/A; the crossing is the nonzero one
    A = np.array([-2.0, -1e-8, -3.0, 0.0, -1.0])
    B = np.array([1.0, 1e-9, 0.0, 0.0, 1.0])
    Cc = np.zeros(5)
    u = orc.first_root(A, B, Cc)
    np.testing.assert_allclose(u[:2], [0.5, 0.1], rtol=1e-15)
    assert u[2] == 0.0 and u[3] == 0.0
    assert u[4] == 1.0
    # A == 0: linear case u = -C/B
    u = orc.first_root(np.zeros(3), np.array([-2.0, -1.0, -0.5]), np.array([1.0, 1.0, 0.25]))
    np.testing.assert_allclose(u, [0.5, 1.0, 0.5], rtol=1e-15)
    # two roots inside (0, 1]: the first crossing is the smaller one
    # (u - 0.2)(u - 0.8) = u^2 - u + 0.16
    u = orc.first_root(np.array([1.0]), np.array([-1.0]), np.array([0.16]))
    np.testing.assert_allclose(u, [0.2], rtol=1e-14)
    # tiny distance to the vertex: relative accuracy of the small root
    u = orc.first_root(np.array([0.3]), np.array([-2.0]), np.array([1e-200]))
    np.testing.assert_allclose(u, [0.5e-200], rtol=1e-14)
    # double root at the tangency, disc rounded below zero is clamped
    u = orc.first_root(np.array([1.0]), np.array([-1.0]), np.array([0.25]))
    np.testing.assert_allclose(u, [0.5], rtol=1e-7)


def test_root_never_outside_unit_interval(orc):
    rng = np.random.default_rng(7)
    n = 100000
    A = rng.normal(size=n) * 10.0 ** rng.uniform(-8, 3, n)
    B = -np.abs(rng.normal(size=n)) * 10.0 ** rng.uniform(-8, 3, n)
    Cc = np.abs(rng.normal(size=n)) * 10.0 ** rng.uniform(-8, 0, n)
    u = orc.first_root(A, B, Cc)
    assert np.all((u >= 0) & (u <= 1)) and np.all(np.isfinite(u))


def _slot_counts(thr, offsets, v):
    s0, s1 = offsets[v], offsets[v + 1]
    t = np.concatenate([[0], np.minimum(thr[s0:s1].astype(np.float64), 2.0**32)])
    t[-1] = 2.0**32        # the last slot takes every remaining draw
    return np.diff(t)


def test_slot_thresholds_exact_counts(orc):
    rng = np.random.default_rng(1)
    for trial in range(50):
        deg = int(rng.integers(1, 9))
        w = rng.uniform(0, 1, deg) * (rng.random(deg) < 0.7)
        if w.sum() == 0:
            w[0] = 1.0
        g = workloads.star_graph(deg, 1.0, b_center=w)
        thr = orc.thresholds(g)
        counts = _slot_counts(thr, g.vtx_offsets, 0)
        b = g.slot_jump_prob[: deg]
        assert np.all(counts >= 0)
        assert counts.sum() == 2.0**32
        assert np.all(np.abs(counts - b * 2.0**32) <= 1.0 + deg)
        assert np.all(counts[b == 0] == 0)
        # leaves: a single slot takes every draw
        for v in range(1, deg + 1):
            assert thr[g.vtx_offsets[v]] == 2**32


def test_slot_draw_frequencies_in_simulation(orc):
    """Zero-probability slots are never drawn and the drawn slots follow b."""
    b = np.array([0.0, 0.5, 0.0, 0.3, 0.2, 0.0])
    g = workloads.star_graph(6, 1.0, b_center=b)
    st = orc.init(g, 200_000, orc.INIT_AT_VERTEX, vertex=0, seed=3)
    counts = np.bincount(st.edge, minlength=6)
    assert np.all(counts[b == 0] == 0)
    c = orc.simulate(g, st, 0, 50, 1e-3, 8)
    ex = c.exit_slot[:6]
    assert np.all(ex[b == 0] == 0)
    frac = ex / ex.sum()
    np.testing.assert_allclose(frac[b > 0], b[b > 0], atol=5 * np.sqrt(0.25 / ex.sum()))
