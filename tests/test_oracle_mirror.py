"""Pins of the oracle's mirror vertices: leaves that reflect a proposal
leaving the edge through them by its mirror image (the far-end reflection of
the paper's star-graph kernel in the appendix), against what the mathematics fixes."""
import numpy as np
import pytest
from scipy import stats

import workloads
from workloads import stationary


def _folded_cdf(x, m, s, L):
    """CDF on [0, L] of a N(m, s^2) point reflected once at 0 and once at L
    (the images of mass beyond -L or 2L are neglected: below 1e-30 here)."""
    F = stats.norm.cdf
    return ((F((x - m) / s) - F(-m / s)) + (F(-m / s) - F((-x - m) / s))
            + (F((2 * L - m) / s) - F((2 * L - x - m) / s)))


@pytest.mark.parametrize("a,x0", [(-8.0, 0.05), (6.0, 0.9), (0.0, 0.02), (0.0, 0.97)])
def test_one_step_is_the_folded_normal(orc, a, x0):
    """On a segment with mirror ends, one step from x0 with frozen
    coefficients is x0 + a dt + sigma sqrt(dt) Z folded into [0, L]: the
    folded normal law exactly, with no vertex hit and no exit record.  (A
    split at a plain leaf gives a different law under strong drift into the
    vertex, where it bounces up to M times.)"""
    L, sig, dt, N = 1.0, 0.5, 0.04, 200_000
    g = workloads.segment(L, a, 0.0, sig, end_kind=2)
    st = orc.init(g, N, orc.INIT_EXPLICIT, edge=np.zeros(N), pos=np.full(N, x0))
    c = orc.simulate(g, st, 0, 1, dt, 5)
    assert c.hits == 0 and c.exit_slot.sum() == 0 and c.truncations == 0
    assert np.all((st.x > 0.0) & (st.x < L))
    ks = stats.kstest(st.x, lambda x: _folded_cdf(x, x0 + a * dt, sig * np.sqrt(dt), L))
    assert ks.pvalue > 1e-4, ks


def test_image_outside_the_edge_splits(orc):
    """A proposal whose mirror image lies outside the edge (a move longer
    than the edge) is not mirrored: the sub-step splits at the leaf.  On a
    short segment, particle by particle from the exposed main normals: an
    image inside gives that image and no hit; an image outside gives at
    least one hit."""
    L, sig, dt, N, x0 = 0.05, 1.0, 0.01, 4000, 0.02
    g = workloads.segment(L, 0.0, 0.0, sig, end_kind=2)
    st = orc.init(g, N, orc.INIT_EXPLICIT, edge=np.zeros(N), pos=np.full(N, x0))
    seed = 9
    w = orc.main_normals(st.pid, np.zeros(N, np.uint64), seed)
    xt = x0 + sig * np.sqrt(dt) * w
    img = np.where(xt <= 0.0, -xt, np.where(xt >= L, 2 * L - xt, xt))
    inside = (img > 0.0) & (img < L)
    orc.simulate(g, st, 0, 1, dt, seed)
    outside_edge = (xt <= 0.0) | (xt >= L)
    mirrored = outside_edge & inside
    assert mirrored.sum() > 200 and (~inside).sum() > 200
    # (the oracle forms the proposal with fused multiply-adds)
    np.testing.assert_allclose(st.x[mirrored], img[mirrored], rtol=1e-12, atol=1e-15)
    assert np.all(st.hits[mirrored] == 0)
    assert np.all(st.hits[~inside] >= 1)
    np.testing.assert_allclose(st.x[~outside_edge], xt[~outside_edge], rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("case", ["quadratic", "brownian"])
def test_mirror_star_stationary_law(orc, case):
    """Stars with mirror leaves keep the stationary law of reflecting
    leaves: the paper's quadratic 5-edge star truncated at length 2 (the
    closed form restricted to [0, 2] and renormalised), and Brownian motion
    on a 3-edge star of lengths 0.5, 1, 1.5 with uniform jump probabilities
    (uniform by length), where the leaves are reached all the time.
    Time-averaged bin masses within the Monte-Carlo and time-step error
    (total variation); no exit record at the leaves."""
    if case == "quadratic":
        g = workloads.paper_star5("quadratic", length=2.0, leaf_kind=2)
        off, up, tu = workloads.csr_bins(g, 0.05, 40)
        exact = stationary.star_csr_masses(g, off, tu)
    else:
        g = workloads.star_graph(3, [0.5, 1.0, 1.5], sigma=1.0, leaf_kind=2)
        off, up, tu = workloads.csr_bins(g, 0.05, 30)
        lo = np.concatenate([np.concatenate([[0.0], tu[off[e]:off[e + 1] - 1]])
                             for e in range(3)])
        exact = (tu - lo) / 3.0
    assert abs(exact.sum() - 1.0) < 1e-12
    N, dt = 20_000, 1e-3
    if case == "quadratic":
        st = orc.init(g, N, orc.INIT_AT_VERTEX, vertex=0, seed=3)
    else:  # already the stationary law
        st = orc.init(g, N, orc.INIT_UNIFORM_LENGTH, seed=3)
    c = orc.simulate(g, st, 0, 1500, dt, 11)
    acc = np.zeros(off[-1])
    n0 = 1500
    for _ in range(6):
        orc.simulate(g, st, n0, 200, dt, 11, counts=c)
        n0 += 200
        acc += orc.histogram_csr(g, st, off, up).astype(np.float64)
    emp = acc / acc.sum()
    tv = 0.5 * np.abs(emp - exact).sum()
    assert tv < 0.03, tv
    leaves = [s for s in range(g.nnz) if g.slot_orient[s] == 1]
    assert c.exit_slot[leaves].sum() == 0
    assert c.exit_slot.sum() > 0


def test_mirror_vertex_must_be_a_leaf(orc):
    g = workloads.star_graph(3, 1.0)
    g.vtx_kind[0] = 2  # the centre has three slots
    with pytest.raises(ValueError, match="leaf"):
        orc.init(g, 4, orc.INIT_AT_VERTEX, vertex=1, seed=0)
