"""GPU counters over long persistent launches, through the C ABI.

A persistent wave-pool block serves any number of particles in one launch,
so its 32-bit lane tallies and u32 LDS exit and snapshot counters are drained
into 64-bit ones every few hundred iterations of the pool loop, and the
block's totals are 64-bit.  Bars: exact integers.  A single launch whose
per-block step count exceeds 2^32 gives the same totals, exit counts and
histogram as the same run cut into short launches (whose per-block counts
stay far below 2^32), and totals[3] is exactly n * steps; draining after
every iteration gives the same counts as the default.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_02175_amd import binding
    binding.lib()
    return binding


def _state(B, p):
    r = B.mg_particles_read(p, trace=True)
    ex, ab, tot = B.mg_exit_counts(p)
    return r, ex, ab, tot


def test_long_persistent_launch_counts_exact(B):
    """Config 2's star, 2^24 FP32 particles, 6e5 steps at dt = 1e-2 in one
    launch: each of the at most 2048 resident blocks takes more than 2^32
    particle-steps (8192 x 6e5 = 4.9e9).  Against the same run in launches
    of 5000 steps."""
    g, run = workloads.config2()
    G = B.mg_graph_create(g)
    n, steps, dt = 2**24, 600_000, 1e-2
    res = []
    for spl in (0, 5000):
        print(f"long launch: n={n} steps={steps} steps_per_launch={spl}", flush=True)
        p = B.mg_particles_init(G, n, 2, init_seed=1, precision=B.MG_FP32, trace=True,
                                schedule=B.MG_SCHED_POOLS_W8, steps_per_launch=spl)
        B.mg_simulate(p, steps, dt, 5)
        r, ex, ab, tot = _state(B, p)
        h = B.mg_histogram(p, run["bins"])
        assert int(tot[3]) == n * steps
        assert int(tot[2]) == int(r["hits"].astype(np.int64).sum())
        assert int(tot[1]) > int(tot[3]) and int(ab.sum()) == 0 and int(tot[0]) == 0
        assert int(h.sum()) == n
        # every step with a hit records one exit, so there are at most as many
        # exits as hits, and a long run has very many
        assert 0 < int(ex.sum()) <= int(tot[2])
        res.append((r, ex, tot, h))
        del p
    (ra, exa, ta, ha), (rb, exb, tb, hb) = res
    for f in ("edge", "x", "alive", "seqhash", "hits"):
        assert np.array_equal(ra[f], rb[f]), f
    assert np.array_equal(exa, exb)
    assert np.array_equal(ta, tb)
    assert np.array_equal(ha, hb)


@pytest.mark.parametrize("kind", ["single", "batch"])
def test_pool_drain_every_iteration_same_counts(B, monkeypatch, kind):
    """Draining the lane tallies and the LDS exit and snapshot counters after
    every pool iteration (MG_POOL_DRAIN=1) gives the same counts as the
    default drain period, single set (persistent grid) and batched, with
    LDS exit counters, LDS snapshot bins (64 edges x 64 bins) and absorbing
    vertices."""
    star = workloads.star_graph(5, [0.3, 0.5, 0.2, 0.8, 0.4], [-30.0, 5.0, -60.0, 0.0, -10.0],
                                [0, -2.0, 0, 0, 0], 1.0, b_center=[0.3, 0.1, 0.3, 0.2, 0.1])
    star.vtx_kind[2] = 1
    graphs = [workloads.config2()[0], star]
    Gs = [B.mg_graph_create(g) for g in graphs]
    counts = [60_000, 9_000]
    out = []
    for drain in ("1", ""):
        monkeypatch.setenv("MG_POOL_DRAIN", drain)
        sets = []
        for i, (G, c) in enumerate(zip(Gs, counts)):
            p = B.mg_particles_init(G, c, 2, init_seed=i, precision=B.MG_FP32, trace=True,
                                    graph_tag=i, max_splits=3, schedule=B.MG_SCHED_POOLS_W8)
            B.mg_observe_histogram(p, 64, 3)
            sets.append(p)
        if kind == "batch":
            b = B.mg_batch_create(sets)
            B.mg_batch_simulate(b, 700, 5e-3, 3)
            B.mg_batch_simulate(b, 301, 5e-3, 3)
        else:
            for p in sets:
                B.mg_simulate(p, 700, 5e-3, 3)
                B.mg_simulate(p, 301, 5e-3, 3)
        out.append([(_state(B, p), B.mg_observed_histogram(p)) for p in sets])
    for (sa, oa), (sb, ob) in zip(*out):
        ra, rb = sa[0], sb[0]
        for f in ("edge", "x", "alive", "seqhash", "hits"):
            assert np.array_equal(ra[f], rb[f]), f
        for x, y in zip(sa[1:], sb[1:]):
            assert np.array_equal(x, y)
        assert oa[1] == ob[1] and np.array_equal(oa[0], ob[0])
    # the absorbing star lost particles and the snapshots saw it
    (s_star, o_star) = out[0][1]
    assert int(s_star[2].sum()) > 0 and int(s_star[3][0]) > 0


@pytest.mark.parametrize("prec", [0, 1])
def test_repeated_runs_bitwise(B, prec):
    """The same run twice on fresh sets (wave pools whose particle-to-wave
    assignment follows the atomic claims, LDS exit counters, a streamed
    histogram, the event trace) gives the same states, counts,
    histograms and events: every device atomic is an integer add, so no
    result depends on the order in which the waves reach them."""
    # FP32 on the vascular network (absorbing outlets), FP64 on config 2's star
    g, run = workloads.config3() if prec == 1 else workloads.config2()
    dt = run["dt"] if prec == 1 else 1e-2
    G = B.mg_graph_create(g)
    out = []
    for _ in range(2):
        p = B.mg_particles_init(G, 200_003, 2, init_seed=4, precision=prec, trace=True,
                                schedule=B.MG_SCHED_POOLS_W8)
        B.mg_observe_histogram(p, 8, 3)
        B.mg_trace_events(p, [0, 17, 99_999, 200_002])
        B.mg_simulate(p, 400, dt, 5)
        r, ex, ab, tot = _state(B, p)
        obs, ns = B.mg_observed_histogram(p)
        out.append((r, ex, ab, tot, B.mg_histogram(p, 16), obs, ns, B.mg_trace_read(p)[0]))
    a, b = out
    for f in ("edge", "x", "alive", "seqhash", "hits"):
        assert np.array_equal(a[0][f], b[0][f]), f
    for x, y in zip(a[1:], b[1:]):
        assert np.array_equal(np.asarray(x), np.asarray(y))
