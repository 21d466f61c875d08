"""Checkpoint and resume through the C ABI: a set saved after k steps and
loaded again (on the same graph object or one rebuilt from the same
description, under another schedule) continues bit for bit as the set that
was never stopped: states, hashes, hit counts, counters, histograms and the
streamed histogram.  Bad images are refused on the host before anything is
created."""
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


def _state(B, p, bins=16):
    r = B.mg_particles_read(p, trace=True)
    ex, ab, tot = B.mg_exit_counts(p)
    return dict(r, ex=ex, ab=ab, tot=tot, hist=B.mg_histogram(p, bins),
                step=B.mg_particles_step(p))


def _assert_same(a, b):
    for k in a:
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k


def _absorbing_star():
    # leaves 1 and 3 absorb, the drift pushes outward on two edges
    g = workloads.star_graph(5, [0.6, 1.0, 0.8, 1.2, 0.5], drift_a=[2.0, -1.0, 1.0, 0.0, -3.0],
                             drift_c=[-1.0, 0.5, 0.0, 0.0, 1.0], sigma=1.0)
    g.vtx_kind[1] = 1
    g.vtx_kind[3] = 1
    return g


CASES = {
    "langevin64": lambda: workloads.config2()[0],
    "absorbing": _absorbing_star,
    "wentzell": lambda: workloads.wentzell_star(5, seed=7),
}


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("case", sorted(CASES))
def test_resume_equals_straight_run(B, case, prec):
    """300 steps, save, destroy, load, 200 steps == 500 steps straight (the
    resumed set runs the lane schedule, the others wave pools)."""
    g = CASES[case]()
    G = B.mg_graph_create(g)
    dt, seed, n = 1e-2, 11, 3001
    kw = dict(init_seed=5, precision=prec, max_splits=8, graph_tag=3, trace=True,
              schedule=B.MG_SCHED_POOLS_W8)
    ref = B.mg_particles_init(G, n, 2, **kw)
    B.mg_simulate(ref, 500, dt, seed)
    want = _state(B, ref)

    p = B.mg_particles_init(G, n, 2, **kw)
    B.mg_simulate(p, 300, dt, seed)
    img = B.mg_particles_save(p)
    assert img.size == B.mg_particles_image_bytes(p)
    hd = B.image_header(img)
    assert (hd.magic, hd.version, hd.step, hd.n, hd.precision, hd.graph_tag, hd.trace) == \
        (b"MGSETIMG", 1, 300, n, prec, 3, 1)
    mid = _state(B, p)
    del p

    q = B.mg_particles_load(G, img, schedule=B.MG_SCHED_LANES)
    _assert_same(_state(B, q), mid)            # the image holds the whole state
    assert np.array_equal(B.mg_particles_save(q), img)
    B.mg_simulate(q, 200, dt, seed)
    _assert_same(_state(B, q), want)

    # a graph rebuilt from the same description takes the image too
    G2 = B.mg_graph_create(g)
    q2 = B.mg_particles_load(G2, img)
    B.mg_simulate(q2, 120, dt, seed)
    B.mg_simulate(q2, 80, dt, seed)
    _assert_same(_state(B, q2), want)


def test_resume_keeps_the_streamed_histogram(B):
    g, _ = workloads.config2()
    G = B.mg_graph_create(g)
    dt, seed = 1e-2, 3
    ref = B.mg_particles_init(G, 4000, 2, init_seed=1, precision=1)
    B.mg_simulate(ref, 40, dt, seed)
    B.mg_observe_histogram(ref, 12, 7)
    B.mg_simulate(ref, 460, dt, seed)
    want, want_ns = B.mg_observed_histogram(ref)

    p = B.mg_particles_init(G, 4000, 2, init_seed=1, precision=1)
    B.mg_simulate(p, 40, dt, seed)
    B.mg_observe_histogram(p, 12, 7)
    B.mg_simulate(p, 250, dt, seed)
    img = B.mg_particles_save(p)
    hd = B.image_header(img)
    assert (hd.obs_bins, hd.obs_every, hd.obs_start, hd.step) == (12, 7, 40, 290)
    q = B.mg_particles_load(G, img)
    B.mg_simulate(q, 210, dt, seed)
    got, ns = B.mg_observed_histogram(q)
    assert ns == want_ns == 500 // 7 - 40 // 7
    assert np.array_equal(got, want)
    assert np.array_equal(B.mg_histogram(q, 12), B.mg_histogram(ref, 12))


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_members_resume(B, prec):
    """Members of a batch saved after 300 batched steps, loaded (one into a
    torch arena) and batched again for 200: equal to 500 steps of each set
    alone."""
    rng = np.random.default_rng(4)
    graphs = [workloads.star_graph(3, [1.0, 2.0, 0.5]), workloads.random_tree(40, rng),
              workloads.config2()[0]]
    counts = [700, 2000, 5000]
    Gs = [B.mg_graph_create(g) for g in graphs]
    alone, members = [], []
    for i, (G, n) in enumerate(zip(Gs, counts)):
        kw = dict(init_seed=i, precision=prec, graph_tag=i, trace=True)
        alone.append(B.mg_particles_init(G, n, 2, **kw))
        members.append(B.mg_particles_init(G, n, 2, **kw))
    for p in alone:
        B.mg_simulate(p, 500, 1e-2, 9)
    b = B.mg_batch_create(members)
    B.mg_batch_simulate(b, 300, 1e-2, 9)
    imgs = [B.mg_particles_save(p) for p in members]
    del b, members
    loaded = [B.mg_particles_load(G, img, arena="torch" if i == 1 else None)
              for i, (G, img) in enumerate(zip(Gs, imgs))]
    b2 = B.mg_batch_create(loaded)
    B.mg_batch_simulate(b2, 200, 1e-2, 9)
    for pa, pb in zip(alone, loaded):
        _assert_same(_state(B, pb), _state(B, pa))


def _image(B, prec=0, n=257):
    g, _ = workloads.config2()
    G = B.mg_graph_create(g)
    p = B.mg_particles_init(G, n, 2, init_seed=2, precision=prec, trace=True)
    B.mg_simulate(p, 20, 1e-2, 1)
    return g, G, B.mg_particles_save(p)


def _refused(B, G, img, msg):
    with pytest.raises(B.MgError) as ei:
        B.mg_particles_load(G, img)
    assert ei.value.status == B.MG_EINVAL
    assert msg in str(ei.value), str(ei.value)


def test_bad_images_refused(B):
    g, G, img = _image(B)
    off = {f[0]: getattr(B.mg_image_header, f[0]).offset for f in B.mg_image_header._fields_}
    ef0 = 96                         # the state words follow the header
    pos0 = ef0 + ((257 * 4 + 7) // 8) * 8

    _refused(B, G, img[:95], "shorter than its header")
    _refused(B, G, img[:-8], "expected")
    bad = img.copy(); bad[0] ^= 1
    _refused(B, G, bad, "not a particle-set image")
    bad = img.copy(); bad[off["version"]] = 2
    _refused(B, G, bad, "version")
    other = B.mg_graph_create(workloads.config1()[0])
    _refused(B, other, img, "another graph")
    # a graph of the same shape with other coefficients
    g2, _ = workloads.config2(seed=5)
    _refused(B, B.mg_graph_create(g2), img, "another graph")
    bad = img.copy(); bad[ef0 + 4 * 5: ef0 + 4 * 6] = np.frombuffer(
        np.uint32(g.n_edges).tobytes(), np.uint8)
    _refused(B, G, bad, "particle 5: edge out of range")
    bad = img.copy(); bad[ef0 + 4 * 6 + 3] |= 0x40         # FP32 flag in FP64
    _refused(B, G, bad, "particle 6: FP32 reference-end flag")
    bad = img.copy(); bad[pos0 + 8 * 7: pos0 + 8 * 8] = np.frombuffer(
        np.float64(np.nan).tobytes(), np.uint8)
    _refused(B, G, bad, "particle 7: position outside its edge")
    bad = img.copy(); bad[pos0 + 8 * 8: pos0 + 8 * 9] = np.frombuffer(
        np.float64(-1e-3).tobytes(), np.uint8)
    _refused(B, G, bad, "particle 8: position outside its edge")
    bad = img.copy(); bad[off["max_splits"]] = 0
    _refused(B, G, bad, "header out of range")
    bad = img.copy(); bad[off["obs_every"]] = 5     # on, with 0 bins
    _refused(B, G, bad, "streamed-histogram")

    # FP32 image: a negative distance is refused where the end is not a
    # Wentzell vertex; an unchanged image loads
    g, G, img = _image(B, prec=1)
    bad = img.copy(); bad[pos0 + 8 * 3: pos0 + 8 * 3 + 4] = np.frombuffer(
        np.float32(-0.25).tobytes(), np.uint8)
    _refused(B, G, bad, "particle 3: position outside its edge")
    assert B.mg_particles_step(B.mg_particles_load(G, img)) == 20


def test_save_arguments_checked(B):
    import ctypes as C
    import torch
    g, G, img = _image(B)
    p = B.mg_particles_load(G, img)
    L = B.lib()
    need = B.mg_particles_image_bytes(p)
    buf = np.zeros(need, np.uint8)
    assert L.mg_particles_save(p.handle, B._p(buf), need - 1) == B.MG_EINVAL
    dev = torch.zeros(need, dtype=torch.uint8, device="cuda")
    assert L.mg_particles_save(p.handle, C.c_void_p(dev.data_ptr()), need) == B.MG_EINVAL
    assert "host memory" in B.mg_last_error()
    assert L.mg_particles_save(p.handle, B._p(buf), need) == B.MG_OK
    assert np.array_equal(buf, img)
