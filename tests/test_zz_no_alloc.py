"""The allocation-free general histogram, mg_histogram_csr_noalloc, through
the C ABI, against mg_histogram_csr on the same particle sets.

Bar: identical integer counts (both run the same kernel over the same
states; only where the bin tables live differs).  Two calls in a row, the
second with smaller tables, so the workspace holds the first call's tables
and counters when the second starts; host and device outputs; tables
beyond the workspace rejected with MG_EINVAL and no device work.
"""
import ctypes as C

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

SCRATCH = 32 << 20


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_02175_amd import binding
    binding.lib()
    return binding


def _bins(g, rng, lo, hi):
    counts = rng.integers(lo, hi, size=g.n_edges)
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    up = np.concatenate([np.sort(rng.uniform(0, L, c - 1)).tolist() + [L]
                         for L, c in zip(g.length, counts)])
    return off, up


def test_noalloc_histogram_equals_allocating_one(B):
    import torch
    rng = np.random.default_rng(21)
    # first call: config 2's star, FP32, 1e5 particles, about 1.3e5 uneven
    # bins (global counters), host output
    g2, _ = workloads.config2()
    G2 = B.mg_graph_create(g2)
    p2 = B.mg_particles_init(G2, 100_000, 2, init_seed=3, precision=B.MG_FP32)
    B.mg_simulate(p2, 300, 1e-2, 4)
    off2, up2 = _bins(g2, rng, 1000, 3000)
    print(f"no-alloc histogram: call 1, {int(off2[-1])} bins", flush=True)
    want2 = B.mg_histogram_csr(p2, off2, up2)
    got2 = B.mg_histogram_csr_noalloc(p2, off2, up2)
    assert np.array_equal(got2, want2)
    assert int(got2.sum()) == 100_000
    # second call, smaller: config 1's three edges, FP64, 40 bins in all
    # (LDS counters); the workspace still holds call 1's tables and counts
    g1, _ = workloads.config1()
    G1 = B.mg_graph_create(g1)
    p1 = B.mg_particles_init(G1, 5000, 1, vertex=0, init_seed=5)
    B.mg_simulate(p1, 200, 1e-3, 6)
    off1, up1 = _bins(g1, rng, 5, 20)
    print(f"no-alloc histogram: call 2, {int(off1[-1])} bins", flush=True)
    want1 = B.mg_histogram_csr(p1, off1, up1)
    got1 = B.mg_histogram_csr_noalloc(p1, off1, up1)
    assert np.array_equal(got1, want1)
    assert int(got1.sum()) == 5000
    # device output, and call 1 again after call 2
    out = torch.full((int(off2[-1]),), 7, dtype=torch.int64, device="cuda")
    B.mg_histogram_csr_noalloc(p2, off2, up2, out)
    assert np.array_equal(out.cpu().numpy().astype(np.uint64), want2)
    assert np.array_equal(B.mg_histogram_csr_noalloc(p1, off1, up1), want1)


def test_noalloc_histogram_rejects_tables_beyond_the_workspace(B):
    g2, _ = workloads.config2()
    G2 = B.mg_graph_create(g2)
    p2 = B.mg_particles_init(G2, 1000, 2, init_seed=3, precision=B.MG_FP32)
    per_edge = SCRATCH // (16 * g2.n_edges) + 1        # host output: 16 B per bin
    off = (np.arange(g2.n_edges + 1) * per_edge).astype(np.int32)
    up = np.concatenate([np.linspace(L / per_edge, L, per_edge) for L in g2.length])
    out = np.zeros(int(off[-1]), np.uint64)
    print(f"no-alloc histogram: {int(off[-1])} bins, beyond the workspace", flush=True)
    rc = B.lib().mg_histogram_csr_noalloc(p2.handle, off.ctypes.data_as(C.c_void_p),
                                          up.ctypes.data_as(C.c_void_p),
                                          out.ctypes.data_as(C.c_void_p), out.size)
    assert rc == B.MG_EINVAL
    assert "workspace" in B.mg_last_error()
    # the allocating entry point takes the same tables
    h = B.mg_histogram_csr(p2, off, up)
    assert int(h.sum()) == 1000
