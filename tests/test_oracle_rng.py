"""Pins of the oracle's random numbers.

* Philox4x32-10 against rocRAND's host-callable engine (an independent
  implementation of the SC'11 generator), built from the installed headers.
* Box-Muller normals of the main and hit streams against the standard normal
  law (Kolmogorov-Smirnov, moments) and against each other (independence).
* Slot/position bits against the uniform law.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))
ROCRAND_HDR = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"


@pytest.fixture(scope="module")
def rocrand_philox():
    if not os.path.exists(ROCRAND_HDR) or shutil.which("g++") is None:
        pytest.skip("rocRAND headers or g++ not available")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "rr")
    subprocess.run(["g++", "-O1", "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__",
                    os.path.join(HERE, "helpers", "rocrand_philox.cpp"), "-o", exe],
                   check=True, capture_output=True)

    def run(keys, ctrs):
        lines = "".join("%x %x %x %x %x %x\n" % (k[0], k[1], c[0], c[1], c[2], c[3])
                        for k, c in zip(keys, ctrs))
        out = subprocess.run([exe], input=lines, capture_output=True, text=True,
                             check=True).stdout.split()
        return np.array([int(w, 16) for w in out], dtype=np.uint64).reshape(-1, 4)

    yield run
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_rocrand(orc, rocrand_philox):
    rng = np.random.default_rng(11)
    n = 3000
    keys = rng.integers(0, 2**32, size=(n, 2), dtype=np.uint64)
    ctrs = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64)
    ctrs[:, 1] %= 2**30          # rocRAND's offset argument is 4*(c1:c0)
    specials = [((0, 0), (0, 0, 0, 0)), ((0xFFFFFFFF, 0xFFFFFFFF), (0xFFFFFFFF, 2**30 - 1, 0xFFFFFFFF, 0xFFFFFFFF)),
                ((1, 0), (0, 0, 0, 0)), ((0, 0), (1, 0, 0, 0)), ((0, 0), (0, 0, 1, 0)),
                ((0, 0), (0, 0, 0, 1)), ((0, 1), (0, 1, 0, 0))]
    for k, c in specials:
        keys = np.vstack([keys, np.array(k, np.uint64)])
        ctrs = np.vstack([ctrs, np.array(c, np.uint64)])
    ref = rocrand_philox(keys.tolist(), ctrs.tolist())
    got = np.vstack([orc.philox(c[None, :].astype(np.uint32), int(k[0]) | (int(k[1]) << 32))
                     for k, c in zip(keys, ctrs)])
    assert np.array_equal(got.astype(np.uint64), ref)


def test_philox_bytes_uniform(orc):
    n = 1 << 16
    ctr = np.zeros((n, 4), np.uint32)
    ctr[:, 0] = np.arange(n)
    ctr[:, 1] = 7
    out = orc.philox(ctr, 12345)
    by = out.view(np.uint8).ravel()
    counts = np.bincount(by, minlength=256)
    chi2 = ((counts - by.size / 256) ** 2 / (by.size / 256)).sum()
    assert stats.chi2.sf(chi2, 255) > 1e-4
    # every output bit is balanced
    bits = np.unpackbits(out.view(np.uint8).reshape(n, 16), axis=0).mean(axis=0)
    assert np.all(np.abs(bits - 0.5) < 6 * 0.5 / np.sqrt(n))


def _normals(orc, n_particles=8192, n_steps=64, seed=3, tag=0):
    p = np.repeat(np.arange(n_particles, dtype=np.uint32), n_steps)
    n = np.tile(np.arange(n_steps, dtype=np.uint64), n_particles)
    return orc.main_normals(p, n, seed, tag).reshape(n_particles, n_steps)


def test_main_normals_standard_normal(orc):
    w = _normals(orc).ravel()
    ks = stats.kstest(w, "norm")
    assert ks.pvalue > 1e-4
    n = w.size
    assert abs(w.mean()) < 5 / np.sqrt(n)
    assert abs(w.var() - 1) < 5 * np.sqrt(2 / n)
    assert abs(stats.kurtosis(w)) < 5 * np.sqrt(24 / n)
    # The largest magnitude a 32-bit uniform can produce is sqrt(2*33 ln 2).
    assert np.abs(w).max() <= np.sqrt(-2 * np.log(0.5 * 2.0**-32)) + 1e-12


def test_main_normals_independent_across_steps(orc):
    w = _normals(orc)
    n = w.shape[0]
    for lag in (1, 2, 3, 4, 5):
        a, b = w[:, :-lag].ravel(), w[:, lag:].ravel()
        assert abs(np.corrcoef(a, b)[0, 1]) < 5 / np.sqrt(a.size)
        assert abs(np.corrcoef(a * a, b * b)[0, 1]) < 5 / np.sqrt(a.size)
    # different particles and different seeds give different streams
    assert not np.array_equal(w[0], w[1])
    w2 = _normals(orc, seed=4)
    assert abs(np.corrcoef(w.ravel(), w2.ravel())[0, 1]) < 5 / np.sqrt(w.size)
    w3 = _normals(orc, tag=1)
    assert abs(np.corrcoef(w.ravel(), w3.ravel())[0, 1]) < 5 / np.sqrt(w.size)
    # each position within a group of four steps is a standard normal
    for j in range(4):
        assert stats.kstest(w[:, j::4].ravel(), "norm").pvalue > 1e-4


def test_hit_stream(orc):
    m = 200_000
    p = np.arange(m, dtype=np.uint32) % 5000
    n = (np.arange(m, dtype=np.uint64) // 5000)
    k = np.ones(m, np.uint32) + (np.arange(m) % 3).astype(np.uint32)
    r, w = orc.hit_draws(p, n, k, 9)
    assert stats.kstest(w, "norm").pvalue > 1e-4
    u = (r.astype(np.float64) + 0.5) / 2.0**32
    assert stats.kstest(u, "uniform").pvalue > 1e-4
    # the hit stream is not the main stream
    wm = orc.main_normals(p, n, 9)
    assert abs(np.corrcoef(w, wm)[0, 1]) < 5 / np.sqrt(m)
