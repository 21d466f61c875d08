"""FP64 CPU oracle for the timestep-splitting Euler-Maruyama particle step.

TEST INFRASTRUCTURE ONLY: ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` are the only callers.  The product
library never imports, links or executes anything from this directory, and
this directory shares no code with it.

The arithmetic lives in ``mg_oracle.c`` (plain C, FP64, -ffp-contract=off,
OpenMP over particles).  This module compiles it with gcc when needed and
marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mg_oracle.c")
_LIB = os.path.join(_HERE, "libmg_oracle.so")
_lib = None

INIT_EXPLICIT, INIT_AT_VERTEX, INIT_UNIFORM_LENGTH = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile the oracle shared library (gcc, -O2, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Graph(C.Structure):
    _fields_ = [("n_vertices", C.c_int32), ("n_edges", C.c_int32),
                ("edge_init", C.c_void_p), ("edge_term", C.c_void_p),
                ("length", C.c_void_p), ("drift_a", C.c_void_p),
                ("drift_c", C.c_void_p), ("sigma", C.c_void_p),
                ("vtx_offsets", C.c_void_p), ("slot_edge", C.c_void_p),
                ("slot_orient", C.c_void_p), ("slot_jump_prob", C.c_void_p),
                ("vtx_kind", C.c_void_p), ("bin_span", C.c_void_p),
                ("drift_c2", C.c_void_p), ("drift_c3", C.c_void_p),
                ("sigma_c1", C.c_void_p), ("sigma_c2", C.c_void_p),
                ("sigma_c3", C.c_void_p), ("vtx_kill", C.c_void_p),
                ("vtx_sticky", C.c_void_p), ("table_offsets", C.c_void_p),
                ("table_mu", C.c_void_p), ("table_dmu", C.c_void_p),
                ("table_sigma", C.c_void_p), ("table_dsigma", C.c_void_p)]

TABLES = ("table_mu", "table_dmu", "table_sigma", "table_dsigma")

HIGHER = ("drift_c2", "drift_c3", "sigma_c1", "sigma_c2", "sigma_c3")


def lib():
    global _lib
    if _lib is None:
        # MG_ORACLE_LIB points the tests' mutation checks at a deliberately
        # broken build of this file (see tests/test_oracle_mutants.py).
        path = os.environ.get("MG_ORACLE_LIB")
        if not path:
            path = build()
        L = C.CDLL(path)
        vp, i64, u64, i32, u32 = C.c_void_p, C.c_int64, C.c_uint64, C.c_int32, C.c_uint32
        L.or_philox_batch.argtypes = [vp, u64, i64, vp]
        L.or_main_normals.argtypes = [vp, vp, i64, u32, u64, vp]
        L.or_hit_draws.argtypes = [vp, vp, vp, i64, u32, u64, vp, vp]
        L.or_thresholds.argtypes = [vp, vp]
        L.or_thresholds.restype = C.c_int
        L.or_first_root_batch.argtypes = [vp, vp, vp, i64, vp]
        L.or_simulate.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, u64, u64,
                                  C.c_double, u64, u32, i32, vp, vp, vp, i32]
        L.or_simulate.restype = C.c_int
        L.or_simulate_traced.argtypes = [vp, u32, vp, vp, vp, vp, vp, u64, u64,
                                         C.c_double, u64, u32, i32, vp, vp, vp,
                                         i64, vp, vp, vp, vp, vp, vp, vp]
        L.or_simulate_traced.restype = C.c_int
        L.or_init.argtypes = [vp, i64, vp, i32, i32, u64, u32, vp, vp, vp, vp, vp]
        L.or_init.restype = C.c_int
        L.or_init_sources.argtypes = [vp, i64, vp, i32, vp, vp, u64, u32, vp, vp, vp, vp, vp]
        L.or_init_sources.restype = C.c_int
        L.or_histogram.argtypes = [vp, i64, vp, vp, vp, i32, vp]
        L.or_fnv_offset.restype = u64
        _lib = L
    return _lib


def default_threads() -> int:
    """OpenMP threads of a run: OMP_NUM_THREADS when set (a machine's share
    of its cores), else every core the process may use."""
    v = os.environ.get("OMP_NUM_THREADS", "")
    if v.isdigit() and int(v) > 0:
        return int(v)
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class OracleGraph:
    """Holds contiguous copies of a graph description and its ctypes view."""

    def __init__(self, desc):
        self.desc = desc
        self._keep = dict(
            edge_init=np.ascontiguousarray(desc.edge_init, np.int32),
            edge_term=np.ascontiguousarray(desc.edge_term, np.int32),
            length=np.ascontiguousarray(desc.length, np.float64),
            drift_a=np.ascontiguousarray(desc.drift_a, np.float64),
            drift_c=np.ascontiguousarray(desc.drift_c, np.float64),
            sigma=np.ascontiguousarray(desc.sigma, np.float64),
            vtx_offsets=np.ascontiguousarray(desc.vtx_offsets, np.int32),
            slot_edge=np.ascontiguousarray(desc.slot_edge, np.int32),
            slot_orient=np.ascontiguousarray(desc.slot_orient, np.uint8),
            slot_jump_prob=np.ascontiguousarray(desc.slot_jump_prob, np.float64),
            vtx_kind=np.ascontiguousarray(desc.vtx_kind, np.uint8),
        )
        span = getattr(desc, "bin_span", None)
        self._keep["bin_span"] = np.ascontiguousarray(
            self._keep["length"] if span is None else span, np.float64)
        if not np.all(np.isfinite(self._keep["bin_span"])):
            raise ValueError("a semi-infinite edge needs a finite bin_span")
        kind, off = self._keep["vtx_kind"], self._keep["vtx_offsets"]
        if np.any(kind > 3):
            raise ValueError("unknown vertex kind")
        if np.any((kind == 2) & (np.diff(off) != 1)):
            raise ValueError("a mirror vertex must be a leaf (exactly one slot)")
        # higher coefficient terms: absent arrays are passed as NULL (zero)
        hi = []
        for n in HIGHER:
            v = getattr(desc, n, None)
            if v is None:
                hi.append(None)
                continue
            self._keep[n] = np.ascontiguousarray(
                np.broadcast_to(np.asarray(v, np.float64), (int(desc.n_edges),)))
            hi.append(self._keep[n].ctypes.data)
        # Wentzell vertices (kind 3): a_v and c_v, read only at such vertices
        for n in ("vtx_kill", "vtx_sticky"):
            v = getattr(desc, n, None)
            if v is None:
                hi.append(None)
                continue
            self._keep[n] = np.ascontiguousarray(
                np.broadcast_to(np.asarray(v, np.float64), (int(desc.n_vertices),)))
            hi.append(self._keep[n].ctypes.data)
        # tabulated coefficients: knot offsets [E+1] and four knot arrays
        off_t = getattr(desc, "table_offsets", None)
        if off_t is None:
            hi += [None] * 5
        else:
            self._keep["table_offsets"] = np.ascontiguousarray(off_t, np.int32)
            if self._keep["table_offsets"].size != int(desc.n_edges) + 1:
                raise ValueError("table_offsets needs E + 1 entries")
            hi.append(self._keep["table_offsets"].ctypes.data)
            for n in TABLES:
                self._keep[n] = np.ascontiguousarray(getattr(desc, n), np.float64)
                hi.append(self._keep[n].ctypes.data)
        k = self._keep
        self.c = _Graph(int(desc.n_vertices), int(desc.n_edges),
                        *[k[n].ctypes.data for n in (
                            "edge_init", "edge_term", "length", "drift_a",
                            "drift_c", "sigma", "vtx_offsets", "slot_edge",
                            "slot_orient", "slot_jump_prob", "vtx_kind", "bin_span")],
                        *hi)
        self.V = int(desc.n_vertices)
        self.E = int(desc.n_edges)
        self.nnz = int(k["vtx_offsets"][-1])

    @property
    def ref(self):
        return C.byref(self.c)


def as_graph(g) -> OracleGraph:
    return g if isinstance(g, OracleGraph) else OracleGraph(g)


@dataclass
class State:
    """Particle rows: RNG index, edge, position from the edge's initial
    vertex, alive flag, hit-sequence hash, total hits."""
    pid: np.ndarray
    edge: np.ndarray
    x: np.ndarray
    alive: np.ndarray
    seqhash: np.ndarray
    hits: np.ndarray

    def copy(self) -> "State":
        return State(*(a.copy() for a in (self.pid, self.edge, self.x, self.alive,
                                           self.seqhash, self.hits)))

    def take(self, idx) -> "State":
        return State(*(a[idx].copy() for a in (self.pid, self.edge, self.x, self.alive,
                                                self.seqhash, self.hits)))


@dataclass
class Counts:
    exit_slot: np.ndarray
    absorbed: np.ndarray
    truncations: int = 0
    substeps: int = 0
    hits: int = 0


def philox(ctr: np.ndarray, seed: int) -> np.ndarray:
    ctr = np.ascontiguousarray(ctr, np.uint32).reshape(-1, 4)
    out = np.empty_like(ctr)
    lib().or_philox_batch(_ptr(ctr), C.c_uint64(seed), ctr.shape[0], _ptr(out))
    return out


def main_normals(p, n, seed: int, tag: int = 0) -> np.ndarray:
    p = np.ascontiguousarray(p, np.uint32)
    n = np.ascontiguousarray(np.broadcast_to(n, p.shape), np.uint64)
    out = np.empty(p.shape, np.float64)
    lib().or_main_normals(_ptr(p), _ptr(n), p.size, tag, C.c_uint64(seed), _ptr(out))
    return out


def hit_draws(p, n, k, seed: int, tag: int = 0):
    p = np.ascontiguousarray(p, np.uint32)
    n = np.ascontiguousarray(np.broadcast_to(n, p.shape), np.uint64)
    k = np.ascontiguousarray(np.broadcast_to(k, p.shape), np.uint32)
    r = np.empty(p.shape, np.uint32)
    w = np.empty(p.shape, np.float64)
    lib().or_hit_draws(_ptr(p), _ptr(n), _ptr(k), p.size, tag, C.c_uint64(seed), _ptr(r), _ptr(w))
    return r, w


def thresholds(g) -> np.ndarray:
    g = as_graph(g)
    thr = np.zeros(max(g.nnz, 1), np.uint64)
    rc = lib().or_thresholds(g.ref, _ptr(thr))
    if rc != 0:
        raise ValueError("standard vertex without positive jump probability")
    return thr[: g.nnz]


def first_root(A, B, Cc) -> np.ndarray:
    A = np.ascontiguousarray(A, np.float64)
    B = np.ascontiguousarray(np.broadcast_to(B, A.shape), np.float64)
    Cc = np.ascontiguousarray(np.broadcast_to(Cc, A.shape), np.float64)
    u = np.empty(A.shape, np.float64)
    lib().or_first_root_batch(_ptr(A), _ptr(B), _ptr(Cc), A.size, _ptr(u))
    return u


def fnv_offset() -> int:
    return int(lib().or_fnv_offset())


def init(g, n: int, mode: int, *, vertex: int = 0, seed: int = 0, tag: int = 0,
         edge=None, pos=None, pids=None) -> State:
    """Initial particle rows; ``pids`` selects a subset of particle indices."""
    g = as_graph(g)
    pid = np.arange(n, dtype=np.uint32) if pids is None else np.ascontiguousarray(pids, np.uint32)
    m = pid.size
    st = State(pid, np.zeros(m, np.int32), np.zeros(m, np.float64), np.ones(m, np.uint8),
               np.full(m, fnv_offset(), np.uint64), np.zeros(m, np.uint32))
    if mode == INIT_UNIFORM_LENGTH and not np.all(np.isfinite(g._keep["length"])):
        raise ValueError("uniform-by-length init needs finite edges")
    if mode == INIT_EXPLICIT:
        st.edge[:] = np.asarray(edge, np.int32)[pid] if pids is not None else np.asarray(edge, np.int32)
        st.x[:] = np.asarray(pos, np.float64)[pid] if pids is not None else np.asarray(pos, np.float64)
        return st
    rc = lib().or_init(g.ref, m, _ptr(pid), mode, vertex, C.c_uint64(seed), tag,
                       _ptr(st.edge), _ptr(st.x), _ptr(st.alive), _ptr(st.seqhash),
                       _ptr(st.hits))
    if rc != 0:
        raise ValueError(f"or_init failed ({rc})")
    return st


def init_sources(g, n: int, vertices, rates, *, seed: int = 0, tag: int = 0,
                 pids=None) -> State:
    """Particles injected at source vertices (inlets) chosen with probability
    proportional to their rates, each on an incident edge drawn from the
    vertex's b."""
    g = as_graph(g)
    pid = np.arange(n, dtype=np.uint32) if pids is None else np.ascontiguousarray(pids, np.uint32)
    m = pid.size
    st = State(pid, np.zeros(m, np.int32), np.zeros(m, np.float64), np.ones(m, np.uint8),
               np.full(m, fnv_offset(), np.uint64), np.zeros(m, np.uint32))
    v = np.ascontiguousarray(vertices, np.int32)
    r = np.ascontiguousarray(rates, np.float64)
    rc = lib().or_init_sources(g.ref, m, _ptr(pid), int(v.size), _ptr(v), _ptr(r),
                               C.c_uint64(seed), tag, _ptr(st.edge), _ptr(st.x),
                               _ptr(st.alive), _ptr(st.seqhash), _ptr(st.hits))
    if rc != 0:
        raise ValueError(f"or_init_sources failed ({rc})")
    return st


def new_counts(g) -> Counts:
    g = as_graph(g)
    return Counts(np.zeros(max(g.nnz, 1), np.uint64), np.zeros(max(g.V, 1), np.uint64))


def simulate(g, st: State, n0: int, n_steps: int, dt: float, seed: int, *,
             tag: int = 0, max_splits: int = 8, threads: int | None = None,
             counts: Counts | None = None) -> Counts:
    """Advance the rows of ``st`` in place through steps [n0, n0+n_steps)."""
    g = as_graph(g)
    if counts is None:
        counts = new_counts(g)
    sc = np.zeros(3, np.uint64)
    nth = threads if threads is not None else default_threads()
    rc = lib().or_simulate(g.ref, st.pid.size, _ptr(st.pid), _ptr(st.edge), _ptr(st.x),
                           _ptr(st.alive), _ptr(st.seqhash), _ptr(st.hits),
                           C.c_uint64(n0), C.c_uint64(n_steps), C.c_double(dt),
                           C.c_uint64(seed), tag, max_splits, _ptr(counts.exit_slot),
                           _ptr(counts.absorbed), _ptr(sc), int(nth))
    if rc != 0:
        raise ValueError(f"or_simulate failed ({rc})")
    counts.truncations += int(sc[0])
    counts.substeps += int(sc[1])
    counts.hits += int(sc[2])
    return counts


def simulate_traced(g, st: State, row: int, n0: int, n_steps: int, dt: float,
                    seed: int, *, tag: int = 0, max_splits: int = 8, cap: int = 100000):
    """Advance one row and return its per-hit trace as a dict of arrays."""
    g = as_graph(g)
    counts = new_counts(g)
    sc = np.zeros(3, np.uint64)
    e = np.array([st.edge[row]], np.int32)
    x = np.array([st.x[row]], np.float64)
    al = np.array([st.alive[row]], np.uint8)
    hs = np.array([st.seqhash[row]], np.uint64)
    ht = np.array([st.hits[row]], np.uint32)
    t = dict(step=np.zeros(cap, np.uint64), k=np.zeros(cap, np.int32),
             vertex=np.zeros(cap, np.int32), slot=np.zeros(cap, np.int32),
             u=np.zeros(cap), h_after=np.zeros(cap))
    ln = np.zeros(1, np.int64)
    rc = lib().or_simulate_traced(g.ref, int(st.pid[row]), _ptr(e), _ptr(x), _ptr(al),
                                  _ptr(hs), _ptr(ht), C.c_uint64(n0), C.c_uint64(n_steps),
                                  C.c_double(dt), C.c_uint64(seed), tag, max_splits,
                                  _ptr(counts.exit_slot), _ptr(counts.absorbed), _ptr(sc),
                                  cap, _ptr(t["step"]), _ptr(t["k"]), _ptr(t["vertex"]),
                                  _ptr(t["slot"]), _ptr(t["u"]), _ptr(t["h_after"]), _ptr(ln))
    if rc != 0:
        raise ValueError("or_simulate_traced failed")
    st.edge[row], st.x[row], st.alive[row] = e[0], x[0], al[0]
    st.seqhash[row], st.hits[row] = hs[0], ht[0]
    n = int(ln[0])
    counts.truncations, counts.substeps, counts.hits = int(sc[0]), int(sc[1]), int(sc[2])
    return {k: v[:n] for k, v in t.items()}, counts


def histogram(g, st: State, bins: int) -> np.ndarray:
    g = as_graph(g)
    out = np.zeros(g.E * bins, np.uint64)
    lib().or_histogram(g.ref, st.pid.size, _ptr(st.edge), _ptr(st.x), _ptr(st.alive),
                       bins, _ptr(out))
    return out.reshape(g.E, bins)


def observed_histogram(g, st: State, n0: int, n_steps: int, dt: float, seed: int,
                       every: int, bins: int, *, tag: int = 0, max_splits: int = 8,
                       counts: Counts | None = None):
    """Streamed (time-summed) histogram, by its definition: advance the rows
    of ``st`` through steps [n0, n0+n_steps) and, each time the step counter
    reaches a multiple of ``every``, add the snapshot histogram of the alive
    particles (the binning of ``histogram``).  The time average of these
    snapshots estimates the stationary density after burn-in (Sec. 4.1's
    density measurement).  Returns (sum of snapshots [E, bins], number of
    snapshots, counts)."""
    g = as_graph(g)
    if counts is None:
        counts = new_counts(g)
    acc = np.zeros((g.E, bins), np.uint64)
    snaps = 0
    n, end = n0, n0 + n_steps
    while n < end:
        nxt = min(end, (n // every + 1) * every)
        simulate(g, st, n, nxt - n, dt, seed, tag=tag, max_splits=max_splits, counts=counts)
        n = nxt
        if n % every == 0:
            acc += histogram(g, st, bins)
            snaps += 1
    return acc, snaps, counts


def density_l2(lengths, bins: int, counts, ref_density, mass: float = 0.0) -> float:
    """Empirical L2 distance between the density that binned counts estimate
    and a reference density given as bin averages (Sec. 4.1, Fig. "error"):
    the estimate on bin k of edge e is c_ek / (mass w_e) with bin width
    w_e = L_e / bins (mass 0: the total count), and the distance is
    sqrt(sum_e sum_k w_e (estimate - reference)^2)."""
    L = np.asarray(lengths, np.float64)
    c = np.asarray(counts, np.float64).reshape(L.size, bins)
    r = np.asarray(ref_density, np.float64).reshape(L.size, bins)
    total = float(mass) if mass > 0 else float(np.asarray(counts, np.uint64).sum())
    w = (L / bins)[:, None]
    return float(np.sqrt(np.sum(w * (c / (total * w) - r) ** 2)))


def histogram_csr(g, st: State, bin_offsets, bin_upper) -> np.ndarray:
    """Histogram over per-edge bins of any widths and counts (the appendix's
    general histogram kernel): the bins of edge e are bin_offsets[e] ..
    bin_offsets[e+1]-1, with upper boundaries bin_upper (nondecreasing along
    the edge, the last one L_e).  A particle at x goes to the first bin of its
    edge whose upper boundary is >= x, or to the edge's last bin if none is
    (bins have positive widths, so this is the listing's scan over
    accumulated bin lengths).  Written as that scan, one particle at a
    time."""
    g = as_graph(g)
    off = np.asarray(bin_offsets, np.int64)
    up = np.asarray(bin_upper, np.float64)
    out = np.zeros(int(off[-1]), np.uint64)
    for i in range(st.pid.size):
        if not st.alive[i]:
            continue
        e = int(st.edge[i])
        x = float(st.x[i])
        b = int(off[e + 1]) - 1
        for k in range(int(off[e]), int(off[e + 1])):
            if x <= up[k]:
                b = k
                break
        out[b] += 1
    return out
