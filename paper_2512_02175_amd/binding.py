"""ctypes binding of libmetricgraph.so (include/metricgraph.h).

Functions keep the C names and only marshal arguments: every step of the
path runs in the library's HIP kernels.  PyTorch, when present, supplies the
HIP stream (``torch.cuda.current_stream()``) and, on request, the device
memory of a particle set (``arena="torch"``).  There is no fallback: if the
library is not built, loading it raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmetricgraph.so")

MG_OK, MG_EINVAL, MG_ENOMEM, MG_EDEVICE, MG_ESTATE = 0, 1, 2, 3, 4
MG_FP64, MG_FP32 = 0, 1
MG_VTX_STANDARD, MG_VTX_ABSORBING, MG_VTX_MIRROR, MG_VTX_WENTZELL = 0, 1, 2, 3
MG_INIT_EXPLICIT, MG_INIT_AT_VERTEX, MG_INIT_UNIFORM_LENGTH = 0, 1, 2
MG_SCHED_AUTO, MG_SCHED_LANES, MG_SCHED_POOLS, MG_SCHED_POOLS256, MG_SCHED_POOLS_W8 = 0, 1, 2, 3, 4
(MG_VALU_FMA_F32, MG_VALU_FMA_F64, MG_VALU_MAD_U64_U32, MG_VALU_BITOP3, MG_VALU_ADD_U32,
 MG_VALU_LOG_F32) = range(6)

EXPORTED = (
    "mg_graph_create", "mg_graph_destroy", "mg_particles_arena_bytes",
    "mg_particles_init", "mg_particles_init_sources", "mg_particles_destroy", "mg_simulate",
    "mg_histogram",
    "mg_exit_counts", "mg_particles_read", "mg_particles_step", "mg_particles_image_bytes",
    "mg_particles_save", "mg_particles_load", "mg_trace_events", "mg_trace_read",
    "mg_batch_create",
    "mg_batch_simulate", "mg_batch_destroy", "mg_autotune", "mg_histogram_csr",
    "mg_histogram_csr_noalloc", "mg_observe_histogram",
    "mg_observed_histogram", "mg_density_l2", "mg_valu_rate", "mg_last_error",
)


class MgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"[status {status}] {msg}")
        self.status = status


class mg_graph_desc(C.Structure):
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


class mg_options(C.Structure):
    _fields_ = [("precision", C.c_int), ("max_splits", C.c_int32),
                ("graph_tag", C.c_uint32), ("trace", C.c_int32),
                ("steps_per_launch", C.c_int32), ("hip_stream", C.c_void_p),
                ("arena", C.c_void_p), ("arena_bytes", C.c_int64),
                ("schedule", C.c_int32)]


class mg_tuning(C.Structure):
    _fields_ = [("schedule", C.c_int32), ("idle_trigger", C.c_int32),
                ("pool_size", C.c_int32), ("window", C.c_int32), ("n_probes", C.c_int32),
                ("probe_ms", C.c_float * 12), ("steps_per_launch", C.c_int32),
                ("launch_ms", C.c_float * 2)]


class mg_image_header(C.Structure):
    _fields_ = [("magic", C.c_char * 8), ("version", C.c_uint32), ("header_bytes", C.c_uint32),
                ("total_bytes", C.c_uint64), ("graph", C.c_uint64), ("n", C.c_int64),
                ("n_vertices", C.c_int32), ("n_edges", C.c_int32), ("nnz", C.c_int32),
                ("precision", C.c_int32), ("max_splits", C.c_int32),
                ("graph_tag", C.c_uint32), ("trace", C.c_int32), ("obs_bins", C.c_int32),
                ("obs_every", C.c_uint64), ("obs_start", C.c_uint64), ("step", C.c_uint64)]


class mg_event(C.Structure):
    _fields_ = [("pid", C.c_uint32), ("step", C.c_uint32), ("k", C.c_int32),
                ("vertex", C.c_int32), ("slot", C.c_int32), ("reserved", C.c_int32),
                ("u", C.c_double), ("h_after", C.c_double)]


EVENT_DTYPE = np.dtype([(f[0], {C.c_uint32: "<u4", C.c_int32: "<i4", C.c_double: "<f8"}[f[1]])
                        for f in mg_event._fields_])


def image_header(image) -> mg_image_header:
    """The header of a set image (a host byte array)."""
    b = np.ascontiguousarray(image, np.uint8)
    if b.size < C.sizeof(mg_image_header):
        raise ValueError("image shorter than its header")
    return mg_image_header.from_buffer_copy(b[:C.sizeof(mg_image_header)].tobytes())


_lib = None


def lib() -> C.CDLL:
    """Loads the HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2512_02175_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64
        L.mg_graph_create.argtypes = [vp, vp]
        L.mg_graph_destroy.argtypes = [vp]
        L.mg_graph_destroy.restype = None
        L.mg_particles_arena_bytes.argtypes = [vp, i64, vp]
        L.mg_particles_arena_bytes.restype = i64
        L.mg_particles_init.argtypes = [vp, i64, C.c_int, vp, vp, i32, u64, vp, vp]
        L.mg_particles_init_sources.argtypes = [vp, i64, i32, vp, vp, u64, vp, vp]
        L.mg_particles_destroy.argtypes = [vp]
        L.mg_particles_destroy.restype = None
        L.mg_simulate.argtypes = [vp, i64, C.c_double, u64]
        L.mg_histogram.argtypes = [vp, i32, vp, i64]
        L.mg_exit_counts.argtypes = [vp, vp, vp, vp]
        L.mg_particles_read.argtypes = [vp, i64, i64, vp, vp, vp, vp, vp]
        L.mg_particles_step.argtypes = [vp]
        L.mg_particles_step.restype = i64
        L.mg_particles_image_bytes.argtypes = [vp]
        L.mg_particles_image_bytes.restype = i64
        L.mg_particles_save.argtypes = [vp, vp, i64]
        L.mg_particles_load.argtypes = [vp, vp, i64, vp, vp]
        L.mg_trace_events.argtypes = [vp, i32, vp, i64]
        L.mg_trace_read.argtypes = [vp, vp, i64, vp]
        L.mg_batch_create.argtypes = [i32, vp, vp]
        L.mg_batch_simulate.argtypes = [vp, i64, C.c_double, u64]
        L.mg_batch_destroy.argtypes = [vp]
        L.mg_batch_destroy.restype = None
        L.mg_autotune.argtypes = [vp, C.c_double, u64, i32, vp]
        L.mg_histogram_csr.argtypes = [vp, vp, vp, vp, i64]
        L.mg_histogram_csr_noalloc.argtypes = [vp, vp, vp, vp, i64]
        L.mg_observe_histogram.argtypes = [vp, i32, i32]
        L.mg_observed_histogram.argtypes = [vp, vp, i64, vp]
        L.mg_density_l2.argtypes = [vp, i32, vp, C.c_double, vp, vp]
        L.mg_valu_rate.argtypes = [i32, i32, C.c_uint32, vp, vp]
        L.mg_last_error.restype = C.c_char_p
        for name in EXPORTED:
            if name not in ("mg_graph_destroy", "mg_particles_destroy",
                            "mg_batch_destroy", "mg_last_error",
                            "mg_particles_arena_bytes", "mg_particles_step",
                            "mg_particles_image_bytes"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def mg_last_error() -> str:
    return lib().mg_last_error().decode()


def _check(st: int):
    if st != MG_OK:
        raise MgError(st, mg_last_error())


def _p(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _torch_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except ImportError:
        pass
    return None


class Graph:
    """Owns an mg_graph handle (destroyed with the object)."""

    def __init__(self, handle, desc):
        self.handle = handle
        self.n_vertices = int(desc.n_vertices)
        self.n_edges = int(desc.n_edges)
        self.nnz = int(desc.vtx_offsets[-1])
        self.length = np.asarray(desc.length, np.float64).copy()

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.mg_graph_destroy(self.handle)
            self.handle = None


class Particles:
    """Owns an mg_particles handle; keeps its graph and arena alive."""

    def __init__(self, handle, graph: Graph, n: int, precision: int, arena=None):
        self.handle = handle
        self.graph = graph
        self.n = n
        self.precision = precision
        self._arena = arena

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.mg_particles_destroy(self.handle)
            self.handle = None


class Batch:
    def __init__(self, handle, sets):
        self.handle = handle
        self.sets = list(sets)

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.mg_batch_destroy(self.handle)
            self.handle = None


def mg_graph_create(desc) -> Graph:
    """``desc`` has the fields of mg_graph_desc as numpy arrays (see
    ``workloads.GraphDesc``)."""
    keep = dict(
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
    opt = []
    for k in ("bin_span", "drift_c2", "drift_c3", "sigma_c1", "sigma_c2", "sigma_c3"):
        v = getattr(desc, k, None)
        if v is None:
            opt.append(None)
        else:
            keep[k] = np.ascontiguousarray(
                np.broadcast_to(np.asarray(v, np.float64), (int(desc.n_edges),)))
            opt.append(keep[k].ctypes.data)
    for k in ("vtx_kill", "vtx_sticky"):     # per vertex
        v = getattr(desc, k, None)
        if v is None:
            opt.append(None)
        else:
            keep[k] = np.ascontiguousarray(
                np.broadcast_to(np.asarray(v, np.float64), (int(desc.n_vertices),)))
            opt.append(keep[k].ctypes.data)
    off_t = getattr(desc, "table_offsets", None)     # tabulated coefficients
    if off_t is None:
        opt += [None] * 5
    else:
        keep["table_offsets"] = np.ascontiguousarray(off_t, np.int32)
        opt.append(keep["table_offsets"].ctypes.data)
        for k in ("table_mu", "table_dmu", "table_sigma", "table_dsigma"):
            keep[k] = np.ascontiguousarray(getattr(desc, k), np.float64)
            opt.append(keep[k].ctypes.data)
    d = mg_graph_desc(int(desc.n_vertices), int(desc.n_edges),
                      *[keep[k].ctypes.data for k in (
                          "edge_init", "edge_term", "length", "drift_a", "drift_c",
                          "sigma", "vtx_offsets", "slot_edge", "slot_orient",
                          "slot_jump_prob", "vtx_kind")],
                      *opt)
    h = C.c_void_p()
    _check(lib().mg_graph_create(C.byref(d), C.byref(h)))
    return Graph(h, desc)


def mg_graph_destroy(g: Graph) -> None:
    if g.handle:
        lib().mg_graph_destroy(g.handle)
        g.handle = None


def _options(precision, max_splits, graph_tag, trace, steps_per_launch, stream,
             arena_ptr=None, arena_bytes=0, schedule=MG_SCHED_AUTO):
    return mg_options(int(precision), int(max_splits), int(graph_tag), int(bool(trace)),
                      int(steps_per_launch),
                      stream if stream is not None else _torch_stream(),
                      arena_ptr, int(arena_bytes), int(schedule))


def mg_particles_arena_bytes(g: Graph, n: int, precision=MG_FP64, trace=False) -> int:
    o = _options(precision, 0, 0, trace, 0, None)
    return int(lib().mg_particles_arena_bytes(g.handle, int(n), C.byref(o)))


def mg_particles_init(g: Graph, n: int, mode: int, *, edge=None, pos=None, vertex: int = 0,
                      init_seed: int = 0, precision: int = MG_FP64, max_splits: int = 8,
                      graph_tag: int = 0, trace: bool = False, steps_per_launch: int = 0,
                      stream=None, arena=None, schedule: int = MG_SCHED_AUTO) -> Particles:
    """``arena``: None (library allocates), "torch" (a torch uint8 CUDA
    tensor of the required size), or a torch tensor to use."""
    e = None if edge is None else np.ascontiguousarray(edge, np.int32)
    x = None if pos is None else np.ascontiguousarray(pos, np.float64)
    arena_obj, aptr, abytes = None, None, 0
    if arena is not None:
        import torch
        need = mg_particles_arena_bytes(g, n, precision, trace)
        arena_obj = (torch.empty(need, dtype=torch.uint8, device="cuda")
                     if isinstance(arena, str) else arena)
        aptr, abytes = C.c_void_p(arena_obj.data_ptr()), arena_obj.numel() * arena_obj.element_size()
    o = _options(precision, max_splits, graph_tag, trace, steps_per_launch, stream, aptr, abytes,
                 schedule)
    h = C.c_void_p()
    _check(lib().mg_particles_init(g.handle, int(n), int(mode), _p(e), _p(x), int(vertex),
                                   C.c_uint64(init_seed), C.byref(o), C.byref(h)))
    return Particles(h, g, int(n), int(precision), arena_obj)


def mg_particles_init_sources(g: Graph, n: int, vertices, rates, *, init_seed: int = 0,
                              precision: int = MG_FP64, max_splits: int = 8,
                              graph_tag: int = 0, trace: bool = False,
                              steps_per_launch: int = 0, stream=None,
                              schedule: int = MG_SCHED_AUTO) -> Particles:
    """Particles injected at source vertices with probabilities proportional
    to ``rates``."""
    v = np.ascontiguousarray(vertices, np.int32)
    r = np.ascontiguousarray(rates, np.float64)
    if v.size != r.size:
        raise ValueError("vertices and rates differ in length")
    o = _options(precision, max_splits, graph_tag, trace, steps_per_launch, stream,
                 schedule=schedule)
    h = C.c_void_p()
    _check(lib().mg_particles_init_sources(g.handle, int(n), int(v.size), _p(v), _p(r),
                                           C.c_uint64(init_seed), C.byref(o), C.byref(h)))
    return Particles(h, g, int(n), int(precision))


def mg_particles_destroy(p: Particles) -> None:
    if p.handle:
        lib().mg_particles_destroy(p.handle)
        p.handle = None


def mg_simulate(p: Particles, n_steps: int, dt: float, seed: int) -> None:
    _check(lib().mg_simulate(p.handle, int(n_steps), float(dt), C.c_uint64(seed)))


def mg_histogram(p: Particles, bins_per_edge: int, out=None):
    """Returns a [E, bins] uint64 numpy array, or fills ``out`` (a numpy
    array or a torch CUDA tensor of int64/uint64 with E*bins elements)."""
    E = p.graph.n_edges
    if out is None:
        out = np.zeros(E * bins_per_edge, np.uint64)
        _check(lib().mg_histogram(p.handle, int(bins_per_edge), _p(out), out.size))
        return out.reshape(E, bins_per_edge)
    if isinstance(out, np.ndarray):
        _check(lib().mg_histogram(p.handle, int(bins_per_edge), _p(out), out.size))
    else:
        _check(lib().mg_histogram(p.handle, int(bins_per_edge), C.c_void_p(out.data_ptr()),
                                  out.numel()))
    return out


def mg_histogram_csr(p: Particles, bin_offsets, bin_upper) -> np.ndarray:
    """Histogram over per-edge bins of any widths: bin_offsets[E+1] (CSR) and
    the bins' upper boundaries; returns counts[bin_offsets[E]]."""
    off = np.ascontiguousarray(np.asarray(bin_offsets, np.int32))
    up = np.ascontiguousarray(np.asarray(bin_upper, np.float64))
    out = np.zeros(max(int(off[-1]), 1), np.uint64)
    _check(lib().mg_histogram_csr(p.handle, _p(off), _p(up), _p(out), out.size))
    return out[: int(off[-1])]


def mg_histogram_csr_noalloc(p: Particles, bin_offsets, bin_upper, out=None) -> np.ndarray:
    """mg_histogram_csr staged in the library's fixed per-GPU workspace
    instead of allocated device memory.  ``out``: an optional uint64 numpy
    array or device tensor of at least bin_offsets[E] counters (default: a
    new host array); returns the counts."""
    off = np.ascontiguousarray(np.asarray(bin_offsets, np.int32))
    up = np.ascontiguousarray(np.asarray(bin_upper, np.float64))
    nb = int(off[-1])
    if out is None:
        out = np.zeros(max(nb, 1), np.uint64)
    if isinstance(out, np.ndarray):
        _check(lib().mg_histogram_csr_noalloc(p.handle, _p(off), _p(up), _p(out), out.size))
        return out[:nb]
    _check(lib().mg_histogram_csr_noalloc(p.handle, _p(off), _p(up),
                                          C.c_void_p(out.data_ptr()), out.numel()))
    return out[:nb]


def mg_observe_histogram(p: Particles, bins_per_edge: int, every: int) -> None:
    """Starts (or restarts, or with every=0 stops) the streamed histogram:
    a snapshot of the alive particles' bins whenever the step counter
    reaches a multiple of ``every``."""
    _check(lib().mg_observe_histogram(p.handle, int(bins_per_edge), int(every)))
    p.obs_bins = int(bins_per_edge) if every else 0


def mg_observed_histogram(p: Particles):
    """(counts as a [E, bins] uint64 array, number of snapshots)."""
    nb = getattr(p, "obs_bins", 0)
    E = p.graph.n_edges
    out = np.zeros(max(E * nb, 1), np.uint64)
    ns = C.c_int64()
    _check(lib().mg_observed_histogram(p.handle, _p(out) if nb else None, out.size,
                                       C.byref(ns)))
    return out[: E * nb].reshape(E, nb), int(ns.value)


def mg_density_l2(g: Graph, bins_per_edge: int, counts, ref_density, mass: float = 0.0) -> float:
    """Empirical L2 distance between the density the counts estimate and the
    bin-averaged reference density (both [E, bins] or flat, edge-major)."""
    c = np.ascontiguousarray(np.asarray(counts, np.uint64).ravel())
    r = np.ascontiguousarray(np.asarray(ref_density, np.float64).ravel())
    n = g.n_edges * int(bins_per_edge)
    if c.size != n or r.size != n:
        raise ValueError(f"need {n} counts and reference values")
    out = C.c_double()
    _check(lib().mg_density_l2(g.handle, int(bins_per_edge), _p(c), float(mass), _p(r),
                               C.byref(out)))
    return float(out.value)


def mg_exit_counts(p: Particles):
    """(slot_counts[nnz], absorbed[V], totals[4]) with totals =
    (truncations, sub-steps, vertex hits, particle-steps)."""
    s = np.zeros(max(p.graph.nnz, 1), np.uint64)
    a = np.zeros(max(p.graph.n_vertices, 1), np.uint64)
    t = np.zeros(4, np.uint64)
    _check(lib().mg_exit_counts(p.handle, _p(s), _p(a), _p(t)))
    return s[: p.graph.nnz], a[: p.graph.n_vertices], t


def mg_particles_read(p: Particles, first: int = 0, count: int | None = None, trace=False):
    count = p.n - first if count is None else count
    edge = np.zeros(count, np.int32)
    pos = np.zeros(count, np.float64)
    alive = np.zeros(count, np.uint8)
    sh = np.zeros(count, np.uint64) if trace else None
    hi = np.zeros(count, np.uint32) if trace else None
    _check(lib().mg_particles_read(p.handle, int(first), int(count), _p(edge), _p(pos),
                                   _p(alive), _p(sh), _p(hi)))
    out = dict(edge=edge, x=pos, alive=alive)
    if trace:
        out.update(seqhash=sh, hits=hi)
    return out


def mg_particles_step(p: Particles) -> int:
    return int(lib().mg_particles_step(p.handle))


def mg_particles_image_bytes(p: Particles) -> int:
    return int(lib().mg_particles_image_bytes(p.handle))


def mg_particles_save(p: Particles) -> np.ndarray:
    """The set's image (a host uint8 array) after every queued step."""
    img = np.empty(mg_particles_image_bytes(p), np.uint8)
    _check(lib().mg_particles_save(p.handle, _p(img), int(img.size)))
    return img


def mg_particles_load(g: Graph, image, *, steps_per_launch: int = 0, stream=None,
                      schedule: int = MG_SCHED_AUTO, arena=None) -> Particles:
    """A new set on ``g`` from an image of mg_particles_save; precision,
    max_splits, graph_tag and trace come from the image.  ``arena`` as in
    mg_particles_init."""
    img = np.ascontiguousarray(image, np.uint8)
    arena_obj, aptr, abytes = None, None, 0
    if arena is not None:
        import torch
        hd = image_header(img)
        need = mg_particles_arena_bytes(g, int(hd.n), int(hd.precision), bool(hd.trace))
        arena_obj = (torch.empty(need, dtype=torch.uint8, device="cuda")
                     if isinstance(arena, str) else arena)
        aptr, abytes = C.c_void_p(arena_obj.data_ptr()), arena_obj.numel() * arena_obj.element_size()
    o = _options(MG_FP64, 0, 0, False, steps_per_launch, stream, aptr, abytes, schedule)
    h = C.c_void_p()
    _check(lib().mg_particles_load(g.handle, _p(img), int(img.size), C.byref(o), C.byref(h)))
    hd = image_header(img)
    q = Particles(h, g, int(hd.n), int(hd.precision), arena_obj)
    q.obs_bins = int(hd.obs_bins)
    return q


def mg_trace_events(p: Particles, ids, capacity: int = 1 << 16) -> None:
    """Records every vertex hit of particles ``ids`` (empty: trace off)."""
    a = np.ascontiguousarray(ids, np.int64)
    _check(lib().mg_trace_events(p.handle, int(a.size), _p(a) if a.size else None,
                                 int(capacity)))
    p.ev_cap = int(capacity) if a.size else 0


def mg_trace_read(p: Particles):
    """(records as a structured array sorted by particle, step and hit
    index, number of hits recorded including dropped ones)."""
    n = C.c_int64()
    _check(lib().mg_trace_read(p.handle, None, 0, C.byref(n)))
    kept = min(int(n.value), getattr(p, "ev_cap", 0))
    out = np.zeros(max(kept, 1), EVENT_DTYPE)
    _check(lib().mg_trace_read(p.handle, _p(out), kept, C.byref(n)))
    out = out[:kept]
    return out[np.lexsort((out["k"], out["step"], out["pid"]))], int(n.value)


def mg_batch_create(sets) -> Batch:
    arr = (C.c_void_p * len(sets))(*[s.handle for s in sets])
    h = C.c_void_p()
    _check(lib().mg_batch_create(len(sets), arr, C.byref(h)))
    return Batch(h, sets)


def mg_batch_simulate(b: Batch, n_steps: int, dt: float, seed: int) -> None:
    _check(lib().mg_batch_simulate(b.handle, int(n_steps), float(dt), C.c_uint64(seed)))


def mg_batch_destroy(b: Batch) -> None:
    if b.handle:
        lib().mg_batch_destroy(b.handle)
        b.handle = None


def mg_autotune(p: Particles, dt: float, seed: int = 0, probe_steps: int = 0) -> dict:
    """Times the FP32 schedules on a scratch copy of the set and keeps the
    fastest; returns the choice and the probe times (ms)."""
    t = mg_tuning()
    _check(lib().mg_autotune(p.handle, float(dt), C.c_uint64(seed), int(probe_steps),
                             C.byref(t)))
    return dict(schedule=int(t.schedule), idle_trigger=int(t.idle_trigger),
                pool_size=int(t.pool_size), window=int(t.window), n_probes=int(t.n_probes),
                probe_ms=[float(t.probe_ms[i]) for i in range(t.n_probes)],
                steps_per_launch=int(t.steps_per_launch),
                launch_ms=[float(t.launch_ms[0]), float(t.launch_ms[1])])


def mg_valu_rate(op: int, waves_per_simd: int = 8, iters: int = 16384):
    """Measured issue rate of one VALU instruction kind (lane-ops/s) and the
    timed launch's milliseconds."""
    rate = C.c_double()
    ms = C.c_float()
    _check(lib().mg_valu_rate(int(op), int(waves_per_simd), int(iters), C.byref(rate),
                              C.byref(ms)))
    return float(rate.value), float(ms.value)
