"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point the public header declares, and rejects invalid inputs
before touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "metricgraph.h")


@pytest.fixture(scope="module")
def B():
    from paper_2512_02175_amd import binding
    try:
        binding.lib()
    except ImportError as e:
        pytest.skip(str(e))
    return binding


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mg_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_path():
    names = _declared()
    for n in ("mg_graph_create", "mg_particles_init", "mg_simulate", "mg_histogram",
              "mg_exit_counts", "mg_batch_create", "mg_batch_simulate"):
        assert n in names


def test_library_exports_every_declared_symbol(B):
    L = B.lib()
    for n in _declared():
        assert hasattr(L, n), n
    assert set(_declared()) == set(B.EXPORTED)


def test_binding_uses_the_c_names(B):
    for n in _declared():
        assert callable(getattr(B, n)), n


def _desc(**over):
    g = workloads.star_graph(3, 1.0)
    for k, v in over.items():
        setattr(g, k, v)
    return g


@pytest.mark.parametrize("mutate,msg", [
    (lambda g: setattr(g, "length", np.array([1.0, -1.0, 1.0])), "length"),
    (lambda g: setattr(g, "length", np.array([1.0, np.nan, 1.0])), "length"),
    (lambda g: setattr(g, "sigma", np.array([1.0, 0.0, 1.0])), "sigma"),
    (lambda g: setattr(g, "drift_a", np.array([1.0, np.inf, 1.0])), "drift_a"),
    (lambda g: setattr(g, "slot_jump_prob", g.slot_jump_prob * 1.01), "sum"),
    (lambda g: setattr(g, "slot_jump_prob", np.where(np.arange(6) == 0, -0.1, g.slot_jump_prob)), ">= 0"),
    (lambda g: setattr(g, "slot_orient", np.zeros(6, np.uint8)), "does not end there"),
    (lambda g: setattr(g, "slot_edge", np.array([0, 0, 2, 0, 1, 2], np.int32)), ""),
    (lambda g: setattr(g, "vtx_offsets", np.array([0, 3, 2, 5, 6], np.int32)), "decreases"),
    (lambda g: setattr(g, "edge_term", np.array([1, 2, 9], np.int32)), "out of range"),
    (lambda g: setattr(g, "vtx_kind", np.array([7, 0, 0, 0], np.uint8)), "kind"),
])
def test_invalid_graphs_rejected(B, mutate, msg):
    g = _desc()
    mutate(g)
    with pytest.raises(B.MgError) as ei:
        B.mg_graph_create(g)
    assert ei.value.status == B.MG_EINVAL
    assert msg in str(ei.value)


def test_zero_probability_standard_vertex_rejected(B):
    g = workloads.star_graph(2, 1.0, b_center=[1.0, 0.0])
    g.slot_jump_prob[g.vtx_offsets[2]] = 0.0      # leaf 2 has no way out
    with pytest.raises(B.MgError) as ei:
        B.mg_graph_create(g)
    assert "no positive jump probability" in str(ei.value)


def test_null_arguments(B):
    L = B.lib()
    h = C.c_void_p()
    assert L.mg_graph_create(None, C.byref(h)) == B.MG_EINVAL
    assert L.mg_particles_init(None, 10, 0, None, None, 0, 0, None, C.byref(h)) == B.MG_EINVAL
    assert L.mg_simulate(None, 1, 0.1, 0) == B.MG_EINVAL
    assert L.mg_histogram(None, 4, None, 0) == B.MG_EINVAL
    assert L.mg_batch_create(0, None, C.byref(h)) == B.MG_EINVAL
    L.mg_graph_destroy(None)
    L.mg_particles_destroy(None)
    L.mg_batch_destroy(None)
    assert "batch" in B.mg_last_error() or B.mg_last_error() != ""


def test_particle_count_limit(B):
    """A set holds at most 2^32 - 2^20 particles (the persistent launch's
    32-bit claim counter then cannot wrap); the count is checked before
    anything touches the device."""
    L = B.lib()
    h = C.c_void_p()
    for n in (0, -1, 2**32 - 2**20 + 1, 2**32 - 1, 2**40):
        assert L.mg_particles_init(None, n, 2, None, None, 0, 0, None, C.byref(h)) == B.MG_EINVAL
        assert "2^32 - 2^20" in B.mg_last_error()
    assert L.mg_particles_init(None, 2**32 - 2**20, 2, None, None, 0, 0, None,
                               C.byref(h)) == B.MG_EINVAL
    assert "graph is NULL" in B.mg_last_error()


def _cubic(**hi):
    g = workloads.segment(2.0, 0.0, 0.0, 1.0)
    for k, v in hi.items():
        setattr(g, k, np.asarray(v, np.float64))
    return g


def _wentzell(a, c, b, kind=3):
    """Segment whose vertex 0 is a Wentzell vertex with a_v = a, c_v = c and
    jump probability b."""
    g = workloads.segment(1.0, 0.0, 0.0, 1.0)
    g.vtx_kind[0] = kind
    g.slot_jump_prob[g.vtx_offsets[0]] = b
    g.vtx_kill = np.array([a, 0.0])
    g.vtx_sticky = np.array([c, 0.0])
    return g


def _table(knots, sig=lambda x: 1.0 + 0.0 * x, dsig=lambda x: 0.0 * x, length=1.0,
           cubic=False):
    """Segment with a drift and diffusion table of knots + 1 entries."""
    g = workloads.segment(1.0, 0.0, 0.0, 1.0)
    if knots >= 1:
        workloads.tabulate(g, knots, lambda e, x: -x, lambda e, x: -1.0 + 0 * x,
                           lambda e, x: sig(x), lambda e, x: dsig(x))
    else:
        g.table_offsets = np.array([0, 1])
        g.table_mu = g.table_dmu = g.table_dsigma = np.zeros(1)
        g.table_sigma = np.ones(1)
    if not np.isfinite(length):
        g.length[:] = length
        g.bin_span = np.array([2.0])
    if cubic:
        g.drift_c2 = np.array([0.5])
    return g


@pytest.mark.parametrize("make,msg", [
    # a mirror vertex must be a leaf (the centre of a star has three slots)
    (lambda: workloads.from_edges(4, [0, 0, 0], [1, 2, 3], 1.0, vtx_kind=[2, 0, 0, 0]),
     "leaf"),
    # sigma(x) = (1 - 2x)^2 vanishes inside the edge; its ends are positive
    (lambda: _cubic(sigma_c1=[-4.0], sigma_c2=[4.0]), "sigma(x)"),
    # sigma(x) = 1 - 3x^2 + x^3 turns negative at x = 1
    (lambda: _cubic(sigma_c2=[-3.0], sigma_c3=[1.0]), "sigma(x)"),
    # sigma(x) = (1 - 2x)^2 - 1e-12 x^3 is -1.25e-13 at x = 1/2: the
    # critical point must come from the cancellation-free formula (the
    # textbook form puts it at 0.50004, where sigma is 7.9e-9)
    (lambda: _cubic(sigma_c1=[-4.0], sigma_c2=[4.0], sigma_c3=[-1e-12]), "sigma(x)"),
    (lambda: _cubic(drift_c3=[np.nan]), "not finite"),
    (lambda: workloads.from_edges(2, [0], [1], [np.inf], bin_span=2.0), None),
    # Wentzell vertices: a_v + sum b + c_v must be 1, a_v and c_v >= 0, and
    # some b > 0 (the particle must be able to leave)
    (lambda: _wentzell(0.2, 0.1, 0.6), "not 1"),
    (lambda: _wentzell(-0.1, 0.0, 1.1), ">= 0"),
    (lambda: _wentzell(0.0, np.nan, 1.0), ">= 0"),
    (lambda: _wentzell(0.5, 0.5, 0.0), "no positive jump probability"),
    (lambda: _wentzell(0.2, 0.1, 0.7, kind=4), "unknown kind"),
    # tabulated coefficients: at least 2 knots, a positive sigma on the
    # whole edge (1 - 2 sin(pi x) dips below 0 between knots 0 and 1 here),
    # finite edges, no cubic terms beside a table
    (lambda: _table(0), "at least 2 knots"),
    (lambda: _table(4, sig=lambda x: 1.0 - 1.2 * np.sin(np.pi * x),
                    dsig=lambda x: -1.2 * np.pi * np.cos(np.pi * x)), "sigma(x)"),
    (lambda: _table(4, length=np.inf), "finite edge"),
    (lambda: _table(4, cubic=True), "replaces the cubic terms"),
])
def test_method_variant_graphs_checked(B, make, msg):
    """Mirror vertices, cubic coefficients and Wentzell vertices are validated
    on the host: the bad cases are refused with the reason, the good ones
    pass validation
    (which is all that runs here; building the device tables needs a GPU)."""
    g = make()
    if msg is None:
        g.drift_c2 = np.array([0.1])  # higher terms need a finite edge
        msg = "finite edge"
    with pytest.raises(B.MgError) as ei:
        B.mg_graph_create(g)
    assert ei.value.status == B.MG_EINVAL
    assert msg in str(ei.value), str(ei.value)


def test_struct_layouts_match_the_header(B, tmp_path):
    """The binding's ctypes structs have the header's field offsets and
    sizes (compiled with the host C compiler from include/metricgraph.h)."""
    structs = {"mg_graph_desc": B.mg_graph_desc, "mg_options": B.mg_options,
               "mg_tuning": B.mg_tuning, "mg_image_header": B.mg_image_header,
               "mg_event": B.mg_event}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "metricgraph.h"',
             "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for f in cls._fields_:
            lines.append(f'  printf("{name} {f[0]} %zu\\n", offsetof({name}, {f[0]}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe),
                    str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        s, f, v = line.split()
        got[(s, f)] = int(v)
    for name, cls in structs.items():
        assert got[(name, "size")] == C.sizeof(cls), name
        for f in cls._fields_:
            assert got[(name, f[0])] == getattr(cls, f[0]).offset, (name, f[0])


@pytest.mark.parametrize("args", [(6, 8, 16), (-1, 8, 16), (0, 0, 16), (0, 9, 16), (0, 8, 0),
                                  (0, 8, (1 << 20) + 1)])
def test_valu_rate_arguments_checked(B, args):
    """The VALU calibration refuses an unknown instruction kind and counts out
    of range before touching the device."""
    rate = C.c_double()
    st = B.lib().mg_valu_rate(*args, C.byref(rate), None)
    assert st == B.MG_EINVAL, (args, st)
    assert B.mg_last_error()


def test_checkpoint_arguments_checked(B):
    """Save and load refuse NULL handles and buffers before touching the
    device."""
    L = B.lib()
    h = C.c_void_p()
    buf = np.zeros(256, np.uint8)
    assert L.mg_particles_image_bytes(None) == -1
    assert L.mg_particles_save(None, B._p(buf), buf.size) == B.MG_EINVAL
    assert L.mg_particles_load(None, B._p(buf), buf.size, None, None) == B.MG_EINVAL
    assert "out is NULL" in B.mg_last_error()
    assert L.mg_particles_load(None, B._p(buf), buf.size, None, C.byref(h)) == B.MG_EINVAL
    assert "NULL argument" in B.mg_last_error() and not h.value
    with pytest.raises(ValueError):
        B.image_header(buf[:95])
