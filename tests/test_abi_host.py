"""Host-only checks of the C ABI: the library loads, exports every declared entry point, and rejects
bad descriptors on the host with the documented codes before any HIP call."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2406_04008_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    txt = open(os.path.join(ROOT, "include", "collage.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(collage_[a-z_]+)\s*\(", txt)))


def test_header_and_binding_agree():
    declared = _declared_symbols()
    bound = sorted(n for n, _, _ in _lib.SIGNATURES)
    assert declared == bound


def test_library_loads_and_exports_every_symbol():
    lib = _lib.load()
    for name in _declared_symbols():
        assert hasattr(lib, name), name
    assert b"gfx950" in lib.collage_version()


def _desc(B=1, N=1, V=4, w=(16,), h=(16,), k=(1.0,), shapes=(0, 1), voff=(0, 4)):
    keep = dict(w=np.array(w, np.int32), h=np.array(h, np.int32), k=np.array(k, np.float32),
                s=np.array(shapes, np.int32), v=np.array(voff, np.int32))
    d = _lib.SceneDesc()
    d.num_layouts, d.num_shapes, d.num_verts = B, N, V
    d.layout_width = keep["w"].ctypes.data_as(_lib._i32p)
    d.layout_height = keep["h"].ctypes.data_as(_lib._i32p)
    d.layout_scale = keep["k"].ctypes.data_as(_lib._f32p)
    d.layout_shapes = keep["s"].ctypes.data_as(_lib._i32p)
    d.vert_offset = keep["v"].ctypes.data_as(_lib._i32p)
    d.verts = 0x1000  # never dereferenced: validation fails before any device access
    d.mask = 0x2000
    d.tau, d.r_cut, d.r_pad = 0.5, 8.0, 0.0
    d.w_overlap = d.w_contain = d.w_fill = 1.0
    d.code_capacity = -1
    return d, keep


@pytest.mark.parametrize("mutate,code", [
    (lambda d: setattr(d, "num_layouts", 0), _lib.ERR_INVALID),
    (lambda d: setattr(d, "tau", 0.0), _lib.ERR_INVALID),
    (lambda d: setattr(d, "tau", float("nan")), _lib.ERR_INVALID),
    (lambda d: setattr(d, "r_cut", -1.0), _lib.ERR_INVALID),
    (lambda d: setattr(d, "w_fill", float("inf")), _lib.ERR_INVALID),
    (lambda d: setattr(d, "w_uniform", float("nan")), _lib.ERR_INVALID),
    (lambda d: setattr(d, "tile", 12), _lib.ERR_UNSUPPORTED),
    (lambda d: setattr(d, "tile", 256), _lib.ERR_UNSUPPORTED),
    (lambda d: setattr(d, "flags", 0x80), _lib.ERR_UNSUPPORTED),
    (lambda d: setattr(d, "flags", 0x3), _lib.ERR_UNSUPPORTED),
    (lambda d: setattr(d, "w_wmse", float("inf")), _lib.ERR_INVALID),
    (lambda d: setattr(d, "w_objdown", float("nan")), _lib.ERR_INVALID),
    (lambda d: setattr(d, "code_capacity", -2), _lib.ERR_INVALID),
    (lambda d: setattr(d, "unit_capacity", -2), _lib.ERR_INVALID),
    (lambda d: setattr(d, "bin_chunk", 1025), _lib.ERR_INVALID),
    (lambda d: setattr(d, "num_shapes", 2), _lib.ERR_SIZE),
    (lambda d: setattr(d, "num_verts", 5), _lib.ERR_SIZE),
    (lambda d: setattr(d, "mask", None), _lib.ERR_INVALID),
    (lambda d: setattr(d, "verts", None), _lib.ERR_INVALID),
])
def test_descriptor_validation(mutate, code):
    lib = _lib.load()
    d, keep = _desc()
    mutate(d)
    out = ctypes.c_void_p()
    rc = lib.collage_scene_create(ctypes.byref(d), ctypes.byref(out))
    assert rc == code, (rc, _lib.last_error())
    assert out.value is None
    assert len(_lib.last_error()) > 0


def test_offsets_validation():
    lib = _lib.load()
    out = ctypes.c_void_p()
    d, keep = _desc(w=(0,))
    assert lib.collage_scene_create(ctypes.byref(d), ctypes.byref(out)) == _lib.ERR_INVALID
    d, keep = _desc(k=(-1.0,))
    assert lib.collage_scene_create(ctypes.byref(d), ctypes.byref(out)) == _lib.ERR_INVALID
    d, keep = _desc(B=2, w=(16, 16), h=(16, 16), k=(1.0, 1.0), shapes=(0, 1, 0))
    assert lib.collage_scene_create(ctypes.byref(d), ctypes.byref(out)) == _lib.ERR_INVALID
    d, keep = _desc(N=2, V=4, shapes=(0, 2), voff=(0, 3, 1))
    assert lib.collage_scene_create(ctypes.byref(d), ctypes.byref(out)) == _lib.ERR_INVALID
    d, keep = _desc(V=40000, voff=(0, 40000))
    assert lib.collage_scene_create(ctypes.byref(d), ctypes.byref(out)) == _lib.ERR_INVALID
    assert lib.collage_scene_create(None, ctypes.byref(out)) == _lib.ERR_INVALID


def test_timer_argument_errors():
    # checked on the host before any HIP call
    lib = _lib.load()
    out = ctypes.c_void_p()
    assert lib.collage_timer_create(0, ctypes.byref(out)) == _lib.ERR_INVALID
    assert lib.collage_timer_create(65537, ctypes.byref(out)) == _lib.ERR_INVALID
    assert lib.collage_timer_create(4, None) == _lib.ERR_INVALID
    ms = (ctypes.c_float * 4)()
    assert lib.collage_timer_elapsed(None, ms) == _lib.ERR_INVALID
    lib.collage_timer_destroy(None)  # a no-op
    assert lib.collage_iterate_n(None, None, None, None, None, None, None, None, None, 0.5, 0.9, 0.999, 1e-8,
                                 None, 0, 1, None, None) == _lib.ERR_INVALID


def test_null_scene_calls_fail_cleanly():
    lib = _lib.load()
    nb = ctypes.c_size_t()
    assert lib.collage_workspace_size(None, ctypes.byref(nb)) == _lib.ERR_INVALID
    assert lib.collage_forward(None, None, None, None, None, None, 0, None) == _lib.ERR_INVALID
    assert lib.collage_backward(None, None, None, None, None, 0, None) == _lib.ERR_INVALID
    assert lib.collage_backward_vertices(None, None, None, None, None, None, 0, None) == _lib.ERR_INVALID
    assert lib.collage_forward_backward(None, None, None, None, None, None, None, 0, None) == _lib.ERR_INVALID
    assert lib.collage_graph_launch(None, 1, None) == _lib.ERR_INVALID
    assert lib.collage_adam_reset(None, None, None, None, None) == _lib.ERR_INVALID
    st = (ctypes.c_int32 * _lib.STATUS_WORDS)()
    assert lib.collage_read_status(None, None, 0, st, None) == _lib.ERR_INVALID
    out_g = ctypes.c_void_p()
    # graph capture is refused on the NULL stream and for unknown flags before any HIP call
    assert lib.collage_graph_create(None, None, None, None, None, None, None, None, None, 0.5, 0.9, 0.999, 1e-8,
                                    None, 0, 1, 0, None, ctypes.byref(out_g)) == _lib.ERR_INVALID
    assert lib.collage_graph_create(None, None, None, None, None, None, None, None, None, 0.5, 0.9, 0.999, 1e-8,
                                    None, 0, 1, 2, ctypes.c_void_p(1), ctypes.byref(out_g)) == _lib.ERR_UNSUPPORTED
