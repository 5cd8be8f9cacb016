"""ctypes declarations of libcollage.so (the C ABI of include/collage.h).

Marshalling only: every computation happens in the HIP kernels behind these entry points.  Loading
fails loudly if the library has not been built (run ``python -c "import __graft_entry__ as g; g.build()"``
or ``python paper_2406_04008_amd/build.py``).
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libcollage.so")

OK = 0
GRAPH_RESET_ADAM = 1
ERR_INVALID = -1
ERR_SIZE = -2
ERR_WORKSPACE = -3
ERR_HIP = -4
ERR_UNSUPPORTED = -5
FLAG_NONE = 0
FLAG_AREA_MEAN = 1
LOSS_TERMS = 9  # overlap, contain, fill, pad, down, uniform, wmse, centre, objdown
STATUS_WORDS = 8
STATIC_SCRATCH_BYTES = 64 << 20  # the scratch of collage_forward_backward_static
STATUS_NONFINITE = 0  # (epoch, item) pairs of the last call whose parameters were not all finite
STATUS_CHUNKS = 1  # 64-pixel chunks of the last epoch's coverage pass
STATUS_RESCANNED = 2  # of those, chunks the adjoint rescanned (beyond the code capacity)
STATUS_UNIT_OVERFLOW = 3  # (epoch, layout) pairs whose work units did not fit the layout's pool (results invalid)
STATUS_GRAD_RANGE = 4  # adjoint pieces whose sums were beyond the fixed-point gradient range (gradients invalid)

_i32p = ctypes.POINTER(ctypes.c_int32)
_f32p = ctypes.POINTER(ctypes.c_float)
_vp = ctypes.c_void_p


class SceneDesc(ctypes.Structure):
    _fields_ = [
        ("num_layouts", ctypes.c_int32), ("num_shapes", ctypes.c_int32), ("num_verts", ctypes.c_int32),
        ("layout_width", _i32p), ("layout_height", _i32p), ("layout_scale", _f32p), ("layout_shapes", _i32p),
        ("vert_offset", _i32p),
        ("verts", _vp), ("rho", _vp), ("mask", _vp), ("stroke", _vp),
        ("tau", ctypes.c_float), ("r_cut", ctypes.c_float), ("r_pad", ctypes.c_float),
        ("w_overlap", ctypes.c_float), ("w_contain", ctypes.c_float), ("w_fill", ctypes.c_float),
        ("w_pad", ctypes.c_float), ("w_down", ctypes.c_float), ("w_uniform", ctypes.c_float),
        ("w_wmse", ctypes.c_float), ("w_centre", ctypes.c_float), ("w_objdown", ctypes.c_float),
        ("tile", ctypes.c_int32), ("code_capacity", ctypes.c_int32), ("bin_chunk", ctypes.c_int32),
        ("flags", ctypes.c_uint32), ("unit_capacity", ctypes.c_int32),
    ]


# (name, restype, argtypes) of every exported entry point
SIGNATURES = [
    ("collage_scene_create", ctypes.c_int, [ctypes.POINTER(SceneDesc), ctypes.POINTER(_vp)]),
    ("collage_scene_destroy", None, [_vp]),
    ("collage_workspace_size", ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
    ("collage_scene_info", ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    ("collage_read_status", ctypes.c_int, [_vp, _vp, ctypes.c_size_t, _i32p, _vp]),
    ("collage_forward", ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    ("collage_backward", ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    ("collage_forward_backward", ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    ("collage_backward_vertices", ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    ("collage_forward_backward_static", ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    ("collage_step", ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                    ctypes.c_float, _vp]),
    ("collage_iterate", ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_float, ctypes.c_float,
                                       ctypes.c_float, ctypes.c_float, _vp, ctypes.c_size_t, _vp]),
    ("collage_render_shapes", ctypes.c_int, [_vp, _vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, ctypes.c_size_t,
                                             _vp]),
    ("collage_graph_create", ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_float,
                                            ctypes.c_float, ctypes.c_float, ctypes.c_float, _vp, ctypes.c_size_t,
                                            ctypes.c_int32, ctypes.c_uint32, _vp, ctypes.POINTER(_vp)]),
    ("collage_adam_reset", ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    ("collage_iterate_n", ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_float,
                                         ctypes.c_float, ctypes.c_float, ctypes.c_float, _vp, ctypes.c_size_t,
                                         ctypes.c_int32, _vp, _vp]),
    ("collage_timer_create", ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(_vp)]),
    ("collage_timer_elapsed", ctypes.c_int, [_vp, _f32p]),
    ("collage_timer_destroy", None, [_vp]),
    ("collage_graph_launch", ctypes.c_int, [_vp, ctypes.c_int32, _vp]),
    ("collage_graph_destroy", None, [_vp]),
    ("collage_last_error", ctypes.c_char_p, []),
    ("collage_version", ctypes.c_char_p, []),
]

_LIB = None


class CollageError(RuntimeError):
    def __init__(self, code, where):
        msg = last_error()
        super().__init__(f"{where} failed with code {code}: {msg}")
        self.code = code


def load():
    """Loads libcollage.so (raises if it is missing: there is no fallback path)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_2406_04008_amd/build.py (hipcc, gfx950)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB


def last_error() -> str:
    if _LIB is None:
        return ""
    v = _LIB.collage_last_error()
    return v.decode() if v else ""


def check(code, where):
    if code != OK:
        raise CollageError(code, where)
