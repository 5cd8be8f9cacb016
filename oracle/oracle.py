"""ctypes front end of the FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import this module.  The product
path (the HIP library and its binding) never does.  It converts a ``Scene`` (seeded inputs) and
parameters into double-precision arrays and calls ``liboracle.so`` (built from ``collage_oracle.c``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "collage_oracle.c")

NTERMS = 9  # loss terms per layout: overlap, contain, fill, pad, down, uniform, wmse, centre, objdown

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


class _OracleScene(ctypes.Structure):
    _fields_ = [
        ("B", ctypes.c_int32), ("N", ctypes.c_int32), ("V", ctypes.c_int32),
        ("width", _ip), ("height", _ip), ("scale", _dp), ("shape_off", _ip), ("vert_off", _ip),
        ("verts", _dp), ("mask", _dp),
        ("tau", ctypes.c_double), ("r_cut", ctypes.c_double), ("r_pad", ctypes.c_double),
        ("w", ctypes.c_double * 9),
        ("use_cutoff", ctypes.c_int32), ("use_bbox", ctypes.c_int32),
        ("stroke", _dp),
        ("area_mean", ctypes.c_int32),
    ]


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (IEEE semantics: no fast-math)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-Wall", "-o", LIB_PATH + ".tmp",
               SRC_PATH, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        build()
        L = ctypes.CDLL(LIB_PATH)
        L.oracle_forward.argtypes = [ctypes.POINTER(_OracleScene), _dp, _dp, _dp, _dp]
        L.oracle_render.argtypes = [ctypes.POINTER(_OracleScene), _dp, ctypes.c_int, ctypes.c_int, _dp, _dp]
        L.oracle_signed_distance.argtypes = [ctypes.POINTER(_OracleScene), _dp, ctypes.c_int, ctypes.c_int, _dp, _ip]
        L.oracle_backward.argtypes = [ctypes.POINTER(_OracleScene), _dp, _dp, _dp]
        L.oracle_backward_full.argtypes = [ctypes.POINTER(_OracleScene), _dp, _dp, _dp, _dp]
        L.oracle_nearest_ambiguity.argtypes = [ctypes.POINTER(_OracleScene), _dp, _dp, ctypes.c_double,
                                               ctypes.c_double, _dp]
        L.oracle_adam.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp, ctypes.c_int, _dp, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double]
        L.oracle_collage_lr.argtypes = [ctypes.POINTER(_OracleScene), _dp, ctypes.c_double, _dp]
        L.oracle_quality.argtypes = [ctypes.POINTER(_OracleScene), _dp, _dp, ctypes.POINTER(ctypes.c_int64)]
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        _LIB = L
    return _LIB


def _d(a):
    return np.ascontiguousarray(a, np.float64)


def _ptr(a, t=_dp):
    return a.ctypes.data_as(t) if a is not None else None


class Oracle:
    """FP64 oracle bound to one scene at one level."""

    def __init__(self, scene, level=None, use_cutoff=True, use_bbox=True, mask=None):
        self.scene = scene
        w, h, k, off = scene.layout_arrays(level)
        self.widths, self.heights = w.astype(np.int32), h.astype(np.int32)
        self.scales = _d(k)
        self.shape_off = off.astype(np.int32)
        self.vert_off = np.ascontiguousarray(scene.vert_off, np.int32)
        self.verts = _d(scene.verts).reshape(-1)
        self.mask = _d(scene.packed_mask(level) if mask is None else mask).reshape(-1)
        self.pix_off = np.concatenate([[0], np.cumsum(self.widths.astype(np.int64) * self.heights)])
        s = _OracleScene()
        s.B, s.N, s.V = scene.num_layouts, scene.num_shapes, scene.num_verts
        s.width, s.height = _ptr(self.widths, _ip), _ptr(self.heights, _ip)
        s.scale = _ptr(self.scales)
        s.shape_off, s.vert_off = _ptr(self.shape_off, _ip), _ptr(self.vert_off, _ip)
        s.verts = _ptr(self.verts) if self.verts.size else None
        s.mask = _ptr(self.mask) if self.mask.size else None
        s.tau, s.r_cut, s.r_pad = scene.tau, scene.r_cut, scene.r_pad
        for i, wv in enumerate(scene.weights()):
            s.w[i] = wv
        s.use_cutoff, s.use_bbox = int(use_cutoff), int(use_bbox and use_cutoff)
        self.stroke = None if getattr(scene, "stroke", None) is None else _d(scene.stroke)
        s.stroke = _ptr(self.stroke) if self.stroke is not None and self.stroke.size else None
        s.area_mean = int(bool(getattr(scene, "area_mean", False)))
        self._s = s

    @property
    def num_pixels(self):
        return int(self.pix_off[-1])

    def forward(self, params):
        p = _d(params).reshape(-1)
        S = np.zeros(self.num_pixels)
        Sp = np.zeros(self.num_pixels)
        loss = np.zeros(NTERMS * self.scene.num_layouts)
        rc = lib().oracle_forward(ctypes.byref(self._s), _ptr(p), _ptr(S), _ptr(Sp), _ptr(loss))
        assert rc == 0
        return S, Sp, loss.reshape(-1, NTERMS)

    def loss(self, params, dloss=None):
        _, _, L = self.forward(params)
        if dloss is None:
            return float(L.sum())
        return float((L * np.asarray(dloss, np.float64).reshape(L.shape)).sum())

    def render(self, params, first=0, count=None):
        count = self.scene.num_shapes - first if count is None else count
        p = _d(params).reshape(-1)
        sizes = []
        for q in range(first, first + count):
            b = self._layout_of(q)
            sizes.append(int(self.widths[b]) * int(self.heights[b]))
        tot = int(sum(sizes))
        A = np.zeros(max(tot, 1))
        Ap = np.zeros(max(tot, 1))
        rc = lib().oracle_render(ctypes.byref(self._s), _ptr(p), first, count, _ptr(A), _ptr(Ap))
        assert rc == 0
        return A[:tot], Ap[:tot]

    def signed_distance(self, params, first=0, count=None):
        count = self.scene.num_shapes - first if count is None else count
        p = _d(params).reshape(-1)
        tot = 0
        for q in range(first, first + count):
            b = self._layout_of(q)
            tot += int(self.widths[b]) * int(self.heights[b])
        sd = np.zeros(max(tot, 1))
        e = np.zeros(max(tot, 1), np.int32)
        rc = lib().oracle_signed_distance(ctypes.byref(self._s), _ptr(p), first, count, _ptr(sd), _ptr(e, _ip))
        assert rc == 0
        return sd[:tot], e[:tot]

    def backward(self, params, dloss=None):
        p = _d(params).reshape(-1)
        B = self.scene.num_layouts
        dl = np.ones(NTERMS * B) if dloss is None else _d(dloss).reshape(-1)
        if dl.size != NTERMS * B:
            raise ValueError(f"dloss must have {NTERMS} entries per layout")
        g = np.zeros(4 * max(self.scene.num_shapes, 1))
        rc = lib().oracle_backward(ctypes.byref(self._s), _ptr(p), _ptr(dl), _ptr(g))
        assert rc == 0
        return g[: 4 * self.scene.num_shapes].reshape(-1, 4)

    def nearest_ambiguity(self, params, delta_abs, delta_rel, dloss=None):
        """[N,4]: per item and component, the sum over its pixels of the largest change of the pixel's
        gradient terms if an edge that is not a neighbour of its nearest edge, within
        delta_abs + delta_rel |p - k t| of the nearest distance, were taken as the nearest edge."""
        p = _d(params).reshape(-1)
        B = self.scene.num_layouts
        dl = np.ones(NTERMS * B) if dloss is None else _d(dloss).reshape(-1)
        if dl.size != NTERMS * B:
            raise ValueError(f"dloss must have {NTERMS} entries per layout")
        out = np.zeros(4 * max(self.scene.num_shapes, 1))
        rc = lib().oracle_nearest_ambiguity(ctypes.byref(self._s), _ptr(p), _ptr(dl), float(delta_abs),
                                            float(delta_rel), _ptr(out))
        assert rc == 0
        return out[: 4 * self.scene.num_shapes].reshape(-1, 4)

    def backward_vertices(self, params, dloss=None):
        """(grad [N,4], grad_verts [V,2]): the gradient with respect to the parameters and to every
        outline vertex in its item's frame."""
        p = _d(params).reshape(-1)
        B = self.scene.num_layouts
        dl = np.ones(NTERMS * B) if dloss is None else _d(dloss).reshape(-1)
        if dl.size != NTERMS * B:
            raise ValueError(f"dloss must have {NTERMS} entries per layout")
        g = np.zeros(4 * max(self.scene.num_shapes, 1))
        gv = np.zeros(2 * max(self.scene.num_verts, 1))
        rc = lib().oracle_backward_full(ctypes.byref(self._s), _ptr(p), _ptr(dl), _ptr(g), _ptr(gv))
        assert rc == 0
        return g[: 4 * self.scene.num_shapes].reshape(-1, 4), gv[: 2 * self.scene.num_verts].reshape(-1, 2)

    def fd_vertex_gradient(self, params, vertices, h=1e-4, dloss=None):
        """Central differences of the total loss with respect to the listed vertices ([len, 2]), each
        coordinate stepped by h canonical px in the item frame."""
        out = np.zeros((len(vertices), 2))
        for r, m in enumerate(vertices):
            for c in range(2):
                base = self.verts[2 * m + c]
                self.verts[2 * m + c] = base + h
                lp = self.loss(params, dloss)
                self.verts[2 * m + c] = base - h
                lm = self.loss(params, dloss)
                self.verts[2 * m + c] = base
                out[r, c] = (lp - lm) / (2 * h)
        return out

    def learning_rates(self, lr_px=None):
        lr_px = self.scene.lr_px if lr_px is None else lr_px
        lr = np.zeros(4 * max(self.scene.num_shapes, 1))
        rho = _d(self.scene.rho)
        lib().oracle_collage_lr(ctypes.byref(self._s), _ptr(rho), lr_px, _ptr(lr))
        return lr[: 4 * self.scene.num_shapes].reshape(-1, 4)

    def adam(self, params, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        """In-place Adam on double arrays; returns (params, m, v)."""
        p, g, mm, vv, l = (_d(a).reshape(-1).copy() for a in (params, grad, m, v, lr))
        rc = lib().oracle_adam(p.size, _ptr(p), _ptr(g), _ptr(mm), _ptr(vv), int(t), _ptr(l), beta1, beta2, eps)
        assert rc == 0
        shp = np.shape(params)
        return p.reshape(shp), mm.reshape(shp), vv.reshape(shp)

    def fd_gradient(self, params, h_t=1e-4, h_rim=1e-4, dloss=None, shapes=None):
        """Central differences of the total loss; theta and s are stepped by h_rim / (k * rho_i).

        The loss is only piecewise smooth in the parameters (a pixel centre crossing a medial axis
        of an outline is a kink of its signed distance), so a step of 1e-3 px can straddle kinks and
        miss the derivative by ~1e-3 relative; 1e-4 px agrees with 1e-5 and 1e-6 to ~1e-9."""
        p0 = _d(params).reshape(-1, 4)
        N = p0.shape[0]
        shapes = range(N) if shapes is None else shapes
        g = np.full((N, 4), np.nan)
        for q in shapes:
            b = self._layout_of(q)
            k = float(self.scales[b])
            rho = float(self.scene.rho[q])
            hs = [h_t / k, h_t / k, h_rim / (k * rho), h_rim / (k * rho)]
            for c in range(4):
                pp, pm = p0.copy(), p0.copy()
                pp[q, c] += hs[c]
                pm[q, c] -= hs[c]
                g[q, c] = (self.loss(pp, dloss) - self.loss(pm, dloss)) / (2 * hs[c])
        return g

    def quality(self, params):
        """Sec. 6 metrics per layout on hard rasters (sd >= 0 covers a pixel, M >= 1/2 is the target):
        (metrics [B, 3] = LC, OO, EA;  counts [B, 4] = target, covered in target, overlap, covered outside)."""
        p = _d(params).reshape(-1)
        B = self.scene.num_layouts
        out = np.zeros(3 * B)
        cnt = np.zeros(4 * B, np.int64)
        rc = lib().oracle_quality(ctypes.byref(self._s), _ptr(p), _ptr(out), cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
        assert rc == 0
        return out.reshape(B, 3), cnt.reshape(B, 4)

    def _layout_of(self, q):
        return int(np.searchsorted(self.shape_off, q, side="right") - 1)

    def layout_images(self, flat):
        out = []
        for b in range(self.scene.num_layouts):
            a, z = self.pix_off[b], self.pix_off[b + 1]
            out.append(flat[a:z].reshape(self.heights[b], self.widths[b]))
        return out


def set_threads(n: int):
    lib().oracle_set_threads(int(n))


def num_threads() -> int:
    return int(lib().oracle_num_threads())
