"""Seeded synthetic inputs for the image-space collage hot path.

This module only *constructs inputs*: item outlines (as closed polygons in each item's local frame),
container masks sampled at pixel centres, and initial per-item transforms.  It contains none of the
method's arithmetic (no coverage, no losses, no gradients, no optimizer), so both the GPU path and the
FP64 oracle can consume the same scenes without sharing any of the computation they are compared on.

Item representation follows the paper's "Vector Representation" paragraph (Sec. 3): each item is a
closed outline; cubic Bezier outlines are flattened once, in the item's local frame, at 8 parameter
values per segment (flattening commutes with the rigid transform of eq. 2, since Bezier curves are
affine invariant).  The local frame is centred on the outline's area centroid, which is the rotation
and scaling centre of eq. 2.  The container image of Sec. 4 (interior black, exterior white) is given
as its complement M = 1 inside, 0 outside, sampled at pixel centres (i + 1/2, j + 1/2), y down.

All randomness comes from ``numpy.random.default_rng(seed)`` (PCG64) with a fixed draw order, so a
(config, seed) pair names one scene exactly.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
from typing import List, Optional, Sequence

import numpy as np

TWO_PI = 2.0 * math.pi


# ----------------------------------------------------------------------------------------------------
# Data containers
# ----------------------------------------------------------------------------------------------------
@dataclasses.dataclass
class Layout:
    """One independent collage: a container in canonical pixels and a contiguous range of items."""

    width_ref: int  # canonical canvas width (pixels at scale k = 1)
    height_ref: int
    shape_begin: int
    shape_end: int
    # Container = union of rotated ellipses (cx, cy, a, b, phi) and rotated rectangles (cx, cy, hw, hh, phi),
    # all in canonical pixels.  ``full`` makes the whole canvas the container.
    ellipses: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0, 5)))
    rects: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0, 5)))
    full: bool = False

    @property
    def num_shapes(self) -> int:
        return self.shape_end - self.shape_begin


@dataclasses.dataclass
class Scene:
    """A batch of layouts plus the constants of the loss (all lengths in *level* pixels)."""

    name: str
    verts: np.ndarray  # [V, 2] float32, local frame, canonical px, centroid at the origin
    vert_off: np.ndarray  # [N + 1] int32 CSR offsets into verts
    rho: np.ndarray  # [N] float32, max vertex radius |v| (rim radius) in canonical px
    params: np.ndarray  # [N, 4] float32 initial (t_x, t_y, theta, s), canonical px / radians
    layouts: List[Layout]
    levels: List[int]  # level sides for coarse-to-fine; scale k = level / level_ref
    level_ref: int
    # per item stroke half-width in canonical px: 0 for a closed outline (coverage from the signed
    # distance, positive inside); > 0 for an open polyline stroked to that half-width (coverage from
    # k |s| w - d, with d the distance to the polyline); None = every item is a closed outline
    stroke: Optional[np.ndarray] = None
    tau: float = 0.5
    r_cut: float = 8.0
    r_pad: float = 0.0
    w_overlap: float = 1.0
    w_contain: float = 1.0
    w_fill: float = 1.0
    w_pad: float = 0.0
    w_down: float = 0.0
    w_uniform: float = 0.0  # uniform (dilation) term, off unless a scene sets it
    w_wmse: float = 0.0     # weighted mean square error containment (penalty 1 inside, 100 outside)
    w_centre: float = 0.0   # central force towards the canvas centre (image space)
    w_objdown: float = 0.0  # downward force on the item origins (object space)
    area_mean: bool = False  # overlap, contain, fill, pad and wmse divided by the canvas area
    steps_per_level: int = 300
    lr_px: float = 0.5
    seed: int = 0

    # -------- sizes --------
    @property
    def num_shapes(self) -> int:
        return int(self.vert_off.shape[0] - 1)

    @property
    def num_verts(self) -> int:
        return int(self.verts.shape[0])

    @property
    def num_layouts(self) -> int:
        return len(self.layouts)

    def scale(self, level: Optional[int] = None) -> float:
        lv = self.level_ref if level is None else level
        return float(lv) / float(self.level_ref)

    def canvas(self, layout: Layout, level: Optional[int] = None):
        k = self.scale(level)
        return int(round(layout.width_ref * k)), int(round(layout.height_ref * k))

    def layout_arrays(self, level: Optional[int] = None):
        """(widths[B], heights[B], scales[B], shape_offsets[B+1]) for one level."""
        k = self.scale(level)
        w = np.array([self.canvas(L, level)[0] for L in self.layouts], np.int32)
        h = np.array([self.canvas(L, level)[1] for L in self.layouts], np.int32)
        ks = np.full(len(self.layouts), k, np.float32)
        off = np.array([L.shape_begin for L in self.layouts] + [self.layouts[-1].shape_end], np.int32)
        return w, h, ks, off

    def masks(self, level: Optional[int] = None) -> List[np.ndarray]:
        k = self.scale(level)
        return [container_mask(L, *self.canvas(L, level), k) for L in self.layouts]

    def packed_mask(self, level: Optional[int] = None) -> np.ndarray:
        return np.concatenate([m.reshape(-1) for m in self.masks(level)]).astype(np.float32)

    def pixel_offsets(self, level: Optional[int] = None) -> np.ndarray:
        w, h, _, _ = self.layout_arrays(level)
        return np.concatenate([[0], np.cumsum(w.astype(np.int64) * h)]).astype(np.int64)

    def weights(self):
        """Loss weights in term order: overlap, contain, fill, pad, down, uniform."""
        return (self.w_overlap, self.w_contain, self.w_fill, self.w_pad, self.w_down, self.w_uniform, self.w_wmse,
                self.w_centre, self.w_objdown)

    def signature(self) -> str:
        h = hashlib.sha1()
        for a in (self.verts, self.vert_off, self.params) + (() if self.stroke is None else (self.stroke,)):
            h.update(np.ascontiguousarray(a).tobytes())
        for L in self.layouts:
            h.update(np.array([L.width_ref, L.height_ref, L.shape_begin, L.shape_end], np.int64).tobytes())
        return h.hexdigest()[:16]

    def layout_subset(self, b: int) -> "Scene":
        """Layout `b` alone, as a one-layout scene with the same constants and levels."""
        lay = self.layouts[b]
        v0, v1 = int(self.vert_off[lay.shape_begin]), int(self.vert_off[lay.shape_end])
        return dataclasses.replace(
            self, name=f"{self.name}[{b}]", verts=self.verts[v0:v1],
            stroke=None if self.stroke is None else self.stroke[lay.shape_begin:lay.shape_end],
            vert_off=(self.vert_off[lay.shape_begin:lay.shape_end + 1] - v0).astype(np.int32),
            rho=self.rho[lay.shape_begin:lay.shape_end], params=self.params[lay.shape_begin:lay.shape_end],
            layouts=[Layout(lay.width_ref, lay.height_ref, 0, lay.num_shapes, lay.ellipses, lay.rects, lay.full)])

    def with_params(self, params: np.ndarray) -> "Scene":
        return dataclasses.replace(self, params=np.ascontiguousarray(params, np.float32))


# ----------------------------------------------------------------------------------------------------
# Outlines (local frame)
# ----------------------------------------------------------------------------------------------------
def regular_polygon(n: int, radius: float, phase: float = 0.0) -> np.ndarray:
    m = np.arange(n, dtype=np.float64)
    ang = phase + TWO_PI * m / n
    return np.stack([radius * np.cos(ang), radius * np.sin(ang)], 1)


def star_polygon(points: int, r_outer: float, ratio: float) -> np.ndarray:
    """2*points vertices alternating r_outer and ratio*r_outer at angles pi*m/points."""
    m = np.arange(2 * points, dtype=np.float64)
    r = np.where(m % 2 == 0, r_outer, ratio * r_outer)
    ang = math.pi * m / points
    return np.stack([r * np.cos(ang), r * np.sin(ang)], 1)


def rectangle(half_w: float, half_h: float) -> np.ndarray:
    return np.array([[-half_w, -half_h], [half_w, -half_h], [half_w, half_h], [-half_w, half_h]], np.float64)


def flatten_closed_cubic(ctrl: np.ndarray, samples_per_segment: int = 8) -> np.ndarray:
    """Closed chain of cubic Beziers with 3K control points; segment m uses points 3m..3m+3 (mod 3K).

    Sampled at t = j / samples_per_segment, j = 0..samples_per_segment-1, so the next segment's t = 0
    point is not duplicated.
    """
    n = ctrl.shape[0]
    assert n % 3 == 0 and n >= 3
    K = n // 3
    t = np.arange(samples_per_segment, dtype=np.float64) / samples_per_segment
    b0 = (1 - t) ** 3
    b1 = 3 * (1 - t) ** 2 * t
    b2 = 3 * (1 - t) * t ** 2
    b3 = t ** 3
    out = []
    for m in range(K):
        p0, p1, p2, p3 = (ctrl[(3 * m + j) % n] for j in range(4))
        out.append(b0[:, None] * p0 + b1[:, None] * p1 + b2[:, None] * p2 + b3[:, None] * p3)
    return np.concatenate(out, 0)


def polygon_area_centroid(P: np.ndarray):
    x, y = P[:, 0], P[:, 1]
    xn, yn = np.roll(x, -1), np.roll(y, -1)
    cr = x * yn - xn * y
    A = 0.5 * cr.sum()
    cx = ((x + xn) * cr).sum() / (6 * A)
    cy = ((y + yn) * cr).sum() / (6 * A)
    return A, np.array([cx, cy])


def is_simple_polygon(P: np.ndarray) -> bool:
    """O(E^2) proper-intersection test between all pairs of non-adjacent edges (vectorised)."""
    n = P.shape[0]
    A = P
    B = np.roll(P, -1, 0)

    def orient(a, b, c):
        return (b[..., 0] - a[..., 0]) * (c[..., 1] - a[..., 1]) - (b[..., 1] - a[..., 1]) * (c[..., 0] - a[..., 0])

    a1, b1 = A[:, None, :], B[:, None, :]
    a2, b2 = A[None, :, :], B[None, :, :]
    d1 = orient(a2, b2, a1)
    d2 = orient(a2, b2, b1)
    d3 = orient(a1, b1, a2)
    d4 = orient(a1, b1, b2)
    hit = (d1 * d2 < 0) & (d3 * d4 < 0)
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    adjacent = (np.abs(i - j) <= 1) | (np.abs(i - j) == n - 1)
    return not bool((hit & ~adjacent).any())


def jittered_bezier(rng: np.random.Generator, segments: int, radius: float, max_tries: int = 50) -> np.ndarray:
    """3K control points at angles 2*pi*j/3K, radius * U(0.7, 1.3), flattened to 8 points per segment."""
    for _ in range(max_tries):
        n = 3 * segments
        jit = rng.uniform(0.7, 1.3, n)
        ang = TWO_PI * np.arange(n) / n
        ctrl = np.stack([radius * jit * np.cos(ang), radius * jit * np.sin(ang)], 1)
        P = flatten_closed_cubic(ctrl, 8)
        if is_simple_polygon(P):
            return P
    raise RuntimeError("could not draw a simple Bezier outline")


def recentre(P: np.ndarray) -> np.ndarray:
    """Moves the area centroid to the origin (the vertex mean for outlines without area)."""
    if P.shape[0] < 3:
        return P - P.mean(0)
    A, c = polygon_area_centroid(P)
    if not (abs(A) > 1e-12 and np.all(np.isfinite(c))):
        return P - P.mean(0)
    return P - c


# ----------------------------------------------------------------------------------------------------
# Containers
# ----------------------------------------------------------------------------------------------------
def container_mask(layout: Layout, width: int, height: int, k: float) -> np.ndarray:
    """M[j, i] = 1 if the pixel centre ((i + 1/2)/k, (j + 1/2)/k) lies in the container, else 0."""
    if layout.full:
        return np.ones((height, width), np.float32)
    xs = (np.arange(width, dtype=np.float64) + 0.5) / k
    ys = (np.arange(height, dtype=np.float64) + 0.5) / k
    X, Y = np.meshgrid(xs, ys)
    inside = np.zeros((height, width), bool)
    for cx, cy, a, b, phi in layout.ellipses:
        c, s = math.cos(phi), math.sin(phi)
        u = c * (X - cx) + s * (Y - cy)
        v = -s * (X - cx) + c * (Y - cy)
        inside |= (u / a) ** 2 + (v / b) ** 2 <= 1.0
    for cx, cy, hw, hh, phi in layout.rects:
        c, s = math.cos(phi), math.sin(phi)
        u = c * (X - cx) + s * (Y - cy)
        v = -s * (X - cx) + c * (Y - cy)
        inside |= (np.abs(u) <= hw) & (np.abs(v) <= hh)
    return inside.astype(np.float32)


def random_ellipses(rng: np.random.Generator, count: int, width: float, height: float, lo: float, hi: float):
    """Centres U(1/4, 3/4) * (W, H), semi-axes U(lo, hi), orientation U(0, pi); drawn in that order."""
    centres = rng.uniform(0.25, 0.75, (count, 2)) * np.array([width, height])
    axes = rng.uniform(lo, hi, (count, 2))
    phi = rng.uniform(0.0, math.pi, count)
    return np.concatenate([centres, axes, phi[:, None]], 1)


def random_rects(rng: np.random.Generator, count: int, width: float, height: float, lo: float, hi: float):
    centres = rng.uniform(0.25, 0.75, (count, 2)) * np.array([width, height])
    half = rng.uniform(lo, hi, (count, 2))
    phi = rng.uniform(0.0, math.pi, count)
    return np.concatenate([centres, half, phi[:, None]], 1)


def place_in_mask(rng: np.random.Generator, mask: np.ndarray, count: int) -> np.ndarray:
    """(t_x, t_y, theta, s): a uniformly chosen container pixel + U(0,1)^2 offset, theta U(0, 2pi), s = 1."""
    jj, ii = np.nonzero(mask > 0.5)
    if jj.size == 0:
        jj, ii = np.nonzero(np.ones_like(mask))
    pick = rng.integers(0, jj.size, count)
    off = rng.uniform(0.0, 1.0, (count, 2))
    theta = rng.uniform(0.0, TWO_PI, count)
    p = np.zeros((count, 4), np.float64)
    p[:, 0] = ii[pick] + off[:, 0]
    p[:, 1] = jj[pick] + off[:, 1]
    p[:, 2] = theta
    p[:, 3] = 1.0
    return p


# ----------------------------------------------------------------------------------------------------
# Assembly
# ----------------------------------------------------------------------------------------------------
def assemble(name: str, outlines: Sequence[np.ndarray], params: np.ndarray, layouts: List[Layout],
             levels: List[int], level_ref: int, stroke: Optional[Sequence[float]] = None, **consts) -> Scene:
    """Items with stroke > 0 are open polylines: centred on their vertex mean (a polyline has no area),
    rim radius max |v| + stroke."""
    w = np.zeros(len(outlines)) if stroke is None else np.asarray(stroke, np.float64)
    outlines = [(np.asarray(P, np.float64) - np.asarray(P, np.float64).mean(0)) if w[i] > 0 else
                recentre(np.asarray(P, np.float64)) for i, P in enumerate(outlines)]
    counts = [P.shape[0] for P in outlines]
    vert_off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    verts = (np.concatenate(outlines, 0) if outlines else np.zeros((0, 2))).astype(np.float32)
    rho = np.array([np.sqrt((np.asarray(P, np.float32).astype(np.float64) ** 2).sum(1)).max() + w[i]
                    for i, P in enumerate(outlines)] if outlines else [], np.float32)
    return Scene(name=name, verts=np.ascontiguousarray(verts), vert_off=vert_off, rho=rho,
                 params=np.ascontiguousarray(params, np.float32).reshape(-1, 4), layouts=layouts,
                 levels=levels, level_ref=level_ref,
                 stroke=None if stroke is None else np.ascontiguousarray(w, np.float32), **consts)


def random_walk_polyline(rng: np.random.Generator, vertices: int, step_lo: float, step_hi: float) -> np.ndarray:
    """An open polyline: `vertices` points, each step of length U(step_lo, step_hi) in a uniform direction."""
    steps = rng.uniform(step_lo, step_hi, vertices - 1)
    ang = rng.uniform(0.0, TWO_PI, vertices - 1)
    P = np.zeros((vertices, 2))
    P[1:, 0] = np.cumsum(steps * np.cos(ang))
    P[1:, 1] = np.cumsum(steps * np.sin(ang))
    return P


def config1(seed: int = 0) -> Scene:
    """64x64 canvas, disk container r = 28 at (32, 32); 8 regular 16-gons of radius U(3, 6)."""
    rng = np.random.default_rng(seed)
    W = H = 64
    lay = Layout(W, H, 0, 8, ellipses=np.array([[32.0, 32.0, 28.0, 28.0, 0.0]]))
    radii = rng.uniform(3.0, 6.0, 8)
    outlines = [regular_polygon(16, r) for r in radii]
    params = place_in_mask(rng, container_mask(lay, W, H, 1.0), 8)
    return assemble("config1", outlines, params, [lay], [64], 64, tau=0.5, r_cut=8.0, r_pad=0.0,
                    w_overlap=1.0, w_contain=1.0, w_fill=1.0, w_pad=0.0, w_down=0.0,
                    steps_per_level=200, seed=seed)


def config2(seed: int = 0) -> Scene:
    """256x256, union of 6 ellipses (semi-axes U(30, 90)); 100 stars with 5..12 points."""
    rng = np.random.default_rng(seed)
    W = H = 256
    ell = random_ellipses(rng, 6, W, H, 30.0, 90.0)
    lay = Layout(W, H, 0, 100, ellipses=ell)
    n = rng.integers(5, 13, 100)
    r_o = rng.uniform(6.0, 14.0, 100)
    q = rng.uniform(0.4, 0.8, 100)
    outlines = [star_polygon(int(a), b, c) for a, b, c in zip(n, r_o, q)]
    params = place_in_mask(rng, container_mask(lay, W, H, 1.0), 100)
    return assemble("config2", outlines, params, [lay], [256], 256, tau=0.5, r_cut=8.0, r_pad=0.0,
                    w_overlap=1.0, w_contain=1.0, w_fill=1.0, w_pad=0.0, w_down=0.0,
                    steps_per_level=200, seed=seed)


def config3(seed: int = 0, num_shapes: int = 500) -> Scene:
    """Coarse-to-fine 128 -> 256 -> 512 -> 1024 (reference level 512), 10-ellipse container with
    semi-axes U(60, 180), 500 jittered closed cubic-Bezier outlines (4..16 segments, radius U(4, 20)),
    padding 2 px and downward force weight 1e-3."""
    rng = np.random.default_rng(seed)
    W = H = 512
    ell = random_ellipses(rng, 10, W, H, 60.0, 180.0)
    lay = Layout(W, H, 0, num_shapes, ellipses=ell)
    K = rng.integers(4, 17, num_shapes)
    r = rng.uniform(4.0, 20.0, num_shapes)
    outlines = [jittered_bezier(rng, int(k), float(rr)) for k, rr in zip(K, r)]
    params = place_in_mask(rng, container_mask(lay, W, H, 1.0), num_shapes)
    return assemble("config3", outlines, params, [lay], [128, 256, 512, 1024], 512, tau=0.5, r_cut=8.0,
                    r_pad=2.0, w_overlap=1.0, w_contain=1.0, w_fill=1.0, w_pad=1.0, w_down=1e-3,
                    steps_per_level=300, seed=seed)


def config4(seed: int = 0, num_layouts: int = 64) -> Scene:
    """Batched: layouts of side {128, 256, 384, 512}, 20..400 items each (50/50 star / Bezier),
    each with its own 6-ellipse container (semi-axes U(30, 90) * side / 256).  Coarse-to-fine levels
    1 -> 2 -> 4 with reference level 4: canvases at a quarter, half and full side."""
    rng = np.random.default_rng(seed)
    outlines, params, layouts = [], [], []
    begin = 0
    for _ in range(num_layouts):
        side = int(rng.choice([128, 256, 384, 512]))
        n = int(rng.integers(20, 401))
        f = side / 256.0
        ell = random_ellipses(rng, 6, side, side, 30.0 * f, 90.0 * f)
        lay = Layout(side, side, begin, begin + n, ellipses=ell)
        for _ in range(n):
            if rng.random() < 0.5:
                pts = int(rng.integers(5, 13))
                outlines.append(star_polygon(pts, float(rng.uniform(6.0, 14.0)), float(rng.uniform(0.4, 0.8))))
            else:
                outlines.append(jittered_bezier(rng, int(rng.integers(4, 17)), float(rng.uniform(4.0, 20.0))))
        params.append(place_in_mask(rng, container_mask(lay, side, side, 1.0), n))
        layouts.append(lay)
        begin += n
    return assemble("config4", outlines, np.concatenate(params, 0), layouts, [1, 2, 4], 4, tau=0.5, r_cut=8.0,
                    r_pad=2.0, w_overlap=1.0, w_contain=1.0, w_fill=1.0, w_pad=1.0, w_down=1e-3,
                    steps_per_level=300, seed=seed)


def config5(seed: int = 0, num_shapes: int = 2000) -> Scene:
    """Open shapes: 2048 x 2048 canvas (coarse-to-fine 256 -> 512 -> 1024 -> 2048, reference 2048), a
    container made of 10 ellipses and 10 rotated rectangles (sizes U(30, 90) x 2048 / 256), 2000 open
    polylines of 3..12 vertices (random-walk steps U(3, 15) px) stroked to half-width 1.5 px, padding 2 px,
    downward force weight 1e-3."""
    rng = np.random.default_rng(seed)
    W = H = 2048
    f = W / 256.0
    lay = Layout(W, H, 0, num_shapes, ellipses=random_ellipses(rng, 10, W, H, 30.0 * f, 90.0 * f),
                 rects=random_rects(rng, 10, W, H, 30.0 * f, 90.0 * f))
    nv = rng.integers(3, 13, num_shapes)
    outlines = [random_walk_polyline(rng, int(n), 3.0, 15.0) for n in nv]
    params = place_in_mask(rng, container_mask(lay, W, H, 1.0), num_shapes)
    return assemble("config5", outlines, params, [lay], [256, 512, 1024, 2048], 2048,
                    stroke=np.full(num_shapes, 1.5), tau=0.5, r_cut=8.0, r_pad=2.0, w_overlap=1.0,
                    w_contain=1.0, w_fill=1.0, w_pad=1.0, w_down=1e-3, steps_per_level=300, seed=seed)


def paper_loss_preset(scene: Scene) -> Scene:
    """The weights of Sec. 4.2 (eq. 8): containment alpha = 3e3 on the WMSE of eq. 5, overlap beta = 8e4,
    uniform gamma = 5e-4, with the 1 / (w h) of eqs. 5 and 6; every other term off."""
    return dataclasses.replace(scene, w_overlap=8e4, w_contain=0.0, w_fill=0.0, w_pad=0.0, w_down=0.0,
                               w_uniform=5e-4, w_wmse=3e3, w_centre=0.0, w_objdown=0.0, area_mean=True)


def random_scene(seed: int, sizes: Sequence[tuple], shapes_per_layout: Sequence[int], kinds=("poly", "star", "bezier"),
                 radius=(3.0, 12.0), r_pad: float = 2.0, w_pad: float = 1.0, w_down: float = 1e-3,
                 off_canvas: float = 0.0, name: str = "random") -> Scene:
    """Generic test scenes: any canvas sizes (ragged w.r.t. tiles), mixed outline kinds, random
    scale in [0.7, 1.4], and optionally a fraction of items pushed partly or wholly off the canvas."""
    rng = np.random.default_rng(seed)
    outlines, params, layouts, stroke = [], [], [], []
    begin = 0
    for (W, H), n in zip(sizes, shapes_per_layout):
        ell = random_ellipses(rng, 3, W, H, 0.15 * min(W, H), 0.45 * min(W, H))
        lay = Layout(W, H, begin, begin + n, ellipses=ell)
        for _ in range(n):
            kind = kinds[int(rng.integers(0, len(kinds)))]
            r = float(rng.uniform(*radius))
            w = 0.0
            if kind == "poly":
                outlines.append(regular_polygon(int(rng.integers(3, 20)), r, float(rng.uniform(0, TWO_PI))))
            elif kind == "star":
                outlines.append(star_polygon(int(rng.integers(5, 13)), r, float(rng.uniform(0.4, 0.8))))
            elif kind == "open":
                outlines.append(random_walk_polyline(rng, int(rng.integers(2, 9)), 0.3 * r, 0.9 * r))
                w = float(rng.uniform(0.6, 2.5))
            else:
                outlines.append(jittered_bezier(rng, int(rng.integers(4, 9)), r))
            stroke.append(w)
        p = place_in_mask(rng, container_mask(lay, W, H, 1.0), n)
        p[:, 3] = rng.uniform(0.7, 1.4, n)
        if off_canvas > 0 and n > 0:
            sel = rng.random(n) < off_canvas
            p[sel, 0] = rng.uniform(-25.0, W + 25.0, int(sel.sum()))
        params.append(p)
        layouts.append(lay)
        begin += n
    P = np.concatenate(params, 0) if params else np.zeros((0, 4))
    return assemble(name, outlines, P, layouts, [1], 1, stroke=stroke if "open" in kinds else None, tau=0.5,
                    r_cut=8.0, r_pad=r_pad, w_overlap=1.0, w_contain=1.0, w_fill=1.0, w_pad=w_pad, w_down=w_down,
                    seed=seed)


def single_shape_scene(outline: np.ndarray, width: int, height: int, t, theta: float = 0.0, s: float = 1.0,
                       mask: str = "none", recentre_outline: bool = True, **consts) -> Scene:
    """One item on a canvas; mask 'none' (all zero), 'full', or 'disk' (inscribed disk)."""
    P = np.asarray(outline, np.float64)
    if recentre_outline:
        P = recentre(P)
    if mask == "full":
        lay = Layout(width, height, 0, 1, full=True)
    elif mask == "disk":
        r = 0.45 * min(width, height)
        lay = Layout(width, height, 0, 1, ellipses=np.array([[width / 2, height / 2, r, r, 0.0]]))
    else:
        lay = Layout(width, height, 0, 1)
    params = np.array([[t[0], t[1], theta, s]], np.float64)
    sc = Scene(name="single", verts=P.astype(np.float32), vert_off=np.array([0, P.shape[0]], np.int32),
               rho=np.array([np.sqrt((P.astype(np.float32).astype(np.float64) ** 2).sum(1)).max()], np.float32),
               params=params.astype(np.float32), layouts=[lay], levels=[1], level_ref=1)
    return dataclasses.replace(sc, **consts)


def multi_shape_scene(outlines: Sequence[np.ndarray], params: np.ndarray, width: int, height: int,
                      mask: str = "none", stroke: Optional[Sequence[float]] = None, **consts) -> Scene:
    if mask == "full":
        lay = Layout(width, height, 0, len(outlines), full=True)
    elif mask == "disk":
        r = 0.45 * min(width, height)
        lay = Layout(width, height, 0, len(outlines), ellipses=np.array([[width / 2, height / 2, r, r, 0.0]]))
    else:
        lay = Layout(width, height, 0, len(outlines))
    sc = assemble("multi", outlines, np.asarray(params, np.float64), [lay], [1], 1, stroke=stroke)
    return dataclasses.replace(sc, **consts)


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}


def make_scene(config_id: int, seed: int = 0) -> Scene:
    return CONFIGS[config_id](seed)
