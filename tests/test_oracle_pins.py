"""Pins of the FP64 oracle against facts fixed by the paper's definitions and by mathematics.

None of these tests re-types the oracle's formulas: each compares it with a closed form, an
independent algorithm (winding numbers, 1-D quadrature of a radially symmetric integrand), an
invariant, a library routine (torch.optim.Adam) or its own central finite differences.
"""
import dataclasses
import math

import numpy as np
import pytest
from scipy import integrate

from oracle.oracle import Oracle
from paper_2406_04008_amd import scenes as S

TAU = 0.5
R_CUT = 8.0


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _alpha(sd, tau=TAU, r_cut=R_CUT, shift=0.0):
    """Coverage profile as a function of signed distance, written for the quadrature only."""
    x = sd + shift
    return np.where(x < -r_cut, 0.0, _sigmoid(x / tau))


def _offset_average(fn, base, n=4):
    """Mean of fn(centre) over an n x n stratified grid of sub-pixel offsets.  The pixel-grid sampling
    ripple is periodic in the offset with zero mean, so averaging leaves the continuum value."""
    vals = [fn((base[0] + (a + 0.5) / n, base[1] + (b + 0.5) / n)) for a in range(n) for b in range(n)]
    return np.mean(vals, 0)


def _fine_circle(radius, n=1024):
    P = S.regular_polygon(n, radius)
    area = 0.5 * n * radius ** 2 * math.sin(2 * math.pi / n)
    return P, area, math.sqrt(area / math.pi)


def _radial_integral(f, r_eff, upper):
    """2*pi * int_0^upper f(r_eff - rho) rho d rho, split at the kinks of the integrand."""
    pts = sorted({0.0, max(r_eff - 6, 0.0), r_eff, r_eff + 2.0, r_eff + R_CUT, r_eff + R_CUT + 2.0, upper})
    tot = 0.0
    for a, b in zip(pts[:-1], pts[1:]):
        if b > a:
            v, _ = integrate.quad(lambda rho: f(r_eff - rho) * rho, a, b, limit=400, epsabs=1e-12, epsrel=1e-12)
            tot += v
    return 2 * math.pi * tot


# --------------------------------------------------------------------------------------------------
# Geometry: signed distance and the even-odd rule
# --------------------------------------------------------------------------------------------------
def test_rectangle_signed_distance_closed_form():
    """Axis-aligned rectangle at a generic offset: sd has a closed form at every pixel centre."""
    hw, hh = 7.3, 4.1
    cx, cy = 20.37, 15.81
    sc = S.single_shape_scene(S.rectangle(hw, hh), 40, 32, (cx, cy), 0.0, 1.0)
    o = Oracle(sc)
    sd, _ = o.signed_distance(sc.params)
    sd = sd.reshape(32, 40)
    # the scene stores float32 values: use exactly those
    cx, cy = (float(v) for v in sc.params[0, :2])
    hw, hh = (float(v) for v in np.abs(sc.verts[0]))
    X, Y = np.meshgrid(np.arange(40) + 0.5, np.arange(32) + 0.5)
    dx, dy = np.abs(X - cx) - hw, np.abs(Y - cy) - hh
    outside = np.hypot(np.maximum(dx, 0), np.maximum(dy, 0))
    inside = np.minimum(-dx, -dy)
    expect = np.where((dx > 0) | (dy > 0), -outside, inside)
    np.testing.assert_allclose(sd, expect, atol=1e-9)


def _winding(P, x, y):
    """Winding number by summing signed angles (independent of the crossing rule)."""
    A = P[:, None, :] - np.stack([x, y], -1)[None]
    B = np.roll(P, -1, 0)[:, None, :] - np.stack([x, y], -1)[None]
    cross = A[..., 0] * B[..., 1] - A[..., 1] * B[..., 0]
    dot = (A * B).sum(-1)
    return np.arctan2(cross, dot).sum(0) / (2 * math.pi)


@pytest.mark.parametrize("kind", ["star", "bezier"])
def test_inside_rule_matches_winding_number(kind):
    rng = np.random.default_rng(3)
    P = S.star_polygon(7, 11.0, 0.45) if kind == "star" else S.jittered_bezier(rng, 9, 11.0)
    sc = S.single_shape_scene(P, 32, 32, (16.13, 15.77), 0.37, 1.1)
    o = Oracle(sc)
    sd, _ = o.signed_distance(sc.params)
    # transformed outline, by the definition of eq. 2 (rotation about the local origin, then shift)
    Pl = sc.verts.astype(np.float64)
    th, s = float(sc.params[0, 2]), float(sc.params[0, 3])
    R = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    Pw = (s * Pl) @ R.T + sc.params[0, :2].astype(np.float64)
    X, Y = np.meshgrid(np.arange(32) + 0.5, np.arange(32) + 0.5)
    w = _winding(Pw, X.ravel(), Y.ravel())
    inside = np.abs(w) > 0.5
    assert np.array_equal(sd > 0, inside)


# --------------------------------------------------------------------------------------------------
# Coverage and the five loss terms against 1-D quadrature (circle) and closed forms
# --------------------------------------------------------------------------------------------------
def _circle_scene(radius, mask="none", copies=1, centre=(32.31, 31.73), size=64, **kw):
    P, area, r_eff = _fine_circle(radius)
    params = np.array([[centre[0], centre[1], 0.0, 1.0]] * copies)
    sc = S.multi_shape_scene([P] * copies, params, size, size, mask=mask, **kw)
    return sc, area, r_eff


def test_P1_area_closed_form_fine_polygon():
    """sum_p alpha = A + pi^3 tau^2 / 3 for a smooth convex outline (coarea with offset-curve length)."""
    P, area, _ = _fine_circle(15.0)

    def f(c):
        sc = S.single_shape_scene(P, 64, 64, c, 0.0, 1.0, w_overlap=0, w_contain=1, w_fill=0)
        return Oracle(sc).forward(sc.params)[2][0, 1]

    excess = math.pi ** 3 * TAU ** 2 / 3
    val = _offset_average(f, (31.9, 31.3))
    assert abs(val - (area + excess)) < 2e-4, (val, area + excess)


@pytest.mark.parametrize("n,angle", [(4, 0.4363), (3, 1.1), (6, 0.2), (4, 0.0)])
def test_P1_area_closed_form_convex_polygon(n, angle):
    """Convex polygon: sum alpha = A + (pi^2 tau^2 / 12) (2 pi + sum_m 2 cot(phi_m / 2)).

    Replacing the Euclidean distance by the largest half-plane distance would move the value by
    (pi^2 tau^2 / 12) (sum 2 cot - 2 pi) = 0.13 .. 0.85 here; the tolerance is 5e-3."""
    R = 11.0
    P = S.regular_polygon(n, R)
    area = 0.5 * n * R ** 2 * math.sin(2 * math.pi / n)
    phi = math.pi * (n - 2) / n
    excess = (math.pi ** 2 * TAU ** 2 / 12) * (2 * math.pi + n * 2 / math.tan(phi / 2))

    def f(c):
        sc = S.single_shape_scene(P, 48, 48, c, angle, 1.0, w_overlap=0, w_contain=1, w_fill=0)
        return Oracle(sc).forward(sc.params)[2][0, 1]

    val = _offset_average(f, (23.9, 23.3))
    assert abs(val - (area + excess)) < 5e-3, (val, area + excess)


def test_P2_subpixel_translation_invariance():
    P = S.regular_polygon(256, 15.0)
    perim = 256 * 2 * 15.0 * math.sin(math.pi / 256)
    rng = np.random.default_rng(0)
    vals = []
    for _ in range(16):
        off = rng.uniform(0, 1, 2)
        sc = S.single_shape_scene(P, 48, 48, (24 + off[0], 24 + off[1]), 0.3, 1.0, w_contain=1)
        vals.append(Oracle(sc).forward(sc.params)[2][0, 1])
    assert (max(vals) - min(vals)) <= 3e-4 * perim


def test_loss_terms_against_radial_quadrature():
    """Every loss term of a (fine) disk against an independent 2-D -> 1-D radial integral."""
    r = 12.0
    H = 64
    P, _, r_eff = _fine_circle(r)
    upper = r_eff + R_CUT + 5.0

    def terms(mask, copies=1):
        def f(c):
            params = np.array([[c[0], c[1], 0.0, 1.0]] * copies)
            sc = S.multi_shape_scene([P] * copies, params, H, H, mask=mask, w_overlap=1, w_contain=1,
                                     w_fill=1, w_pad=1, w_down=1, r_pad=2.0)
            return Oracle(sc).forward(sc.params)[2][0]
        return f

    base = (31.9, 31.3)
    cy = base[1] + 0.5  # mean centre height over the offset grid
    # full mask: no containment loss, fill = sum (1 - S)^2; zero mask: containment = sum S
    L = _offset_average(terms("full"), base)
    I_alpha = _radial_integral(lambda sd: _alpha(sd), r_eff, upper)
    I_fill = _radial_integral(lambda sd: 1.0 - (1.0 - _alpha(sd)) ** 2, r_eff, upper)
    assert L[0] == 0.0  # one item never overlaps itself
    assert abs(L[1]) < 1e-12
    assert abs(L[2] - (H * H - I_fill)) < 2e-3, (L[2], H * H - I_fill)
    assert L[3] == 0.0  # a single item's padded coverage never exceeds 1
    assert abs(L[4] - (H - cy) * I_alpha) < 2e-2, (L[4], (H - cy) * I_alpha)
    L0 = _offset_average(terms("none"), base)
    assert abs(L0[1] - I_alpha) < 2e-4, (L0[1], I_alpha)
    # coincident pair: overlap and padding terms
    L2 = _offset_average(terms("none", copies=2), base)
    I_ov = _radial_integral(lambda sd: np.maximum(2 * _alpha(sd) - 1, 0) ** 2, r_eff, upper)
    I_pad = _radial_integral(lambda sd: np.maximum(2 * _alpha(sd, shift=2.0) - 1, 0) ** 2, r_eff, upper)
    assert abs(L2[0] - I_ov) < 2e-3, (L2[0], I_ov)
    assert abs(L2[3] - I_pad) < 2e-3, (L2[3], I_pad)
    # and the leading terms of the analytic expansion A - 2 tau P + 8 pi tau^2 ln 2
    A, Pm = math.pi * r_eff ** 2, 2 * math.pi * r_eff
    assert abs(L2[0] - (A - 2 * TAU * Pm + 8 * math.pi * TAU ** 2 * math.log(2))) < 5e-2


# --------------------------------------------------------------------------------------------------
# Gradient pins
# --------------------------------------------------------------------------------------------------
def test_P3_scale_derivative_is_twice_area_over_s():
    P = S.regular_polygon(128, 9.0)
    area = 0.5 * 128 * 81.0 * math.sin(2 * math.pi / 128)
    s = 1.3
    sc = S.single_shape_scene(P, 48, 48, (24.21, 23.67), 0.2, s, w_overlap=0, w_contain=1, w_fill=0)
    g = Oracle(sc).backward(sc.params, dloss=[0, 1, 0, 0, 0, 0, 0, 0, 0])
    assert abs(g[0, 3] - 2 * area * s) / (2 * area * s) < 1e-3  # d(s^2 A)/ds
    # translation and rotation leave the total coverage unchanged
    assert abs(g[0, 0]) < 2e-3 * area and abs(g[0, 1]) < 2e-3 * area and abs(g[0, 2]) < 2e-3 * area


def test_P4_gravity_identity():
    """dL_down/dt_y = -k sum_p alpha (moving an item down lowers its potential by its mass)."""
    P = S.regular_polygon(128, 8.0)

    def f(c):
        sc = S.single_shape_scene(P, 48, 48, c, 0.2, 1.0, w_overlap=0, w_contain=1, w_fill=0, w_down=1.0)
        o = Oracle(sc)
        mass = o.forward(sc.params)[2][0, 1]
        g = o.backward(sc.params, dloss=[0, 0, 0, 0, 1, 0, 0, 0, 0])[0]
        return np.array([mass, g[0], g[1]])

    mass, gx, gy = _offset_average(f, (23.9, 20.3))
    assert abs(gy + mass) / mass < 2e-4, (gy, mass)
    assert abs(gx) < 2e-4 * mass


def test_P5_pair_disjoint_zero_overlap_and_padding_threshold():
    R = 6.0
    hexa = S.regular_polygon(12, R)
    d = np.array([math.cos(0.7), math.sin(0.7)])
    c0 = np.array([20.13, 21.37])
    for gap in (0.2, 1.0):
        c1 = c0 + d * (2 * R + gap)
        sc = S.multi_shape_scene([hexa, hexa], np.array([[*c0, 0.1, 1], [*c1, 0.5, 1]]), 48, 48,
                                 w_overlap=1, w_contain=0, w_fill=0, w_pad=1, r_pad=2.0)
        S_, _, L = Oracle(sc).forward(sc.params)
        assert L[0, 0] == 0.0 and S_.max() < 1.0
    # padding: gap >= 2 r_pad gives exactly zero, a 3 px gap between facing squares does not
    sq = S.rectangle(5.0, 5.0)
    for gap, zero in ((4.5, True), (3.0, False)):
        sc = S.multi_shape_scene([sq, sq], np.array([[15.13, 20.37, 0, 1], [15.13 + 10 + gap, 20.37, 0, 1]]),
                                 48, 40, w_overlap=1, w_contain=0, w_fill=0, w_pad=1, r_pad=2.0)
        L = Oracle(sc).forward(sc.params)[2]
        assert L[0, 0] == 0.0
        assert (L[0, 3] == 0.0) == zero, (gap, L[0, 3])


def test_P6_symmetry_zeros():
    sc = S.single_shape_scene(S.rectangle(5.25, 3.0), 64, 64, (32.0, 32.0), 0.0, 1.0, mask="disk",
                              w_overlap=1, w_contain=1, w_fill=1, w_pad=1, r_pad=2.0, w_down=0.0)
    g = Oracle(sc).backward(sc.params)
    scale = np.abs(g[0, 3]) + 1.0
    assert abs(g[0, 0]) < 1e-9 * scale and abs(g[0, 1]) < 1e-9 * scale and abs(g[0, 2]) < 1e-9 * scale


def _fd_check(sc, tol=1e-4, shapes=None):
    o = Oracle(sc)
    g = o.backward(sc.params)
    fd = o.fd_gradient(sc.params, shapes=shapes)
    sel = list(range(sc.num_shapes)) if shapes is None else list(shapes)
    for c in range(4):
        ref = fd[sel, c]
        floor = 0.01 * np.abs(ref).max()
        err = np.abs(g[sel, c] - ref)
        assert np.all(err <= tol * np.maximum(np.abs(ref), floor) + 1e-9), (c, err.max(), ref)


def test_P7_backward_vs_central_differences_three_items():
    rng = np.random.default_rng(1)
    outlines = [S.star_polygon(6, 7.0, 0.5), S.regular_polygon(9, 6.0), S.jittered_bezier(rng, 5, 6.0)]
    params = np.array([[20.3, 22.1, 0.3, 1.0], [27.7, 25.9, 1.2, 1.1], [23.4, 31.2, 2.1, 0.9]])
    sc = S.multi_shape_scene(outlines, params, 48, 48, mask="disk", w_overlap=1, w_contain=1, w_fill=1,
                             w_pad=1, r_pad=2.0, w_down=1e-3)
    _fd_check(sc)


def test_P7_backward_vs_central_differences_config1():
    _fd_check(S.config1(), shapes=[0, 3, 6])


def test_P7_backward_vs_central_differences_two_layouts():
    sc = S.random_scene(5, [(37, 29), (26, 41)], [3, 2], radius=(3.0, 7.0), off_canvas=0.3)
    _fd_check(sc)


def test_P8_adam_matches_torch():
    import torch

    sc = S.config1()
    o = Oracle(sc)
    g = o.backward(sc.params)
    lr = o.learning_rates()
    p0 = sc.params.astype(np.float64)
    # oracle: two steps with the same gradient
    p, m, v = o.adam(p0, g, np.zeros_like(g), np.zeros_like(g), 1, lr)
    p, m, v = o.adam(p, g, m, v, 2, lr)
    # torch: one parameter group per (item, component) with its own learning rate
    params = [torch.tensor(p0[i, c], dtype=torch.float64, requires_grad=True)
              for i in range(p0.shape[0]) for c in range(4)]
    opt = torch.optim.Adam([{"params": [t], "lr": float(lr.reshape(-1)[j])} for j, t in enumerate(params)],
                           betas=(0.9, 0.999), eps=1e-8)
    for _ in range(2):
        for j, t in enumerate(params):
            t.grad = torch.tensor(g.reshape(-1)[j], dtype=torch.float64)
        opt.step()
    pt = np.array([t.item() for t in params]).reshape(-1, 4)
    np.testing.assert_allclose(p, pt, rtol=1e-12, atol=1e-12)


def test_learning_rate_units():
    sc = S.config3() if False else S.random_scene(2, [(40, 40)], [3])
    o = Oracle(sc, level=None)
    lr = o.learning_rates(0.5)
    np.testing.assert_allclose(lr[:, 0], 0.5)
    np.testing.assert_allclose(lr[:, 2], 0.5 / sc.rho.astype(np.float64))


# --------------------------------------------------------------------------------------------------
# Cut-off and culling
# --------------------------------------------------------------------------------------------------
def test_P9_cutoff_and_bbox_culling():
    sc = S.random_scene(7, [(30, 26)], [5], radius=(3.0, 6.0))
    exact = Oracle(sc, use_cutoff=True, use_bbox=False)
    culled = Oracle(sc, use_cutoff=True, use_bbox=True)
    nocut = Oracle(sc, use_cutoff=False, use_bbox=False)
    Se, Spe, Le = exact.forward(sc.params)
    Sc, Spc, Lc = culled.forward(sc.params)
    Sn, Spn, _ = nocut.forward(sc.params)
    assert np.array_equal(Se, Sc) and np.array_equal(Spe, Spc) and np.array_equal(Le, Lc)
    bound = 5 * _sigmoid(-R_CUT / TAU)
    assert np.abs(Sn - Se).max() <= bound and np.abs(Spn - Spe).max() <= bound
    assert np.abs(Sn - Se).max() > 0  # the cut-off does remove the far tail
    np.testing.assert_array_equal(exact.backward(sc.params), culled.backward(sc.params))


def test_empty_and_offcanvas_items():
    sc = S.random_scene(11, [(20, 17)], [2], radius=(3.0, 4.0))
    p = sc.params.copy()
    p[:, 0] = [-50.0, 90.0]  # both far off the canvas
    o = Oracle(sc)
    S_, Sp, L = o.forward(p)
    assert S_.max() == 0.0 and L[0, 0] == 0 and L[0, 1] == 0 and L[0, 4] == 0
    assert L[0, 2] == pytest.approx(sc.w_fill * sc.masks()[0].sum())
    assert np.all(o.backward(p) == 0.0)


# --------------------------------------------------------------------------------------------------
# Open items: a polyline thickened by a disk of radius w (transformed with the item)
# --------------------------------------------------------------------------------------------------
def _stadium(L, w, c, theta, s=1.0, size=48):
    seg = np.array([[-L / 2, 0.0], [L / 2, 0.0]])
    return S.multi_shape_scene([seg], np.array([[c[0], c[1], theta, s]]), size, size, stroke=[w],
                               w_overlap=0, w_contain=1, w_fill=0)


def test_open_segment_distance_closed_form():
    """sd = s w - dist(p, segment): in the segment's frame, dist = hypot(max(|x'| - s L / 2, 0), y')."""
    L, w, th, s, c = 14.6, 1.7, 0.37, 1.2, (23.41, 22.73)
    sc = _stadium(L, w, c, th, s)
    sd = Oracle(sc).signed_distance(sc.params)[0].reshape(48, 48)
    t = sc.params[0].astype(np.float64)
    j, i = np.mgrid[0:48, 0:48]
    dx, dy = i + 0.5 - t[0], j + 0.5 - t[1]
    xr = math.cos(t[2]) * dx + math.sin(t[2]) * dy
    yr = -math.sin(t[2]) * dx + math.cos(t[2]) * dy
    # the scene stores the end points and the half-width as float32
    half, wf = float(sc.verts[1, 0]), float(sc.stroke[0])
    assert float(sc.verts[0, 0]) == -half and float(sc.verts[0, 1]) == 0.0 == float(sc.verts[1, 1])
    ref = t[3] * wf - np.hypot(np.maximum(np.abs(xr) - t[3] * half, 0.0), yr)
    assert np.abs(sd - ref).max() < 1e-9


def test_open_P1_stadium_area_closed_form():
    """sum_p alpha = 2 w L + pi w^2 + pi^3 tau^2 / 3: the inner and outer parallel bodies of a stadium
    have perimeters P -/+ 2 pi x, as for a smooth convex outline."""
    L, w = 14.6, 6.0
    area = 2 * w * L + math.pi * w * w

    def f(c):
        sc = _stadium(L, w, c, 0.31)
        return Oracle(sc).forward(sc.params)[2][0, 1]

    val = _offset_average(f, (23.9, 23.3))
    excess = math.pi ** 3 * TAU ** 2 / 3
    assert abs(val - (area + excess)) < 1e-3, (val, area + excess)


def test_open_P3_scale_derivative():
    """d(sum alpha)/ds = 2 A s: the stroke radius scales with the item (a dropped d(k|s|w)/ds term
    fails this by 4 w (w + L) s)."""
    L, w, s = 14.6, 4.0, 1.3
    area = 2 * w * L + math.pi * w * w
    sc = _stadium(L, w, (24.21, 23.67), 0.2, s, size=64)
    g = Oracle(sc).backward(sc.params, dloss=[0, 1, 0, 0, 0, 0, 0, 0, 0])
    assert abs(g[0, 3] - 2 * area * s) / (2 * area * s) < 2e-3, (g[0, 3], 2 * area * s)
    assert abs(g[0, 0]) < 2e-3 * area and abs(g[0, 1]) < 2e-3 * area and abs(g[0, 2]) < 2e-3 * area


def test_open_P7_backward_vs_central_differences():
    sc = S.random_scene(12, [(56, 48)], [7], kinds=("open", "star", "open"), radius=(4.0, 9.0))
    assert sc.stroke is not None and (sc.stroke > 0).sum() >= 3
    _fd_check(sc)


# --------------------------------------------------------------------------------------------------
# Uniform (dilation) term: O = min(S, 1), A_j = box sum of O over (5 + 6 j)^2 windows (j < 4),
# L = sum_j (b_j / 5) sum_p M relu(1 - A_j)
# --------------------------------------------------------------------------------------------------
UNI_B = (5, 11, 17, 23)


def test_uniform_term_of_an_empty_layout():
    """No items: A_j = 0 everywhere, so the term is (sum_j b_j / 5) * sum_p M = 11.2 sum_p M."""
    sc = dataclasses.replace(S.random_scene(2, [(37, 29)], [0]), w_uniform=1.0)
    _, _, L = Oracle(sc).forward(sc.params)
    M = sc.packed_mask(None).astype(np.float64)
    assert abs(L[0, 5] - sum(b / 5 for b in UNI_B) * M.sum()) < 1e-9 * M.sum()


def test_uniform_term_matches_a_convolution():
    """The term recomputed from the oracle's S with scipy's 2-D convolution as the box sum."""
    from scipy.signal import convolve2d

    sc = dataclasses.replace(S.random_scene(5, [(61, 47)], [6], radius=(3.0, 7.0)), w_uniform=0.7)
    S_, _, L = Oracle(sc).forward(sc.params)
    O = np.minimum(S_.reshape(47, 61), 1.0)
    M = sc.packed_mask(None).astype(np.float64).reshape(47, 61)
    ref = 0.0
    for b in UNI_B:
        A = convolve2d(O, np.ones((b, b)), mode="same", boundary="fill", fillvalue=0.0)
        ref += (b / 5) * (M * np.maximum(1.0 - A, 0.0)).sum()
    assert ref > 1.0 and abs(L[0, 5] - 0.7 * ref) < 1e-10 * ref


def test_uniform_term_backward_vs_central_differences():
    sc = dataclasses.replace(S.random_scene(9, [(52, 44)], [5], radius=(3.0, 6.0)), w_uniform=3.0,
                             w_overlap=0.2, w_contain=0.2, w_fill=0.2)
    _fd_check(sc)


# --------------------------------------------------------------------------------------------------
# The paper's containment loss (eq. 5), the 1 / (w h) of eqs. 5-6, and the force variants of Sec. 5
# --------------------------------------------------------------------------------------------------
def test_wmse_closed_forms():
    """eq. 5 at its two extremes.  No items: the rendering is white (O = 0) and the container black, so
    the sum is the container's pixel count (penalty 1 inside).  One item far larger than the canvas
    covering it (S = 1 at every pixel): the pixels outside the container, at penalty 100."""
    W, H = 37, 29
    sc = S.multi_shape_scene([S.rectangle(2.0, 2.0)], np.array([[-500.0, -500.0, 0.0, 1.0]]), W, H, mask="disk",
                             w_overlap=0, w_contain=0, w_fill=0, w_wmse=1.0)
    M = sc.packed_mask(None).astype(np.float64)
    n_in = M.sum()
    assert 0 < n_in < W * H
    L = Oracle(sc).forward(sc.params)[2]
    assert abs(L[0, 6] - n_in) < 1e-9 * n_in
    big = dataclasses.replace(sc, params=np.array([[18.0, 14.0, 0.0, 1.0]], np.float32),
                              verts=S.rectangle(200.0, 200.0).astype(np.float32))
    Sb, _, Lb = Oracle(big).forward(big.params)
    assert np.all(Sb == 1.0)
    assert abs(Lb[0, 6] - 100.0 * (W * H - n_in)) < 1e-9 * Lb[0, 6]
    # the 1 / (w h) of eq. 5
    Lm = Oracle(dataclasses.replace(big, area_mean=True)).forward(big.params)[2]
    assert abs(Lm[0, 6] - Lb[0, 6] / (W * H)) < 1e-12 * Lb[0, 6]


def test_area_mean_scales_exactly_the_image_mismatch_terms():
    """With area_mean, overlap, contain, fill, pad and wmse (loss and gradient) are divided by each
    layout's own pixel count; down, uniform, centre and objdown are unchanged."""
    sc = dataclasses.replace(S.random_scene(4, [(41, 33), (26, 30)], [6, 4], radius=(3.0, 7.0)), w_uniform=0.3,
                             w_wmse=2.0, w_centre=0.01, w_objdown=0.5)
    o, om = Oracle(sc), Oracle(dataclasses.replace(sc, area_mean=True))
    L, Lm = o.forward(sc.params)[2], om.forward(sc.params)[2]
    areas = np.array([41 * 33, 26 * 30], np.float64)
    for t in range(9):
        f = 1.0 / areas if t in (0, 1, 2, 3, 6) else np.ones(2)
        assert np.all(np.abs(Lm[:, t] - L[:, t] * f) <= 1e-12 * np.abs(L[:, t]) + 1e-300), t
    for t in (1, 6, 7):
        dl = np.zeros((2, 9))
        dl[:, t] = 1.0
        g, gm = o.backward(sc.params, dloss=dl), om.backward(sc.params, dloss=dl)
        f = np.repeat(1.0 / areas if t != 7 else np.ones(2), [6, 4])[:, None]
        assert np.allclose(gm, g * f, rtol=1e-12, atol=0.0), t


def test_centre_force_against_quadrature():
    """sum_p S |p - c| (c the canvas centre) for a fine disk whose centre is 11.3 px from c, against the
    2-D integral in polar coordinates about the disk centre; sub-pixel offsets averaged."""
    r, D, side = 8.0, 11.3, 64
    P, _, r_eff = _fine_circle(r)
    c = side / 2.0
    upper = r_eff + R_CUT + 5.0

    def f(pos):
        sc = S.multi_shape_scene([P], np.array([[pos[0], pos[1], 0.0, 1.0]]), side, side, mask="none",
                                 w_overlap=0, w_contain=0, w_fill=0, w_centre=1.0)
        return Oracle(sc).forward(sc.params)[2][0]

    base = (c + D - 0.5, c - 0.5)
    L = _offset_average(f, base)

    def ring(rho):  # int_0^{2 pi} |rho (cos phi, sin phi) + (D, 0)| d phi
        v, _ = integrate.quad(lambda ph: math.hypot(D + rho * math.cos(ph), rho * math.sin(ph)), 0.0, 2 * math.pi,
                              limit=200, epsabs=1e-11, epsrel=1e-11)
        return v

    pts = sorted({0.0, max(r_eff - 6, 0.0), r_eff, r_eff + 2.0, r_eff + R_CUT, upper})
    ref = 0.0
    for a, b in zip(pts[:-1], pts[1:]):
        v, _ = integrate.quad(lambda rho: _alpha(r_eff - rho) * rho * ring(rho), a, b, limit=200, epsabs=1e-9,
                              epsrel=1e-10)
        ref += v
    # the offset average moves the disk by up to half a pixel about its mean centre; L is smooth in the
    # position, so that leaves a second-order bias well below the bound
    assert abs(L[7] - ref) < 2e-3 * ref, (L[7], ref)
    assert L[0] == 0.0 and L[6] == 0.0 and L[8] == 0.0


def test_object_space_downward_force():
    """sum_i (H - k t_y,i) exactly, and its gradient -k w on t_y only, at a level with k != 1."""
    sc = dataclasses.replace(S.config4(2, num_layouts=3), w_overlap=0.0, w_contain=0.0, w_fill=0.0, w_pad=0.0,
                             w_down=0.0, w_objdown=0.7)
    level = sc.levels[0]
    o = Oracle(sc, level=level)
    w, h, k, off = sc.layout_arrays(level)
    assert k[0] != 1.0
    L = o.forward(sc.params)[2]
    p = sc.params.astype(np.float64)
    for b in range(sc.num_layouts):
        ref = 0.7 * sum(float(h[b]) - float(k[b]) * p[q, 1] for q in range(off[b], off[b + 1]))
        assert abs(L[b, 8] - ref) < 1e-12 * abs(ref)
    g = o.backward(sc.params)
    for b in range(sc.num_layouts):
        assert np.all(g[off[b]:off[b + 1], 1] == -0.7 * float(k[b]))
    assert np.all(g[:, [0, 2, 3]] == 0.0)


def test_new_terms_backward_vs_central_differences():
    sc = dataclasses.replace(S.random_scene(21, [(52, 44)], [5], radius=(3.0, 6.0)), w_overlap=0.5, w_contain=0.0,
                             w_fill=0.0, w_pad=0.0, w_down=0.0, w_wmse=1.0, w_centre=0.05, w_objdown=0.3,
                             area_mean=True)
    _fd_check(sc)


def test_paper_preset():
    sc = S.paper_loss_preset(S.config1())
    assert sc.weights() == (8e4, 0.0, 0.0, 0.0, 0.0, 5e-4, 3e3, 0.0, 0.0) and sc.area_mean


# --------------------------------------------------------------------------------------------------
# Outline (control-point) gradients: dL / d(vertex in the item frame)
# --------------------------------------------------------------------------------------------------
def test_vertex_gradient_vs_central_differences():
    """Closed and open items, vertices at corners and mid-outline, every loss term on."""
    sc = dataclasses.replace(S.random_scene(12, [(56, 48)], [7], kinds=("open", "star", "poly", "bezier"),
                                            radius=(4.0, 9.0)), w_uniform=0.5, w_wmse=0.5, w_centre=0.01)
    o = Oracle(sc)
    _, gv = o.backward_vertices(sc.params)
    rng = np.random.default_rng(5)
    verts = sorted(rng.choice(sc.num_verts, 14, replace=False).tolist())
    fd = o.fd_vertex_gradient(sc.params, verts)
    floor = 0.01 * np.abs(gv).max()
    err = np.abs(gv[verts] - fd)
    assert np.all(err <= 1e-4 * np.maximum(np.abs(fd), floor)), (err.max(), fd)


def test_vertex_gradient_sums_to_the_parameter_gradient():
    """v' = k (R s v + t): dL/dt = R sum_m g_m / s, dL/dtheta = sum_m v_m x g_m and, for a closed item,
    dL/ds = sum_m v_m . g_m / s, with g_m = dL/dv_m."""
    sc = S.config1()
    o = Oracle(sc)
    g, gv = o.backward_vertices(sc.params)
    V = sc.verts.astype(np.float64)
    for q in range(sc.num_shapes):
        a, b = sc.vert_off[q], sc.vert_off[q + 1]
        th, s = float(sc.params[q, 2]), float(sc.params[q, 3])
        R = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
        gm, vm = gv[a:b], V[a:b]
        scale = np.abs(g[q]).max()
        assert np.allclose(R @ gm.sum(0) / s, g[q, :2], rtol=0, atol=1e-9 * scale)
        assert abs((vm[:, 0] * gm[:, 1] - vm[:, 1] * gm[:, 0]).sum() - g[q, 2]) <= 1e-9 * scale
        assert abs((vm * gm).sum() / s - g[q, 3]) <= 1e-9 * scale


# --------------------------------------------------------------------------------------------------
# The update of eq. 4 at a level with k != 1: learning rates in level pixels (large coarse steps)
# --------------------------------------------------------------------------------------------------
def _eq2_vertices(sc, p, k):
    """Transformed vertices of every item, level px (eq. 2 with a uniform scale), for the pin below."""
    out = []
    V = sc.verts.astype(np.float64)
    for q in range(sc.num_shapes):
        a, b = sc.vert_off[q], sc.vert_off[q + 1]
        c, s_ = math.cos(p[q, 2]), math.sin(p[q, 2])
        R = np.array([[c, -s_], [s_, c]])
        out.append(k * (p[q, 3] * V[a:b] @ R.T + p[q, :2]))
    return out


@pytest.mark.parametrize("level", [128, 256, 1024])
def test_first_adam_step_moves_every_item_by_lr_px_level_pixels(level):
    """Adam's first step is lr sign(g) (to eps / |g|).  With the learning rates read in level pixels,
    one step at a level of scale k != 1 moves every item's origin by exactly lr_px level px per axis,
    and its rim point (the vertex at radius rho) by lr_px level px along its arc under theta alone and
    along its ray under s alone, whatever k and rho are.  Learning rates of lr_px * k or lr_px / rho
    without k fail this at every level here."""
    sc = S.config3(0)
    o = Oracle(sc, level=level)
    k = level / sc.level_ref
    assert k != 1.0
    lr_px = sc.lr_px
    rng = np.random.default_rng(level)
    p0 = sc.params.astype(np.float64)
    g = rng.choice([-1.0, 1.0], p0.shape) * rng.uniform(1.0, 10.0, p0.shape)
    z = np.zeros_like(p0)
    p1, _, _ = o.adam(p0, g, z, z, 1, o.learning_rates(lr_px))
    before = _eq2_vertices(sc, p0, k)
    rim = [int(np.argmax(np.hypot(*sc.verts[sc.vert_off[q]:sc.vert_off[q + 1]].astype(np.float64).T)))
           for q in range(sc.num_shapes)]
    # translation alone: every vertex (and the origin) moves by lr_px level px per axis
    pt = p0.copy()
    pt[:, :2] = p1[:, :2]
    for q, (va, vb) in enumerate(zip(before, _eq2_vertices(sc, pt, k))):
        np.testing.assert_allclose(np.abs(vb - va), lr_px, rtol=1e-6)
        assert np.all(np.sign(vb - va)[0] == -np.sign(g[q, :2]))
    # rotation alone: the rim point travels lr_px level px along its circle about the origin k t
    pr = p0.copy()
    pr[:, 2] = p1[:, 2]
    for q, (va, vb) in enumerate(zip(before, _eq2_vertices(sc, pr, k))):
        ra, rb = va[rim[q]] - k * p0[q, :2], vb[rim[q]] - k * p0[q, :2]
        turn = math.atan2(ra[0] * rb[1] - ra[1] * rb[0], ra @ rb)
        assert abs(abs(turn) * np.hypot(*ra) - lr_px) < 1e-6 * lr_px, (q, turn, np.hypot(*ra))
    # scale alone: the rim point moves lr_px level px along its ray
    ps = p0.copy()
    ps[:, 3] = p1[:, 3]
    for q, (va, vb) in enumerate(zip(before, _eq2_vertices(sc, ps, k))):
        assert abs(np.hypot(*(vb[rim[q]] - va[rim[q]])) - lr_px) < 1e-6 * lr_px


# --------------------------------------------------------------------------------------------------
# Open items of several segments: no closing segment, right-angle joins
# --------------------------------------------------------------------------------------------------
U_SIDE = 24.0


def _u_scene(w, theta, s=1.0, c=(31.37, 30.81), size=64):
    """A U: three segments of length U_SIDE with two right-angle joins; the mouth is open."""
    U = np.array([[0.0, U_SIDE], [0.0, 0.0], [U_SIDE, 0.0], [U_SIDE, U_SIDE]])
    return S.multi_shape_scene([U], np.array([[c[0], c[1], theta, s]]), size, size, stroke=[w],
                               w_overlap=0, w_contain=1, w_fill=0)


def test_open_polyline_distance_in_the_mouth_of_a_u():
    """Inside the U's mouth (item frame, arms at x = -/+ s a, base at y = -s a, mouth at y = +s a, with
    a = U_SIDE / 2) the distance to the polyline is min(x + s a, s a - x, y + s a): the open side is no
    segment.  A closing segment from the last vertex to the first would cap it by s a - y."""
    w, th, s = 1.3, 0.41, 1.1
    sc = _u_scene(w, th, s)
    sd = Oracle(sc).signed_distance(sc.params)[0].reshape(64, 64)
    t = sc.params[0].astype(np.float64)
    j, i = np.mgrid[0:64, 0:64]
    dx, dy = i + 0.5 - t[0], j + 0.5 - t[1]
    xr = math.cos(t[2]) * dx + math.sin(t[2]) * dy
    yr = -math.sin(t[2]) * dx + math.cos(t[2]) * dy
    s = t[3]  # the scene's float32 values
    a = s * float(sc.verts[3, 0])
    assert float(sc.verts[3, 0]) == -float(sc.verts[0, 0]) == float(sc.verts[0, 1]) == -float(sc.verts[1, 1])
    mouth = (np.abs(xr) < a) & (yr > -a) & (yr < a)
    ref = s * float(sc.stroke[0]) - np.minimum(np.minimum(xr + a, a - xr), yr + a)
    assert mouth.sum() > 300
    assert np.abs(sd[mouth] - ref[mouth]).max() < 1e-9
    # the pixels nearest the mouth line are far from any segment (a closing segment would be within 1 px)
    near_mouth = mouth & (yr > a - 1.0) & (np.abs(xr) < a / 2)
    assert near_mouth.sum() > 5 and np.all(sd[near_mouth] < -(a / 2 - 2.0))


def test_open_polyline_u_area_closed_form():
    """sum_p alpha of a stroked U by the coarea formula: the level set at distance x outside is the
    boundary of the U stroked to half-width w + x, at depth x < w inside that of half-width w - x, and
    a U stroked to half-width y (no merging of the arms, y < U_SIDE / 2) has the area
        A(y) = 2 y (3 L) + pi y^2 - 2 y^2 (1 - pi / 4)
    (three rectangles, two end caps, and per right-angle join a quarter disk outside minus a y x y
    square counted twice inside), so the perimeter A'(y).  The expected sum is
        A(w) + int_0^r_cut sigma(-x / tau) A'(w + x) dx - int_0^w sigma(-x / tau) A'(w - x) dx,
    by 1-D quadrature.  A closing segment adds 2 w L = 120 px^2."""
    w, L = 2.5, U_SIDE
    assert w + R_CUT < L / 2

    def A(y):
        return 2 * y * 3 * L + math.pi * y * y - 2 * y * y * (1 - math.pi / 4)

    def Ap(y):
        return 6 * L + 2 * math.pi * y - 4 * y * (1 - math.pi / 4)

    out, _ = integrate.quad(lambda x: _sigmoid(-x / TAU) * Ap(w + x), 0.0, R_CUT, epsabs=1e-12, limit=200)
    inn, _ = integrate.quad(lambda x: _sigmoid(-x / TAU) * Ap(w - x), 0.0, w, epsabs=1e-12, limit=200)
    expect = A(w) + out - inn

    def f(c):
        sc = _u_scene(w, 0.29, 1.0, c=c)
        return Oracle(sc).forward(sc.params)[2][0, 1]

    val = _offset_average(f, (31.9, 31.3))
    assert abs(val - expect) < 2e-3 * Ap(w), (val, expect)


# --------------------------------------------------------------------------------------------------
# Quality metrics of Sec. 6 on hard rasters (test tooling): pixel counts of axis-aligned rectangles
# --------------------------------------------------------------------------------------------------
def _centres_in(lo, hi):
    """Number of pixel centres i + 1/2 in [lo, hi] (generic end points: none on a centre)."""
    return max(0, math.floor(hi - 0.5) - math.ceil(lo - 0.5) + 1)


def test_quality_metrics_count_pixels_of_rectangles():
    """Target: an axis-aligned rectangle container; items: three axis-aligned rectangles, two of them
    overlapping and one reaching out of the container.  LC, OO and EA are ratios of pixel-centre
    counts of intervals, which are exact integers here."""
    W, H = 60, 50
    box = (30.3, 24.7, 21.2, 17.9)  # container centre and half-sides
    rects = [((20.2, 20.6), (6.3, 4.1)), ((27.1, 23.3), (5.2, 7.7)), ((47.6, 38.4), (6.9, 5.3))]
    outlines = [S.rectangle(hw, hh) for _, (hw, hh) in rects]
    params = np.array([[c[0], c[1], 0.0, 1.0] for c, _ in rects])
    lay = S.Layout(W, H, 0, 3, rects=np.array([[box[0], box[1], box[2], box[3], 0.0]]))
    sc = S.assemble("quality", outlines, params, [lay], [1], 1)
    # the values the oracle sees (float32 storage)
    P = sc.params.astype(np.float64)
    half = [np.abs(sc.verts[sc.vert_off[q]:sc.vert_off[q + 1]].astype(np.float64)).max(0) for q in range(3)]
    ivx = [(P[q, 0] - half[q][0], P[q, 0] + half[q][0]) for q in range(3)]
    ivy = [(P[q, 1] - half[q][1], P[q, 1] + half[q][1]) for q in range(3)]
    bx, by = (box[0] - box[2], box[0] + box[2]), (box[1] - box[3], box[1] + box[3])

    def cnt(x, y):
        return _centres_in(*x) * _centres_in(*y)

    def cap(u, v):
        return (max(u[0], v[0]), min(u[1], v[1]))

    target = cnt(bx, by)
    # pixels of each item, of the overlap of items 0 and 1, and of each item inside the container
    n = [cnt(ivx[q], ivy[q]) for q in range(3)]
    ov = cnt(cap(ivx[0], ivx[1]), cap(ivy[0], ivy[1]))
    inside = [cnt(cap(ivx[q], bx), cap(ivy[q], by)) for q in range(3)]
    ov_in = cnt(cap(cap(ivx[0], ivx[1]), bx), cap(cap(ivy[0], ivy[1]), by))
    assert ov > 0 and n[2] > inside[2] > 0 and cnt(cap(ivx[2], ivx[1]), cap(ivy[2], ivy[1])) == 0
    covered_in = sum(inside) - ov_in
    covered_out = sum(n) - ov - covered_in
    m, c = Oracle(sc).quality(sc.params)
    assert list(c[0]) == [target, covered_in, ov, covered_out]
    np.testing.assert_allclose(m[0], [covered_in / target, ov / target, covered_out / target], rtol=1e-15)


# --------------------------------------------------------------------------------------------------
# The workload with 8 items on 64 x 64: 200 Adam steps of the oracle end in a packed layout
# --------------------------------------------------------------------------------------------------
def test_config1_two_hundred_adam_steps_reach_a_packed_layout():
    """Sec. 4 (Fig. 2): 200 epochs of forward, backward and the update.  Layouts are local minima,
    not unique, so the end state is checked by bands of the Sec. 6 metrics: the loss falls by more
    than 5x, the items cover over 80% of the disk, and overlap and excess stay under 5% of it.  (The
    seed-0 start covers 17%.)"""
    sc = S.config1(0)
    o = Oracle(sc)
    p = sc.params.astype(np.float64)
    m, v = np.zeros_like(p), np.zeros_like(p)
    lr = o.learning_rates()
    L0 = o.loss(p)
    q0, _ = o.quality(p)
    for t in range(1, 201):
        p, m, v = o.adam(p, o.backward(p), m, v, t, lr)
    L1 = o.loss(p)
    q1, _ = o.quality(p)
    assert L1 < L0 / 5, (L0, L1)
    assert q0[0, 0] < 0.3 and q1[0, 0] > 0.8 and q1[0, 1] < 0.05 and q1[0, 2] < 0.05, (q0, q1)


def test_nearest_ambiguity_is_the_gradient_jump_across_a_medial_axis():
    """An axis-aligned 20.6 x 4.5 rectangle centred on a pixel centre: the pixels of its middle row between
    the short edges are equidistant from the two long edges, which are not neighbours, so the gradient
    jumps there (the row sits on the outline's medial axis).  Moving the item by +-1e-9 px in y breaks
    every tie the same way: the t_y bound must equal the jump of the oracle's own gradient, and t_x and s
    must have none (the normals are vertical; the two nearest points are mirror images).  theta's terms
    flip sign with the pixel's column, so its bound is the sum of their sizes, 2 omega k |dx| per pixel, while
    its jump cancels.  (Half-width minus half-height is not an integer, so no corner bisector meets a pixel
    centre, and no edge passes through one.)"""
    sc = S.single_shape_scene(S.rectangle(10.3, 2.25), 64, 64, t=(32.5, 32.5))
    o = Oracle(sc)
    p = sc.params.astype(np.float64)
    b = o.nearest_ambiguity(p, 0.0, 0.0)[0]
    eps = 1e-9
    gp = o.backward(p + np.array([[0.0, eps, 0.0, 0.0]]))[0]
    gm = o.backward(p - np.array([[0.0, eps, 0.0, 0.0]]))[0]
    assert b[1] > 0.5
    assert abs(b[1] - abs(gp[1] - gm[1])) <= 1e-6 * b[1]
    assert b[0] <= 1e-12 and b[3] <= 1e-12
    assert abs(gp[2] - gm[2]) <= 1e-9 * b[2]
    # theta: the row's pixels within the long edges' reach, each 2 omega |dx| (k = 1, omega the same for all)
    omega = b[1] / (2.0 * 17)  # 17 pixels (|dx| <= 8) carry the t_y jump of 2 omega each
    assert abs(b[2] - sum(2.0 * omega * abs(dx) for dx in range(-8, 9))) <= 1e-9 * b[2]


def test_nearest_ambiguity_needs_a_rival_within_the_resolution():
    """The same rectangle 1e-5 px off the tie: the middle row's long edges are 2e-5 px apart in distance, so
    they count at a resolution of 3e-5 px and not at 1e-5 px; generic layouts have no such pixel."""
    sc = S.single_shape_scene(S.rectangle(10.3, 2.25), 64, 64, t=(32.5, 32.5))
    o = Oracle(sc)
    p = sc.params.astype(np.float64) + np.array([[0.0, 1e-5, 0.0, 0.0]])
    assert o.nearest_ambiguity(p, 3e-5, 0.0)[0, 1] > 0.5
    assert not np.any(o.nearest_ambiguity(p, 1e-5, 0.0))
    for sc in (S.config1(0), S.config2(0)):
        assert not np.any(Oracle(sc).nearest_ambiguity(sc.params, 2.0 ** -20, 2.0 ** -20))
