"""GPU (HIP, through the C ABI) vs the FP64 oracle, element by element, on seeded scenes.

Every case prints its name before touching the GPU so that a failing run names it.
"""
import dataclasses
import math
import sys

import numpy as np
import pytest
import torch

from oracle.oracle import Oracle
from paper_2406_04008_amd import _lib
from paper_2406_04008_amd import scenes as S
from paper_2406_04008_amd.collage import CollageLoss, CollageScene, Timer
from tests.parity_util import check_grad, check_image, check_loss, check_vgrad, grad_error

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _np(t):
    return t.detach().cpu().numpy()


SCENES = {
    "config1": lambda: S.config1(0),
    "ragged": lambda: S.random_scene(3, [(37, 29), (50, 61), (16, 16), (23, 9)], [4, 9, 1, 0], off_canvas=0.3),
    "config2": lambda: S.config2(0),
    # open stroked polylines mixed with closed outlines, ragged canvases, some items off canvas
    "open": lambda: S.random_scene(6, [(71, 53), (40, 66)], [11, 8], kinds=("open", "poly", "open", "star"),
                                   radius=(3.0, 10.0), off_canvas=0.2),
    # every loss term including the uniform one; canvases ragged against the 32-pixel window tiles,
    # one smaller than a tile and empty (all windows empty), items partly off canvas
    "uniform": lambda: dataclasses.replace(
        S.random_scene(14, [(71, 53), (20, 9), (40, 97), (64, 64)], [9, 0, 7, 10], radius=(3.0, 8.0),
                       off_canvas=0.2), w_uniform=0.6),
    # the containment of eq. 5, the central and the object-space downward forces, normalized by area
    "forces": lambda: dataclasses.replace(
        S.random_scene(17, [(61, 47), (33, 70), (18, 18)], [8, 6, 0], radius=(3.0, 8.0), off_canvas=0.2),
        w_contain=0.0, w_fill=0.0, w_wmse=2.0, w_centre=3e-3, w_objdown=0.25, area_mean=True),
}


@pytest.fixture(scope="module")
def oracles():
    cache = {}

    def get(name, level=None):
        key = (name, level)
        if key not in cache:
            sc = SCENES[name]() if name in SCENES else None
            cache[key] = (sc, Oracle(sc, level=level))
        return cache[key]

    return get


@pytest.mark.parametrize("tile", [16, 8, 32, 64, 128])
@pytest.mark.parametrize("name", list(SCENES))
def test_forward_parity(name, tile, oracles):
    sc, o = oracles(name)
    _say("forward", name, "tile", tile)
    cs = CollageScene(sc, tile=tile)
    cov, cov_pad, loss = cs.forward(cs.params_tensor())
    S_, Sp, L = o.forward(sc.params)
    check_image(_np(cov), S_, "S")
    check_image(_np(cov_pad), Sp, "S_pad")
    check_loss(_np(loss), L)


@pytest.mark.parametrize("tile", [16, 8, 32, 64, 128])
@pytest.mark.parametrize("name", list(SCENES))
def test_backward_parity_autograd(name, tile, oracles):
    sc, o = oracles(name)
    _say("backward", name, "tile", tile)
    cs = CollageScene(sc, tile=tile)
    p = cs.params_tensor().requires_grad_(True)
    rng = np.random.default_rng(1)
    dl = rng.uniform(0.5, 2.0, (sc.num_layouts, _lib.LOSS_TERMS))
    loss = CollageLoss.apply(p, cs)
    (loss * torch.tensor(dl, dtype=torch.float32, device=loss.device)).sum().backward()
    g_ref = o.backward(sc.params, dloss=dl)
    check_grad(_np(p.grad), g_ref)


def test_tiles_listing_more_units_than_lds_holds():
    # 1600 small items on a 40 x 40 canvas: the middle 8 x 8 tiles list more than the 1024 units whose
    # chunks and costs the binning kernel keeps in LDS, so the rest are read back from global memory
    sc = S.random_scene(11, [(40, 40)], [1600], kinds=("poly", "star"), radius=(0.8, 2.5))
    _say("many units per tile", sc.num_shapes)
    cs = CollageScene(sc, tile=8)
    from oracle.oracle import Oracle as _O
    o = _O(sc)
    cov, cov_pad, loss, grad = cs.forward_backward(cs.params_tensor())
    S_, Sp, L = o.forward(sc.params)
    check_image(_np(cov), S_, "S")
    check_image(_np(cov_pad), Sp, "S_pad")
    check_loss(_np(loss), L)
    check_grad(_np(grad), o.backward(sc.params))


@pytest.mark.parametrize("code_capacity,bin_chunk", [(-1, 0), (0, 0), (2, 3)])
@pytest.mark.parametrize("tile", [16, 8, 32, 64, 128])
@pytest.mark.parametrize("name", list(SCENES))
def test_fused_parity(name, tile, code_capacity, bin_chunk, oracles):
    sc, o = oracles(name)
    _say("fused", name, "tile", tile, "cache", code_capacity, "chunk", bin_chunk)
    cs = CollageScene(sc, tile=tile, code_capacity=code_capacity, bin_chunk=bin_chunk)
    cov, cov_pad, loss, grad = cs.forward_backward(cs.params_tensor())
    S_, Sp, L = o.forward(sc.params)
    check_image(_np(cov), S_, "S")
    check_image(_np(cov_pad), Sp, "S_pad")
    check_loss(_np(loss), L)
    check_grad(_np(grad), o.backward(sc.params))


@pytest.mark.parametrize("level,tile,code_capacity", [(128, 16, -1), (256, 16, -1), (512, 16, -1), (512, 8, -1),
                                                      (512, 32, -1), (512, 8, 0), (1024, 16, -1), (512, 64, -1),
                                                      (512, 128, -1), (512, 128, 0), (1024, 128, -1)])
def test_metric_scene_levels(level, tile, code_capacity):
    """500 Bezier items, the coarse-to-fine levels of the metric scene; 512 is the benchmark launch, in
    every tile size the autotuner may pick."""
    sc = S.config3(0)
    _say("config3 level", level, "tile", tile, "cache", code_capacity)
    o = Oracle(sc, level=level)
    cs = CollageScene(sc, level=level, tile=tile, code_capacity=code_capacity)
    cov, cov_pad, loss, grad = cs.forward_backward(cs.params_tensor())
    S_, Sp, L = o.forward(sc.params)
    check_image(_np(cov), S_, "S")
    check_image(_np(cov_pad), Sp, "S_pad")
    check_loss(_np(loss), L)
    check_grad(_np(grad), o.backward(sc.params))


def test_render_parity(oracles):
    for name in ("config1", "ragged", "open"):
        sc, o = oracles(name)
        _say("render", name)
        cs = CollageScene(sc)
        A, Ap = cs.render(cs.params_tensor())
        Ar, Apr = o.render(sc.params)
        check_image(_np(A), Ar, "alpha")
        check_image(_np(Ap), Apr, "alpha_pad")


def test_adam_step_matches_torch():
    sc = S.config1(0)
    _say("adam")
    cs = CollageScene(sc)
    p = cs.params_tensor()
    _, _, _, g = cs.forward_backward(p)
    m, v, step = cs.new_state()
    p_lib = p.clone()
    cs.step(p_lib, g, m, v, step)
    cs.step(p_lib, g, m, v, step)
    # torch.optim.Adam with the same per-parameter learning rates (one group per item and component)
    k = 1.0
    lr = np.zeros((sc.num_shapes, 4))
    lr[:, :2] = sc.lr_px / k
    lr[:, 2:] = sc.lr_px / (k * sc.rho.astype(np.float64))[:, None]
    ts = [p[i, c].clone().requires_grad_(True) for i in range(sc.num_shapes) for c in range(4)]
    opt = torch.optim.Adam([{"params": [t], "lr": float(lr.reshape(-1)[j])} for j, t in enumerate(ts)],
                           betas=(0.9, 0.999), eps=1e-8)
    gf = g.reshape(-1)
    for _ in range(2):
        for j, t in enumerate(ts):
            t.grad = gf[j].clone()
        opt.step()
    pt = torch.stack([t.detach() for t in ts]).reshape(-1, 4)
    assert int(step.item()) == 2
    np.testing.assert_allclose(_np(p_lib), _np(pt), rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("level", [128, 1024])
def test_adam_step_at_coarse_and_fine_levels(level):
    """Eq. 4 as Adam at levels of scale k = 0.25 and 2 of the metric scene: two collage_step calls against
    torch.optim.Adam with the learning rates of the definition (lr_px / k for t, lr_px / (k rho_i) for theta
    and s: every item moves by lr_px level px) and against the oracle's update."""
    sc = S.config3(0)
    _say("adam level", level)
    k = level / sc.level_ref
    cs = CollageScene(sc, level=level)
    p = cs.params_tensor()
    _, _, _, g = cs.forward_backward(p, want_cov=False)
    m, v, step = cs.new_state()
    p_lib = p.clone()
    cs.step(p_lib, g, m, v, step)
    cs.step(p_lib, g, m, v, step)
    assert int(step.item()) == 2
    p0, g0 = _np(p).astype(np.float64), _np(g).astype(np.float64)
    lr = np.zeros((sc.num_shapes, 4))
    lr[:, :2] = sc.lr_px / k
    lr[:, 2:] = sc.lr_px / (k * sc.rho.astype(np.float64))[:, None]
    ts = [torch.tensor(p0[i, c], dtype=torch.float64, requires_grad=True) for i in range(sc.num_shapes) for c in range(4)]
    opt = torch.optim.Adam([{"params": [t], "lr": float(lr.reshape(-1)[j])} for j, t in enumerate(ts)],
                           betas=(0.9, 0.999), eps=1e-8)
    for _ in range(2):
        for j, t in enumerate(ts):
            t.grad = torch.tensor(g0.reshape(-1)[j], dtype=torch.float64)
        opt.step()
    pt = np.array([t.item() for t in ts]).reshape(-1, 4)
    o = Oracle(sc, level=level)
    lr_o = o.learning_rates()
    po, mo, vo = o.adam(p0, g0, np.zeros_like(p0), np.zeros_like(p0), 1, lr_o)
    po, mo, vo = o.adam(po, g0, mo, vo, 2, lr_o)
    np.testing.assert_allclose(lr_o, lr, rtol=1e-12)
    np.testing.assert_allclose(_np(p_lib), pt, rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(_np(p_lib), po, rtol=1e-6, atol=1e-6)
    # the step moved the items: by about 2 lr_px level px over two steps where the gradient is not small
    assert np.abs(k * (_np(p_lib)[:, :2] - p0[:, :2])).max() > 0.9 * sc.lr_px


def test_iterate_equals_fused_then_step():
    sc = S.random_scene(4, [(40, 33), (29, 45)], [5, 6])
    _say("iterate")
    cs = CollageScene(sc)
    p0 = cs.params_tensor()
    p1 = p0.clone()
    m1, v1, s1 = cs.new_state()
    m2, v2, s2 = cs.new_state()
    p2 = p0.clone()
    for _ in range(3):
        loss1, g1 = cs.iterate(p1, m1, v1, s1)
        _, _, loss2, g2 = cs.forward_backward(p2)
        cs.step(p2, g2, m2, v2, s2)
        assert torch.equal(loss1, loss2) and torch.equal(g1, g2)
    assert torch.equal(p1, p2) and torch.equal(m1, m2) and torch.equal(v1, v2)
    assert int(s1.item()) == 3 and int(s2.item()) == 3


@pytest.mark.parametrize("tile", [8, 32, 128])
def test_iterate_n_equals_repeated_iterate(tile):
    # inside collage_iterate_n the update kernel transforms the items for the next epoch; the result
    # must be bitwise that of separate epochs
    sc = S.random_scene(4, [(60, 44), (33, 47)], [12, 7], off_canvas=0.2)
    _say("iterate_n", tile)
    cs = CollageScene(sc, tile=tile)
    p1 = cs.params_tensor()
    m1, v1, s1 = cs.new_state()
    for _ in range(5):
        l1, g1 = cs.iterate(p1, m1, v1, s1)
    p2 = cs.params_tensor()
    m2, v2, s2 = cs.new_state()
    l2, g2 = cs.iterate_n(p2, m2, v2, s2, 5)
    torch.cuda.synchronize()
    assert torch.equal(p1, p2) and torch.equal(m1, m2) and torch.equal(v1, v2)
    assert torch.equal(l1, l2) and torch.equal(g1, g2)
    assert int(s1.item()) == int(s2.item()) == 5


@pytest.mark.parametrize("pairs,epochs,stamped", [(3, 7, 3), (10, 7, 7), (2, 7, 2), (1, 1, 1)])
def test_iterate_n_timer_sampling(pairs, epochs, stamped):
    # a timer of c pairs stamps the coverage launches of epochs 0, d, 2d, ... (d = ceil(epochs / c));
    # the timestamps change nothing in what the epochs compute
    sc = S.random_scene(4, [(60, 44), (33, 47)], [12, 7], off_canvas=0.2)
    _say("timer", pairs, epochs)
    cs = CollageScene(sc, tile=16)
    p1 = cs.params_tensor()
    m1, v1, s1 = cs.new_state()
    l1, g1 = cs.iterate_n(p1, m1, v1, s1, epochs)
    p2 = cs.params_tensor()
    m2, v2, s2 = cs.new_state()
    t = Timer(pairs)
    l2, g2 = cs.iterate_n(p2, m2, v2, s2, epochs, timer=t)
    torch.cuda.synchronize()
    assert torch.equal(p1, p2) and torch.equal(l1, l2) and torch.equal(g1, g2)
    ms = t.elapsed_ms()
    assert len(ms) == stamped and np.all(ms > 0) and np.all(ms < 1e3)


def test_graph_replay_matches_eager():
    sc = S.config1(0)
    _say("graph")
    cs = CollageScene(sc)
    p_g = cs.params_tensor()
    m_g, v_g, s_g = cs.new_state()
    loss_g = torch.empty(1, _lib.LOSS_TERMS, device="cuda")
    grad_g = torch.empty(sc.num_shapes, 4, device="cuda")
    g = cs.graph(p_g, m_g, v_g, s_g, loss_g, grad_g, replays_per_launch=2)
    p_e = cs.params_tensor()
    m_e, v_e, s_e = cs.new_state()
    for rep in range(4):
        g.launch(1)
        g.stream.synchronize()
        for _ in range(2):
            loss_e, grad_e = cs.iterate(p_e, m_e, v_e, s_e)
        torch.cuda.synchronize()
        assert torch.equal(p_g, p_e), rep
        assert torch.equal(loss_g, loss_e) and torch.equal(grad_g, grad_e), rep
        assert int(s_g.item()) == int(s_e.item()) == 2 * (rep + 1)


def test_bitwise_deterministic():
    sc = S.config2(0)
    _say("determinism")
    cs = CollageScene(sc)
    p = cs.params_tensor()
    a = cs.forward_backward(p)
    b = cs.forward_backward(p)
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_gradient_vs_central_differences_config2():
    sc = S.config2(0)
    _say("fd config2")
    cs = CollageScene(sc)
    p = cs.params_tensor().requires_grad_(True)
    CollageLoss.apply(p, cs).sum().backward()
    o = Oracle(sc)
    items = [0, 17, 42, 63, 99]
    fd = o.fd_gradient(sc.params, shapes=items)
    g = _np(p.grad)
    full = o.backward(sc.params)
    floor = 0.01 * np.abs(full).max(0)
    for c in range(4):
        err = np.abs(g[items, c] - fd[items, c]) / np.maximum(np.abs(fd[items, c]), floor[c])
        assert err.max() <= 1e-4, (c, err)


def test_open_items_vs_central_differences():
    sc = SCENES["open"]()
    _say("fd open")
    cs = CollageScene(sc)
    p = cs.params_tensor().requires_grad_(True)
    CollageLoss.apply(p, cs).sum().backward()
    o = Oracle(sc)
    items = [i for i in range(sc.num_shapes) if sc.stroke[i] > 0][:6]
    fd = o.fd_gradient(sc.params, shapes=items)
    g = _np(p.grad)
    floor = 0.01 * np.abs(o.backward(sc.params)).max(0)
    for c in range(4):
        err = np.abs(g[items, c] - fd[items, c]) / np.maximum(np.abs(fd[items, c]), floor[c])
        assert err.max() <= 1e-4, (c, err)


def test_uniform_term_vs_central_differences():
    """The uniform term alone (the other weights 0): GPU gradient against central differences."""
    sc = dataclasses.replace(SCENES["uniform"](), w_overlap=0.0, w_contain=0.0, w_fill=0.0, w_pad=0.0,
                             w_down=0.0, w_uniform=1.0)
    _say("fd uniform")
    cs = CollageScene(sc)
    p = cs.params_tensor().requires_grad_(True)
    CollageLoss.apply(p, cs).sum().backward()
    o = Oracle(sc)
    items = list(range(0, sc.num_shapes, 3))
    fd = o.fd_gradient(sc.params, shapes=items)
    g = _np(p.grad)
    floor = 0.01 * np.abs(o.backward(sc.params)).max(0)
    assert np.abs(fd[items]).max() > 0.0
    for c in range(4):
        err = np.abs(g[items, c] - fd[items, c]) / np.maximum(np.abs(fd[items, c]), floor[c])
        assert err.max() <= 1e-4, (c, err)


@pytest.mark.parametrize("level,tile", [(512, 32), (1024, 16)])
def test_uniform_term_metric_scene(level, tile):
    """500 Bezier items with every term including the uniform one."""
    sc = dataclasses.replace(S.config3(0), w_uniform=2e-3)
    _say("config3 uniform level", level, "tile", tile)
    o = Oracle(sc, level=level)
    cs = CollageScene(sc, level=level, tile=tile)
    cov, cov_pad, loss, grad = cs.forward_backward(cs.params_tensor())
    S_, Sp, L = o.forward(sc.params)
    assert L[0, 5] > 0.0
    check_image(_np(cov), S_, "S")
    check_loss(_np(loss), L)
    check_grad(_np(grad), o.backward(sc.params))


@pytest.mark.parametrize("level,tile", [(512, 32), (256, 16)])
def test_paper_loss_preset_metric_scene(level, tile):
    """The weights of eq. 8 (WMSE containment, overlap, uniform; 1 / (w h)) on the 500-item scene."""
    sc = S.paper_loss_preset(S.config3(0))
    _say("config3 paper preset level", level, "tile", tile)
    o = Oracle(sc, level=level)
    cs = CollageScene(sc, level=level, tile=tile)
    cov, cov_pad, loss, grad = cs.forward_backward(cs.params_tensor())
    S_, Sp, L = o.forward(sc.params)
    assert L[0, 6] > 0.0 and L[0, 5] > 0.0 and L[0, 0] > 0.0
    check_loss(_np(loss), L)
    check_grad(_np(grad), o.backward(sc.params))


def test_force_terms_vs_central_differences():
    sc = SCENES["forces"]()
    _say("fd forces")
    cs = CollageScene(sc)
    p = cs.params_tensor().requires_grad_(True)
    CollageLoss.apply(p, cs).sum().backward()
    o = Oracle(sc)
    items = list(range(0, sc.num_shapes, 2))
    fd = o.fd_gradient(sc.params, shapes=items)
    g = _np(p.grad)
    floor = 0.01 * np.abs(o.backward(sc.params)).max(0)
    for c in range(4):
        err = np.abs(g[items, c] - fd[items, c]) / np.maximum(np.abs(fd[items, c]), floor[c])
        assert err.max() <= 1e-4, (c, err)


@pytest.mark.parametrize("code_capacity", [-1, 0])
@pytest.mark.parametrize("tile", [16, 8, 32, 64, 128])
@pytest.mark.parametrize("name", list(SCENES))
def test_vertex_gradient_parity(name, tile, code_capacity, oracles):
    """dLoss/d(outline vertex) and the parameter gradient of the same call, with a random dloss."""
    sc, o = oracles(name)
    _say("vertex grad", name, "tile", tile, "cache", code_capacity)
    cs = CollageScene(sc, tile=tile, code_capacity=code_capacity)
    dl = np.random.default_rng(7).uniform(0.5, 2.0, (sc.num_layouts, _lib.LOSS_TERMS))
    g, gv = cs.backward_vertices(cs.params_tensor(), torch.tensor(dl, dtype=torch.float32, device="cuda"))
    g_ref, gv_ref = o.backward_vertices(sc.params, dloss=dl.astype(np.float32).astype(np.float64))
    check_grad(_np(g), g_ref)
    check_vgrad(_np(gv), gv_ref)
    _, gv2 = cs.backward_vertices(cs.params_tensor(), torch.tensor(dl, dtype=torch.float32, device="cuda"),
                                  want_grad=False)
    assert torch.equal(gv, gv2)


def test_vertex_gradient_metric_scene():
    sc = S.config3(0)
    _say("vertex grad config3 512")
    o = Oracle(sc, level=512)
    cs = CollageScene(sc, level=512, tile=32)
    g, gv = cs.backward_vertices(cs.params_tensor())
    g_ref, gv_ref = o.backward_vertices(sc.params)
    check_grad(_np(g), g_ref)
    check_vgrad(_np(gv), gv_ref)


def test_outline_fitting_to_a_silhouette():
    """Gradient descent (Adam) on the vertices of one circle outline towards a rectangular silhouette
    (the container mask as the target image): the mismatch falls by well over half."""
    sc = S.multi_shape_scene([S.regular_polygon(48, 9.0)], np.array([[32.0, 32.0, 0.0, 1.0]]), 64, 64, mask="none",
                             w_overlap=0.0, w_contain=1.0, w_fill=1.0)
    lay = dataclasses.replace(sc.layouts[0], rects=np.array([[32.0, 32.0, 16.0, 7.0, 0.3]]), full=False)
    sc = dataclasses.replace(sc, layouts=[lay])
    _say("outline fit")
    cs = CollageScene(sc)
    p = cs.params_tensor()
    verts = cs.verts
    opt = torch.optim.Adam([verts], lr=0.15)
    losses = []
    for _ in range(150):
        _, _, loss = cs.forward(p, want_cov=False)
        losses.append(float(loss.sum()))
        _, gv = cs.backward_vertices(p, want_grad=False)
        verts.grad = gv
        opt.step()
    assert np.all(np.isfinite(losses)) and losses[-1] < 0.4 * losses[0], (losses[0], losses[-1])


def test_uniform_term_fractional_mask():
    """Mask values strictly between 0 and 1 on the first layout (its tiles take the exact fixed-point
    tables of the gradient pass) and binary masks on the others (packed flag counts), in one launch."""
    sc = SCENES["uniform"]()
    w, h, _, _ = sc.layout_arrays(None)
    n0 = int(w[0]) * int(h[0])
    m = sc.packed_mask(None).astype(np.float32).copy()
    rng = np.random.default_rng(3)
    m[:n0] *= rng.uniform(0.05, 1.0, n0).astype(np.float32)
    assert np.any((m[:n0] > 0) & (m[:n0] < 1))
    _say("uniform fractional mask")
    o = Oracle(sc, mask=m.astype(np.float64))
    cs = CollageScene(sc, mask=m)
    dl = rng.uniform(0.5, 2.0, (sc.num_layouts, _lib.LOSS_TERMS))
    cov, cov_pad, loss, grad = cs.forward_backward(cs.params_tensor())
    S_, Sp, L = o.forward(sc.params)
    check_loss(_np(loss), L)
    check_grad(_np(grad), o.backward(sc.params))
    g = cs.backward(cs.params_tensor(), torch.tensor(dl, dtype=torch.float32, device="cuda"))
    check_grad(_np(g), o.backward(sc.params, dloss=dl.astype(np.float32).astype(np.float64)))


def test_uniform_term_is_deterministic_and_forward_matches_fused():
    sc = SCENES["uniform"]()
    _say("uniform determinism")
    cs = CollageScene(sc, tile=8)
    p = cs.params_tensor()
    runs = [cs.forward_backward(p) for _ in range(3)]
    for r in runs[1:]:
        for x, y in zip(r, runs[0]):
            assert torch.equal(x, y)
    _, _, loss_f = cs.forward(p)
    assert torch.equal(loss_f, runs[0][2])
    dl = torch.zeros(sc.num_layouts, _lib.LOSS_TERMS, device="cuda")
    dl[:, 5] = 1.0
    g_u = cs.backward(p, dl)
    o = Oracle(sc)
    check_grad(_np(g_u), o.backward(sc.params, dloss=_np(dl).astype(np.float64)))


@pytest.mark.parametrize("level,tile", [(256, 16), (2048, 32), (256, 64), (1024, 128)])
def test_open_scene_levels(level, tile):
    """2000 stroked polylines on the 2048 x 2048 scene at its coarsest and finest levels, and in the tiles
    the schedule's autotuner picks for its levels."""
    sc = S.config5(0)
    _say("config5 level", level, "tile", tile)
    o = Oracle(sc, level=level)
    cs = CollageScene(sc, level=level, tile=tile)
    cov, cov_pad, loss, grad = cs.forward_backward(cs.params_tensor())
    S_, Sp, L = o.forward(sc.params)
    check_image(_np(cov), S_, "S")
    check_image(_np(cov_pad), Sp, "S_pad")
    check_loss(_np(loss), L)
    check_grad(_np(grad), o.backward(sc.params))


def test_edge_cases():
    _say("edge cases")
    # items with 1 and 2 vertices, one huge item covering the canvas, one far off canvas
    outlines = [np.array([[0.0, 0.0]]), np.array([[-3.0, 0.0], [3.0, 0.5]]), S.regular_polygon(12, 4.0),
                S.star_polygon(5, 6.0, 0.5)]
    params = np.array([[10.3, 11.7, 0.2, 1.0], [20.1, 9.3, 0.4, 1.0], [15.2, 14.9, 0.3, 9.0],
                       [-80.0, 10.0, 0.0, 1.0]])
    sc = S.multi_shape_scene(outlines, params, 33, 27, mask="disk", w_overlap=1, w_contain=1, w_fill=1,
                             w_pad=1, r_pad=2.0, w_down=1e-3)
    sc.rho[:2] = 1.0
    o = Oracle(sc)
    for tile in (8, 16, 64, 128):
        cs = CollageScene(sc, tile=tile)
        cov, cov_pad, loss, grad = cs.forward_backward(cs.params_tensor())
        S_, Sp, L = o.forward(sc.params)
        check_image(_np(cov), S_, "S")
        check_loss(_np(loss), L)
        check_grad(_np(grad), o.backward(sc.params))
    # an empty scene: only the fill term of the container remains
    empty = S.random_scene(1, [(19, 23)], [0])
    cs = CollageScene(empty)
    cov, cov_pad, loss, grad = cs.forward_backward(cs.params_tensor())
    assert float(cov.abs().max()) == 0.0
    check_loss(_np(loss), Oracle(empty).forward(empty.params)[2])
    # non-finite parameters: the item is skipped and its gradient is NaN
    sc2 = S.config1(0)
    p = sc2.params.copy()
    p[3, 0] = np.nan
    cs = CollageScene(sc2)
    _, _, loss, grad = cs.forward_backward(cs.params_tensor(p))
    g = _np(grad)
    assert np.all(np.isnan(g[3])) and np.all(np.isfinite(np.delete(g, 3, 0)))
    assert np.all(np.isfinite(_np(loss)))
    # the status word counts the item once per epoch of the call, and is cleared by the next call
    assert cs.status()[_lib.STATUS_NONFINITE] == 1
    m, v, st = cs.new_state()
    pn = cs.params_tensor(p)
    cs.iterate_n(pn, m, v, st, 3)
    assert cs.status()[_lib.STATUS_NONFINITE] == 3
    cs.forward_backward(cs.params_tensor())
    st_ = cs.status()
    assert st_[_lib.STATUS_NONFINITE] == 0 and st_[_lib.STATUS_CHUNKS] > 0 and st_[_lib.STATUS_RESCANNED] == 0
    assert list(st_[3:]) == [0] * (_lib.STATUS_WORDS - 3)  # no unit overflow, no gradient beyond range
    # with no kept codes, the adjoint rescans every chunk of the pass
    cs0 = CollageScene(sc2, code_capacity=0)
    cs0.forward_backward(cs0.params_tensor())
    st0 = cs0.status()
    assert st0[_lib.STATUS_RESCANNED] == st0[_lib.STATUS_CHUNKS] == st_[_lib.STATUS_CHUNKS]
    # gradient pieces beyond the fixed-point range (2^23) are reported: a fill weight of 1e9 makes every
    # piece of an item that covers container pixels far larger; with the default weight none is
    big = dataclasses.replace(sc2, w_fill=1e9)
    csb = CollageScene(big)
    csb.forward_backward(csb.params_tensor())
    assert csb.status()[_lib.STATUS_GRAD_RANGE] > 0
    assert st_[_lib.STATUS_GRAD_RANGE] == 0


@pytest.mark.parametrize("name,level", [("config3", 512), ("config5", 1024), ("config4", None)])
def test_tile_sizes_give_the_same_bits(name, level):
    # S and S_pad are exact fixed-point sums of per-(pixel, item) values that do not depend on the tiling,
    # the loss sums run over 32 x 32 pixel tiles, and the gradient sums are exact integer sums of
    # per-(pixel, item) terms: every output is bitwise the same at every screen-tile size
    sc = getattr(S, name)(0)
    _say("tile sizes", name, level)
    ref = None
    for tile in (32, 8, 16, 64, 128):
        cs = CollageScene(sc, level=level, tile=tile)
        out = [x.clone() for x in cs.forward_backward(cs.params_tensor())]
        assert cs.status()[_lib.STATUS_GRAD_RANGE] == 0
        if ref is None:
            ref = out
            continue
        for x, y, what in zip(out, ref, ("S", "S_pad", "loss", "grad")):
            assert torch.equal(x, y), (tile, what)


def test_degenerate_scales():
    # s = 0 collapses an item to its centre (sd = minus the distance to that point); s < 0 is a point
    # reflection of the outline; both are valid inputs of eq. 2
    sc = S.config1(0)
    p = sc.params.copy()
    p[1, 3] = 0.0
    p[4, 3] = -0.8
    _say("degenerate scales")
    o = Oracle(sc)
    S_, Sp, L = o.forward(p)
    g_ref = o.backward(p)
    for tile in (8, 16, 64, 128):
        cs = CollageScene(sc, tile=tile)
        cov, cov_pad, loss, grad = cs.forward_backward(cs.params_tensor(p))
        check_image(_np(cov), S_, "S")
        check_loss(_np(loss), L)
        check_grad(_np(grad), g_ref)


@pytest.mark.parametrize("code_capacity", [-1, 0])
def test_items_with_more_edges_than_one_lds_stage(code_capacity):
    # outlines of 300 and 700 edges are staged in LDS in segments of 256 edges (coverage, and the
    # adjoint's rescan when codes are not kept)
    rng = np.random.default_rng(8)
    outlines = [S.regular_polygon(700, 14.0, 0.1), S.star_polygon(150, 12.0, 0.8),
                S.jittered_bezier(rng, 12, 9.0), S.regular_polygon(7, 5.0)]
    params = np.array([[30.3, 29.1, 0.2, 1.0], [44.7, 40.2, 0.4, 1.0], [20.2, 45.9, 0.1, 1.1],
                       [52.6, 18.4, 1.3, 0.9]])
    sc = S.multi_shape_scene(outlines, params, 70, 64, mask="disk", w_overlap=1, w_contain=1, w_fill=1,
                             w_pad=1, r_pad=2.0, w_down=1e-3)
    assert max(np.diff(sc.vert_off)) == 700
    o = Oracle(sc)
    S_, Sp, L = o.forward(sc.params)
    g_ref = o.backward(sc.params)
    for tile in (8, 16, 64, 128):
        _say("long outlines", tile, code_capacity)
        cs = CollageScene(sc, tile=tile, code_capacity=code_capacity)
        cov, cov_pad, loss, grad = cs.forward_backward(cs.params_tensor())
        check_image(_np(cov), S_, "S")
        check_image(_np(cov_pad), Sp, "S_pad")
        check_loss(_np(loss), L)
        check_grad(_np(grad), g_ref)


def test_more_items_than_one_bin_chunk():
    # 1100 items in one layout: the binning kernel takes the layout in two LDS chunks (1024 + 76)
    sc = S.random_scene(21, [(96, 80)], [1100], radius=(1.5, 4.0), off_canvas=0.1)
    _say("1100 items", sc.num_shapes)
    o = Oracle(sc)
    S_, Sp, L = o.forward(sc.params)
    g_ref = o.backward(sc.params)
    for tile in (8, 16):
        cs = CollageScene(sc, tile=tile)
        cov, cov_pad, loss, grad = cs.forward_backward(cs.params_tensor())
        check_image(_np(cov), S_, "S")
        check_image(_np(cov_pad), Sp, "S_pad")
        check_loss(_np(loss), L)
        check_grad(_np(grad), g_ref)


def test_batched_layouts_match_separate_scenes():
    sc = S.config4(0, num_layouts=12)
    _say("batched vs separate", sc.num_shapes)
    cs = CollageScene(sc)
    cov, cov_pad, loss, grad = cs.forward_backward(cs.params_tensor())
    o = Oracle(sc)
    S_, Sp, L = o.forward(sc.params)
    check_image(_np(cov), S_, "S")
    check_loss(_np(loss), L)
    check_grad(_np(grad), o.backward(sc.params))
    # each layout on its own gives bitwise the same per-layout results
    imgs = cs.layout_images(cov)
    for b in (0, 5, 11):
        lay = sc.layouts[b]
        sub = sc.layout_subset(b)
        cs1 = CollageScene(sub)
        c1, _, l1, g1 = cs1.forward_backward(cs1.params_tensor())
        assert torch.equal(c1, imgs[b].reshape(-1))
        assert torch.equal(l1[0], loss[b])
        assert torch.equal(g1, grad[lay.shape_begin:lay.shape_end])


@pytest.mark.parametrize("tile", [32, 16, 128])
def test_full_batch_sampled_layouts(tile):
    # the 64-layout batch at full resolution, in the benchmark's launch; the oracle evaluates a
    # sample of its layouts on their own (layouts are independent)
    sc = S.config4(0)
    _say("full batch", sc.num_layouts, sc.num_shapes, "tile", tile)
    cs = CollageScene(sc, tile=tile)
    cov, cov_pad, loss, grad = cs.forward_backward(cs.params_tensor())
    imgs, imgs_pad = cs.layout_images(cov), cs.layout_images(cov_pad)
    for b in (0, 17, 42, 63):
        sub = sc.layout_subset(b)
        o = Oracle(sub)
        S_, Sp, L = o.forward(sub.params)
        lay = sc.layouts[b]
        check_image(_np(imgs[b]).reshape(-1), S_, f"S[{b}]")
        check_image(_np(imgs_pad[b]).reshape(-1), Sp, f"S_pad[{b}]")
        check_loss(_np(loss[b:b + 1]), L)
        check_grad(_np(grad[lay.shape_begin:lay.shape_end]), o.backward(sub.params))
