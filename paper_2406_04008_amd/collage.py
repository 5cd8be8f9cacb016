"""PyTorch-facing binding of the HIP collage library.

PyTorch supplies device memory and streams only; every step of the hot path runs in the HIP kernels
behind the C ABI (include/collage.h).  There is no CPU fallback: constructing a ``CollageScene``
without a GPU or without the built library raises.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Tuple

import numpy as np
import torch

from . import _lib
from .scenes import Scene


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _need(t: torch.Tensor, shape, name, dtype=torch.float32):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


class CollageScene:
    """One level of a batch of layouts, resident on one GPU.

    tile: screen tile edge (8, 16, 32, 64 or 128 px; 0 = 16); code_capacity: 64-pixel chunks whose
    nearest-edge codes the coverage pass keeps for the adjoint (-1 = default, 0 = none: the adjoint scans
    again); unit_capacity: (tile, item) work units each layout's pool holds (0 = default bound, -1 = every
    item in every tile); an epoch that overflows a pool is counted in status()[STATUS_UNIT_OVERFLOW]."""

    def __init__(self, scene: Scene, level: Optional[int] = None, device="cuda", tile: int = 0,
                 code_capacity: int = -1, bin_chunk: int = 0, flags: int = 0, mask: Optional[np.ndarray] = None,
                 allocate_workspace: bool = True, unit_capacity: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("CollageScene needs a GPU (the HIP library has no CPU path)")
        self.lib = _lib.load()
        self.scene = scene
        self.level = level
        self.device = torch.device(device)
        self.N = scene.num_shapes
        self.B = scene.num_layouts
        w, h, k, off = scene.layout_arrays(level)
        self.widths, self.heights, self.scales = w, h, k
        self._w = np.ascontiguousarray(w, np.int32)
        self._h = np.ascontiguousarray(h, np.int32)
        self._k = np.ascontiguousarray(k, np.float32)
        self._off = np.ascontiguousarray(off, np.int32)
        self._voff = np.ascontiguousarray(scene.vert_off, np.int32)
        dev = self.device
        self.verts = torch.from_numpy(np.ascontiguousarray(scene.verts, np.float32).reshape(-1, 2)).to(dev)
        self.rho = torch.from_numpy(np.ascontiguousarray(scene.rho, np.float32)).to(dev)
        m = scene.packed_mask(level) if mask is None else np.ascontiguousarray(mask, np.float32).reshape(-1)
        self.mask = torch.from_numpy(m).to(dev)
        self.stroke = None
        if getattr(scene, "stroke", None) is not None and scene.num_shapes > 0:
            self.stroke = torch.from_numpy(np.ascontiguousarray(scene.stroke, np.float32)).to(dev)
        d = _lib.SceneDesc()
        d.num_layouts, d.num_shapes, d.num_verts = self.B, self.N, scene.num_verts
        d.layout_width = self._w.ctypes.data_as(_lib._i32p)
        d.layout_height = self._h.ctypes.data_as(_lib._i32p)
        d.layout_scale = self._k.ctypes.data_as(_lib._f32p)
        d.layout_shapes = self._off.ctypes.data_as(_lib._i32p)
        d.vert_offset = self._voff.ctypes.data_as(_lib._i32p)
        d.verts = self.verts.data_ptr() if self.verts.numel() else None
        d.rho = self.rho.data_ptr() if self.rho.numel() else None
        d.mask = self.mask.data_ptr()
        d.stroke = self.stroke.data_ptr() if self.stroke is not None else None
        d.tau, d.r_cut, d.r_pad = scene.tau, scene.r_cut, scene.r_pad
        w = scene.weights()
        (d.w_overlap, d.w_contain, d.w_fill, d.w_pad, d.w_down, d.w_uniform, d.w_wmse, d.w_centre,
         d.w_objdown) = w
        if getattr(scene, "area_mean", False):
            flags |= _lib.FLAG_AREA_MEAN
        d.tile, d.code_capacity, d.bin_chunk, d.flags = tile, code_capacity, bin_chunk, flags
        d.unit_capacity = unit_capacity
        self._desc = d
        h_ = ctypes.c_void_p()
        with torch.cuda.device(dev):
            _lib.check(self.lib.collage_scene_create(ctypes.byref(d), ctypes.byref(h_)), "collage_scene_create")
        self.handle = h_
        nb = ctypes.c_size_t()
        _lib.check(self.lib.collage_workspace_size(self.handle, ctypes.byref(nb)), "collage_workspace_size")
        self.workspace_bytes = int(nb.value)
        npx, nt = ctypes.c_int64(), ctypes.c_int64()
        _lib.check(self.lib.collage_scene_info(self.handle, ctypes.byref(npx), ctypes.byref(nt)), "collage_scene_info")
        self.num_pixels, self.num_tiles = int(npx.value), int(nt.value)
        # allocate_workspace=False: only the size (for callers that decide on it), no compute calls
        self.workspace = (torch.empty(max(self.workspace_bytes, 256), dtype=torch.uint8, device=dev)
                          if allocate_workspace else None)
        self.tile = tile if tile else 16

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.lib.collage_scene_destroy(h)
            self.handle = None

    # ------------------------------------------------------------------------------------------
    def _ws(self):
        if self.workspace is None:
            raise RuntimeError("this CollageScene was created without a workspace")
        return _ptr(self.workspace), self.workspace.numel()

    def status(self, stream=None) -> np.ndarray:
        """The device status words of the workspace after the work queued on `stream` (the current stream
        by default): [STATUS_NONFINITE] counts the (epoch, item) pairs of the last call with non-finite
        parameters.  Waits for the stream."""
        out = np.zeros(_lib.STATUS_WORDS, np.int32)
        ws, nb = self._ws()
        st = ctypes.c_void_p(stream.cuda_stream) if stream is not None else _stream(self.device)
        _lib.check(self.lib.collage_read_status(self.handle, ws, nb, out.ctypes.data_as(_lib._i32p), st),
                   "collage_read_status")
        return out

    def params_tensor(self, params=None) -> torch.Tensor:
        p = self.scene.params if params is None else params
        if isinstance(p, torch.Tensor):
            return p.to(self.device, torch.float32).contiguous()
        return torch.from_numpy(np.ascontiguousarray(p, np.float32).reshape(-1, 4)).to(self.device)

    def forward(self, params: torch.Tensor, want_cov: bool = True):
        _need(params, (self.N, 4), "params")
        cov = torch.empty(self.num_pixels, device=self.device) if want_cov else None
        cov_pad = torch.empty(self.num_pixels, device=self.device) if want_cov else None
        loss = torch.empty(self.B, _lib.LOSS_TERMS, device=self.device)
        ws, nb = self._ws()
        rc = self.lib.collage_forward(self.handle, _ptr(params), _ptr(cov), _ptr(cov_pad), _ptr(loss), ws, nb,
                                      _stream(self.device))
        _lib.check(rc, "collage_forward")
        return cov, cov_pad, loss

    def backward(self, params: torch.Tensor, dloss: torch.Tensor):
        _need(params, (self.N, 4), "params")
        _need(dloss, (self.B, _lib.LOSS_TERMS), "dloss")
        grad = torch.empty(self.N, 4, device=self.device)
        ws, nb = self._ws()
        rc = self.lib.collage_backward(self.handle, _ptr(params), _ptr(dloss), _ptr(grad), ws, nb,
                                       _stream(self.device))
        _lib.check(rc, "collage_backward")
        return grad

    def backward_vertices(self, params: torch.Tensor, dloss: Optional[torch.Tensor] = None, want_grad: bool = True):
        """(grad [N,4] or None, grad_verts [V,2]): the gradient of sum(dloss * loss) (dloss = 1 when None)
        with respect to the parameters and to the outline vertices in their item frames.  The vertices
        are read from `self.verts` on every call, so they can be optimized in place."""
        _need(params, (self.N, 4), "params")
        if dloss is None:
            dloss = torch.ones(self.B, _lib.LOSS_TERMS, device=self.device)
        _need(dloss, (self.B, _lib.LOSS_TERMS), "dloss")
        grad = torch.empty(self.N, 4, device=self.device) if want_grad else None
        grad_verts = torch.empty(self.scene.num_verts, 2, device=self.device)
        ws, nb = self._ws()
        rc = self.lib.collage_backward_vertices(self.handle, _ptr(params), _ptr(dloss), _ptr(grad), _ptr(grad_verts),
                                                ws, nb, _stream(self.device))
        _lib.check(rc, "collage_backward_vertices")
        return grad, grad_verts

    def forward_backward(self, params: torch.Tensor, want_cov: bool = True, loss: Optional[torch.Tensor] = None,
                         grad: Optional[torch.Tensor] = None):
        _need(params, (self.N, 4), "params")
        cov = torch.empty(self.num_pixels, device=self.device) if want_cov else None
        cov_pad = torch.empty(self.num_pixels, device=self.device) if want_cov else None
        loss = torch.empty(self.B, _lib.LOSS_TERMS, device=self.device) if loss is None else loss
        grad = torch.empty(self.N, 4, device=self.device) if grad is None else grad
        _need(loss, (self.B, _lib.LOSS_TERMS), "loss")
        _need(grad, (self.N, 4), "grad")
        ws, nb = self._ws()
        rc = self.lib.collage_forward_backward(self.handle, _ptr(params), _ptr(cov), _ptr(cov_pad), _ptr(loss),
                                               _ptr(grad), ws, nb, _stream(self.device))
        _lib.check(rc, "collage_forward_backward")
        return cov, cov_pad, loss, grad

    def forward_backward_static(self, params: torch.Tensor, want_cov: bool = True,
                                loss: Optional[torch.Tensor] = None, grad: Optional[torch.Tensor] = None):
        """forward_backward on the library's static scratch instead of this scene's workspace
        (collage_forward_backward_static: no device allocation inside the call)."""
        _need(params, (self.N, 4), "params")
        cov = torch.empty(self.num_pixels, device=self.device) if want_cov else None
        cov_pad = torch.empty(self.num_pixels, device=self.device) if want_cov else None
        loss = torch.empty(self.B, _lib.LOSS_TERMS, device=self.device) if loss is None else loss
        grad = torch.empty(self.N, 4, device=self.device) if grad is None else grad
        _need(loss, (self.B, _lib.LOSS_TERMS), "loss")
        _need(grad, (self.N, 4), "grad")
        rc = self.lib.collage_forward_backward_static(self.handle, _ptr(params), _ptr(cov), _ptr(cov_pad), _ptr(loss),
                                                      _ptr(grad), _stream(self.device))
        _lib.check(rc, "collage_forward_backward_static")
        return cov, cov_pad, loss, grad

    def new_state(self):
        """Zeroed Adam state (m, v, step) for this scene's parameters."""
        m = torch.zeros(self.N, 4, device=self.device)
        v = torch.zeros(self.N, 4, device=self.device)
        step = torch.zeros(1, dtype=torch.int32, device=self.device)
        return m, v, step

    def reset_state(self, m, v, step):
        """Zeroes the Adam state in a kernel on the current stream (collage_adam_reset)."""
        _need(m, (self.N, 4), "m")
        _need(v, (self.N, 4), "v")
        _need(step, (1,), "step", torch.int32)
        _lib.check(self.lib.collage_adam_reset(self.handle, _ptr(m), _ptr(v), _ptr(step), _stream(self.device)),
                   "collage_adam_reset")

    def step(self, params, grad, m, v, step, lr_px=None, betas=(0.9, 0.999), eps=1e-8):
        lr_px = self.scene.lr_px if lr_px is None else lr_px
        for t, n in ((params, "params"), (grad, "grad"), (m, "m"), (v, "v")):
            _need(t, (self.N, 4), n)
        _need(step, (1,), "step", torch.int32)
        rc = self.lib.collage_step(self.handle, _ptr(params), _ptr(grad), _ptr(m), _ptr(v), _ptr(step), lr_px,
                                   betas[0], betas[1], eps, _stream(self.device))
        _lib.check(rc, "collage_step")

    def iterate(self, params, m, v, step, loss=None, grad=None, cov=None, cov_pad=None, lr_px=None,
                betas=(0.9, 0.999), eps=1e-8):
        """One epoch: forward, loss, backward, Adam.  Returns (loss, grad) of this epoch."""
        lr_px = self.scene.lr_px if lr_px is None else lr_px
        loss = torch.empty(self.B, _lib.LOSS_TERMS, device=self.device) if loss is None else loss
        grad = torch.empty(self.N, 4, device=self.device) if grad is None else grad
        ws, nb = self._ws()
        rc = self.lib.collage_iterate(self.handle, _ptr(params), _ptr(cov), _ptr(cov_pad), _ptr(loss), _ptr(grad),
                                      _ptr(m), _ptr(v), _ptr(step), lr_px, betas[0], betas[1], eps, ws, nb,
                                      _stream(self.device))
        _lib.check(rc, "collage_iterate")
        return loss, grad

    def iterate_n(self, params, m, v, step, epochs: int, loss=None, grad=None, timer: Optional["Timer"] = None,
                  stream=None, lr_px=None, betas=(0.9, 0.999), eps=1e-8):
        """`epochs` epochs in one call (collage_iterate_n); with a timer of c pairs, the coverage kernels of
        epochs 0, d, 2d, ... (d = ceil(epochs / c)) are timestamped.  Returns (loss, grad) of the last epoch."""
        lr_px = self.scene.lr_px if lr_px is None else lr_px
        loss = torch.empty(self.B, _lib.LOSS_TERMS, device=self.device) if loss is None else loss
        grad = torch.empty(self.N, 4, device=self.device) if grad is None else grad
        ws, nb = self._ws()
        st = ctypes.c_void_p(stream.cuda_stream) if stream is not None else _stream(self.device)
        rc = self.lib.collage_iterate_n(self.handle, _ptr(params), None, None, _ptr(loss), _ptr(grad), _ptr(m),
                                        _ptr(v), _ptr(step), lr_px, betas[0], betas[1], eps, ws, nb, epochs,
                                        timer.handle if timer is not None else None, st)
        _lib.check(rc, "collage_iterate_n")
        return loss, grad

    def render(self, params: torch.Tensor, first: int = 0, count: Optional[int] = None) -> Tuple[torch.Tensor, torch.Tensor]:
        _need(params, (self.N, 4), "params")
        count = self.N - first if count is None else count
        off = self._off
        total = 0
        for q in range(first, first + count):
            b = int(np.searchsorted(off, q, side="right") - 1)
            total += int(self._w[b]) * int(self._h[b])
        alpha = torch.empty(max(total, 1), device=self.device)
        alpha_pad = torch.empty(max(total, 1), device=self.device)
        ws, nb = self._ws()
        rc = self.lib.collage_render_shapes(self.handle, _ptr(params), first, count, _ptr(alpha), _ptr(alpha_pad), ws,
                                            nb, _stream(self.device))
        _lib.check(rc, "collage_render_shapes")
        return alpha[:total], alpha_pad[:total]

    def graph(self, params, m, v, step, loss, grad, cov=None, cov_pad=None, lr_px=None, betas=(0.9, 0.999),
              eps=1e-8, replays_per_launch: int = 1, stream: Optional[torch.cuda.Stream] = None,
              reset_adam: bool = False) -> "CollageGraph":
        """A captured hipGraph of `replays_per_launch` epochs (optionally preceded by the Adam reset)."""
        lr_px = self.scene.lr_px if lr_px is None else lr_px
        return CollageGraph(self, params, m, v, step, loss, grad, cov, cov_pad, lr_px, betas, eps,
                            replays_per_launch, stream, reset_adam)

    def layout_images(self, flat: torch.Tensor):
        out, o = [], 0
        for w, h in zip(self._w, self._h):
            out.append(flat[o:o + int(w) * int(h)].view(int(h), int(w)))
            o += int(w) * int(h)
        return out


class CollageGraph:
    """A hipGraph of `replays_per_launch` epochs of collage_iterate, captured by the library."""

    def __init__(self, cs: CollageScene, params, m, v, step, loss, grad, cov, cov_pad, lr_px, betas, eps,
                 replays_per_launch, stream, reset_adam=False):
        self.cs = cs
        self.stream = stream if stream is not None else torch.cuda.Stream(cs.device)
        self._keep = (params, m, v, step, loss, grad, cov, cov_pad)
        ws, nb = cs._ws()
        h = ctypes.c_void_p()
        torch.cuda.current_stream(cs.device).synchronize()
        rc = cs.lib.collage_graph_create(cs.handle, _ptr(params), _ptr(cov), _ptr(cov_pad), _ptr(loss), _ptr(grad),
                                         _ptr(m), _ptr(v), _ptr(step), lr_px, betas[0], betas[1], eps, ws, nb,
                                         replays_per_launch, _lib.GRAPH_RESET_ADAM if reset_adam else 0,
                                         ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        _lib.check(rc, "collage_graph_create")
        self.handle = h
        self.replays_per_launch = replays_per_launch

    def launch(self, count: int = 1):
        rc = self.cs.lib.collage_graph_launch(self.handle, count, ctypes.c_void_p(self.stream.cuda_stream))
        _lib.check(rc, "collage_graph_launch")

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.cs.lib.collage_graph_destroy(h)
            self.handle = None


class Timer:
    """HIP event pairs owned by the library (see collage_timer_create)."""

    def __init__(self, count: int):
        self.lib = _lib.load()
        self.count = count
        h = ctypes.c_void_p()
        _lib.check(self.lib.collage_timer_create(count, ctypes.byref(h)), "collage_timer_create")
        self.handle = h

    def elapsed_ms(self) -> np.ndarray:
        """Durations of the pairs the last iterate_n call recorded (the unrecorded tail is dropped)."""
        out = np.zeros(self.count, np.float32)
        _lib.check(self.lib.collage_timer_elapsed(self.handle, out.ctypes.data_as(_lib._f32p)), "collage_timer_elapsed")
        return out[~np.isnan(out)]

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.lib.collage_timer_destroy(h)
            self.handle = None


class CollageLoss(torch.autograd.Function):
    """loss[B,9] = CollageLoss.apply(params[N,4], scene): the weighted loss terms of every layout.

    The backward recomputes the coverage and each pixel's nearest edge in the HIP adjoint kernel;
    only the parameters are saved between the passes."""

    @staticmethod
    def forward(ctx, params: torch.Tensor, cs: CollageScene):
        p = params.detach().contiguous()
        _, _, loss = cs.forward(p, want_cov=False)
        ctx.save_for_backward(p)
        ctx.cs = cs
        return loss

    @staticmethod
    def backward(ctx, dloss: torch.Tensor):
        (p,) = ctx.saved_tensors
        grad = ctx.cs.backward(p, dloss.to(torch.float32).contiguous())
        return grad, None
