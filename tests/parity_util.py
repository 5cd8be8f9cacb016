"""Comparison helpers for GPU-vs-oracle parity (the tolerances of the hot path).

  images  (S, S_pad, per-item alpha): |gpu - ref| <= 1e-5 absolute
  loss    each term: |gpu - ref| <= 1e-5 |ref| (+1e-9 for exact zeros)
  grads   |g - g_ref| <= 1e-4 max(|g_ref|, 0.01 max_items |g_ref| of that component)
  vertex grads  the same, over vertices and the two components
"""
import numpy as np

IMG_ATOL = 1e-5
LOSS_RTOL = 1e-5
GRAD_RTOL = 1e-4


def check_image(gpu, ref, what="image", atol=IMG_ATOL):
    gpu = np.asarray(gpu, np.float64).reshape(-1)
    ref = np.asarray(ref, np.float64).reshape(-1)
    assert gpu.shape == ref.shape, (what, gpu.shape, ref.shape)
    err = np.abs(gpu - ref)
    i = int(np.argmax(err)) if err.size else 0
    assert err.size == 0 or err[i] <= atol, f"{what}: max |err| {err[i]:.3e} at {i} (gpu {gpu[i]}, ref {ref[i]})"
    return float(err.max()) if err.size else 0.0


def check_loss(gpu, ref, what="loss", rtol=LOSS_RTOL):
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    err = np.abs(gpu - ref)
    bound = rtol * np.abs(ref) + 1e-9
    assert np.all(err <= bound), f"{what}: gpu {gpu} ref {ref} rel {err / np.maximum(np.abs(ref), 1e-30)}"
    return float((err / np.maximum(np.abs(ref), 1e-30)).max()) if err.size else 0.0


def grad_error(gpu, ref, slack=None):
    """Largest |g - g_ref| / max(|g_ref|, floor) over items and components; with slack ([N,4], >= 0), the
    part of each difference beyond the slack (a difference within its slack counts as 0)."""
    gpu = np.asarray(gpu, np.float64).reshape(-1, 4)
    ref = np.asarray(ref, np.float64).reshape(-1, 4)
    if ref.size == 0:
        return 0.0
    floor = 0.01 * np.abs(ref).max(0)
    denom = np.maximum(np.abs(ref), floor[None, :])
    denom = np.where(denom > 0, denom, 1.0)
    diff = np.abs(gpu - ref)
    if slack is not None:
        diff = np.maximum(diff - np.asarray(slack, np.float64).reshape(-1, 4), 0.0)
    return float((diff / denom).max())


def check_grad(gpu, ref, what="grad", rtol=GRAD_RTOL, slack=None):
    """The gradient bar; slack ([N,4]) widens it per item and component by an amount the oracle derived
    (the nearest-edge ambiguity bound: pixels whose nearest edge float32 cannot resolve)."""
    e = grad_error(gpu, ref, slack)
    if e > rtol:
        g = np.asarray(gpu, np.float64).reshape(-1, 4)
        r = np.asarray(ref, np.float64).reshape(-1, 4)
        floor = 0.01 * np.abs(r).max(0)
        diff = np.abs(g - r)
        if slack is not None:
            diff = np.maximum(diff - np.asarray(slack, np.float64).reshape(-1, 4), 0.0)
        rel = diff / np.maximum(np.maximum(np.abs(r), floor[None, :]), 1e-30)
        i, c = np.unravel_index(int(np.argmax(rel)), rel.shape)
        raise AssertionError(f"{what}: relative error {e:.3e} > {rtol} at item {i} component {c}: "
                             f"gpu {g[i, c]!r} ref {r[i, c]!r} floor {floor[c]!r}")
    return e


def check_vgrad(gpu, ref, what="vertex grad", rtol=GRAD_RTOL):
    g = np.asarray(gpu, np.float64).reshape(-1, 2)
    r = np.asarray(ref, np.float64).reshape(-1, 2)
    if r.size == 0:
        return 0.0
    floor = 0.01 * np.abs(r).max(0)
    denom = np.maximum(np.abs(r), floor[None, :])
    denom = np.where(denom > 0, denom, 1.0)
    rel = np.abs(g - r) / denom
    i, c = np.unravel_index(int(np.argmax(rel)), rel.shape)
    assert rel[i, c] <= rtol, f"{what}: relative error {rel[i, c]:.3e} at vertex {i} component {c}: gpu {g[i, c]!r} ref {r[i, c]!r}"
    return float(rel.max())
