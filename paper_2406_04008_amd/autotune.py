"""Launch-configuration autotuner for one scene level.

The knobs of the scene (tile edge T in {8, 16, 32}, and the code capacity that decides whether the
adjoint reads the coverage pass's nearest-edge codes or rescans) change only the speed: every
configuration computes the same quantities to the same tolerance against the oracle.  The tuner times whole epochs
(collage_iterate_n) of every candidate from the same parameters on the GPU it will run on, and keeps
the fastest.  Results are cached per (scene signature, level, device name) in memory and, if a path
is given, in a JSON file.
"""
from __future__ import annotations

import itertools
import json
import os
from dataclasses import asdict, dataclass
from typing import Dict, Iterable, List, Optional, Tuple

import torch

from . import _lib
from .collage import CollageScene
from .scenes import Scene


@dataclass(frozen=True)
class LaunchConfig:
    tile: int = 16
    code_capacity: int = -1
    bin_chunk: int = 0

    def scene_kwargs(self) -> dict:
        return {"tile": self.tile, "code_capacity": self.code_capacity, "bin_chunk": self.bin_chunk}


DEFAULT_SPACE = [LaunchConfig(t, c, 0) for t, c in itertools.product((8, 16, 32, 64, 128), (-1, 0))]
# candidates whose workspace exceeds this are not tried (with the default unit pools no standard workload
# comes near it; a scene created with unit_capacity=-1 holds every item in every tile, which grows with
# canvas area x items)
MAX_WORKSPACE_BYTES = 8 << 30

_CACHE: Dict[str, Tuple[LaunchConfig, Dict[str, float]]] = {}


def _key(scene: Scene, level: Optional[int], device) -> str:
    name = torch.cuda.get_device_name(device) if torch.cuda.is_available() else "none"
    lv = scene.level_ref if level is None else level
    return f"{scene.signature()}:{lv}:{scene.r_cut}:{scene.r_pad}:{name}"


def time_config(scene: Scene, level: Optional[int], cfg: LaunchConfig, epochs: int = 20, repeats: int = 3,
                device="cuda") -> float:
    """Median over `repeats` of the mean epoch time (ms) of `epochs` epochs from the scene's parameters."""
    cs = CollageScene(scene, level=level, device=device, **cfg.scene_kwargs())
    p0 = cs.params_tensor()
    p = p0.clone()
    m, v, st = cs.new_state()
    loss = torch.empty(cs.B, _lib.LOSS_TERMS, device=cs.device)
    grad = torch.empty(cs.N, 4, device=cs.device)
    stream = torch.cuda.Stream(cs.device)
    times: List[float] = []
    with torch.cuda.stream(stream):
        for r in range(repeats + 1):
            p.copy_(p0)
            m.zero_()
            v.zero_()
            st.zero_()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            cs.iterate_n(p, m, v, st, epochs, loss=loss, grad=grad, stream=stream)
            e1.record(stream)
            stream.synchronize()
            if r > 0:  # the first round warms up
                times.append(e0.elapsed_time(e1) / epochs)
    times.sort()
    return times[len(times) // 2]


def workspace_bytes(scene: Scene, level: Optional[int], cfg: LaunchConfig, device="cuda") -> int:
    """The workspace a configuration needs, without allocating it."""
    return CollageScene(scene, level=level, device=device, allocate_workspace=False, **cfg.scene_kwargs()).workspace_bytes


def tune(scene: Scene, level: Optional[int] = None, space: Optional[Iterable[LaunchConfig]] = None,
         epochs: int = 20, repeats: int = 3, device="cuda", cache_path: Optional[str] = None,
         force: bool = False, max_workspace_bytes: int = MAX_WORKSPACE_BYTES) -> Tuple[LaunchConfig, Dict[str, float]]:
    """Fastest configuration of `space` for `scene` at `level`, and the time (ms/epoch) of every one tried
    (candidates needing more than `max_workspace_bytes` of workspace are skipped)."""
    key = _key(scene, level, device)
    if not force:
        if key in _CACHE:
            return _CACHE[key]
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                disk = json.load(f)
            if key in disk:
                best = LaunchConfig(**disk[key]["best"])
                _CACHE[key] = (best, disk[key]["times"])
                return _CACHE[key]
    times: Dict[str, float] = {}
    best, best_t = None, float("inf")
    for cfg in (DEFAULT_SPACE if space is None else list(space)):
        if workspace_bytes(scene, level, cfg, device) > max_workspace_bytes:
            continue
        t = time_config(scene, level, cfg, epochs=epochs, repeats=repeats, device=device)
        times[json.dumps(asdict(cfg), sort_keys=True)] = t
        if t < best_t:
            best, best_t = cfg, t
    if best is None:
        raise ValueError("empty search space (or every candidate's workspace above max_workspace_bytes)")
    _CACHE[key] = (best, times)
    if cache_path:
        disk = {}
        if os.path.exists(cache_path):
            with open(cache_path) as f:
                disk = json.load(f)
        disk[key] = {"best": asdict(best), "times": times}
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(disk, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return best, times


def tune_levels(scene: Scene, levels: Optional[Iterable[int]] = None, **kw) -> Dict[int, LaunchConfig]:
    """One tuned configuration per level of the coarse-to-fine schedule."""
    return {int(L): tune(scene, level=int(L), **kw)[0] for L in (scene.levels if levels is None else levels)}
