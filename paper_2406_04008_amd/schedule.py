"""Coarse-to-fine optimization schedule (Sec. 4.3 and the hierarchical rows of Table 1).

The layout is optimized at a sequence of increasing resolutions.  Parameters are held in canonical
(reference-level) pixels, so a level switch hands them over unchanged; what changes per level is the
scale k = level / level_ref of the rasterization, the container mask rasterized at that level, and the
learning rates (0.5 level px).  The Adam state is restarted at every level, because the loss changes
scale roughly with the pixel count.

Each level runs as ONE captured hipGraph: the Adam reset followed by all of the level's epochs
(transform, binning, coverage, loss, adjoint, update), replayed with a single launch.  All levels share
the parameter, moment and gradient buffers, so the graphs chain on one stream with no host work between
them.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib
from .collage import CollageScene
from .scenes import Scene


@dataclass
class LevelRun:
    level: int
    steps: int
    tile: int
    loss: Optional[np.ndarray] = None    # [B,9] weighted terms of the level's last epoch
    params: Optional[np.ndarray] = None  # [N,4] parameters at the end of the level
    gpu_ms: float = 0.0                  # HIP-event time of the level's graph launch


@dataclass
class ScheduleResult:
    levels: List[LevelRun] = field(default_factory=list)
    params: Optional[np.ndarray] = None
    gpu_ms: float = 0.0
    wall_s: float = 0.0

    @property
    def epochs(self) -> int:
        return sum(l.steps for l in self.levels)


class CoarseToFine:
    """Runs `scene` through `levels` (default: the scene's own), `steps_per_level` epochs each.

    tile, code_capacity, bin_chunk: the launch configuration of every level (0 / -1 / 0: library
    defaults); `configs` ({level: autotune.LaunchConfig}, e.g. from autotune.tune_levels) overrides them
    per level.
    """

    def __init__(self, scene: Scene, levels: Optional[Sequence[int]] = None, steps_per_level: Optional[int] = None,
                 tile: int = 0, code_capacity: int = -1, bin_chunk: int = 0, device="cuda",
                 lr_px: Optional[float] = None, use_graphs: bool = True, configs: Optional[dict] = None):
        self.scene = scene
        self.levels = [int(x) for x in (scene.levels if levels is None else levels)]
        if not self.levels:
            raise ValueError("no levels")
        self.steps = int(scene.steps_per_level if steps_per_level is None else steps_per_level)
        if not (1 <= self.steps <= 4096):
            raise ValueError("steps_per_level must be 1..4096 (one captured graph per level)")
        self.device = torch.device(device)
        self.lr_px = scene.lr_px if lr_px is None else float(lr_px)
        self.use_graphs = use_graphs
        configs = configs or {}
        plain = {"tile": tile, "code_capacity": code_capacity, "bin_chunk": bin_chunk}
        self.scenes = [CollageScene(scene, level=L, device=self.device,
                                    **(configs[L].scene_kwargs() if L in configs else plain)) for L in self.levels]
        N, B = scene.num_shapes, scene.num_layouts
        dev = self.device
        self.params = torch.zeros(N, 4, device=dev)
        self.m = torch.zeros(N, 4, device=dev)
        self.v = torch.zeros(N, 4, device=dev)
        self.step = torch.zeros(1, dtype=torch.int32, device=dev)
        self.grad = torch.zeros(N, 4, device=dev)
        self.losses = [torch.zeros(B, _lib.LOSS_TERMS, device=dev) for _ in self.levels]
        self.stream = torch.cuda.Stream(dev)
        self.graphs = None
        if use_graphs:
            torch.cuda.synchronize(dev)
            self.graphs = [cs.graph(self.params, self.m, self.v, self.step, self.losses[i], self.grad,
                                    lr_px=self.lr_px, replays_per_launch=self.steps, stream=self.stream,
                                    reset_adam=True)
                           for i, cs in enumerate(self.scenes)]

    def run(self, params=None, keep_level_params: bool = True) -> ScheduleResult:
        """Optimizes from `params` (default: the scene's initial parameters) through every level."""
        p0 = self.scenes[0].params_tensor(params)
        res = ScheduleResult()
        torch.cuda.synchronize(self.device)
        self.params.copy_(p0)
        torch.cuda.synchronize(self.device)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(self.levels) + 1)]
        snaps = []
        t0 = time.perf_counter()
        with torch.cuda.stream(self.stream):
            ev[0].record(self.stream)
            for i, cs in enumerate(self.scenes):
                if self.graphs is not None:
                    self.graphs[i].launch(1)
                else:
                    cs.reset_state(self.m, self.v, self.step)
                    for _ in range(self.steps):
                        cs.iterate(self.params, self.m, self.v, self.step, loss=self.losses[i], grad=self.grad,
                                   lr_px=self.lr_px)
                ev[i + 1].record(self.stream)
                if keep_level_params:
                    snaps.append(self.params.clone())
        self.stream.synchronize()
        res.wall_s = time.perf_counter() - t0
        for i, L in enumerate(self.levels):
            lr = LevelRun(level=L, steps=self.steps, tile=self.scenes[i].tile)
            lr.loss = self.losses[i].cpu().numpy()
            lr.gpu_ms = ev[i].elapsed_time(ev[i + 1])
            if keep_level_params:
                lr.params = snaps[i].cpu().numpy()
            res.levels.append(lr)
        res.gpu_ms = ev[0].elapsed_time(ev[-1])
        res.params = self.params.cpu().numpy()
        return res
