"""Autotuner: picks a configuration from its search space, caches it, and every configuration in the
space computes the same quantities as the oracle (the knobs change speed only)."""
import json
import sys

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2406_04008_amd import autotune
from paper_2406_04008_amd import scenes as S
from paper_2406_04008_amd.collage import CollageScene
from tests.parity_util import check_grad, check_image, check_loss

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def test_tune_picks_from_space_and_caches(tmp_path):
    sc = S.config1(0)
    space = [autotune.LaunchConfig(8, -1, 0), autotune.LaunchConfig(16, 0, 0), autotune.LaunchConfig(32, -1, 256)]
    path = str(tmp_path / "tune.json")
    _say("autotune config1")
    best, times = autotune.tune(sc, space=space, epochs=3, repeats=1, cache_path=path, force=True)
    assert best in space and len(times) == 3 and all(t > 0 for t in times.values())
    assert autotune.tune(sc, space=space)[0] == best  # in-memory cache
    autotune._CACHE.clear()
    assert autotune.tune(sc, space=space, cache_path=path)[0] == best  # file cache
    with open(path) as f:
        assert len(json.load(f)) == 1


def test_every_candidate_matches_oracle():
    sc = S.random_scene(11, [(45, 38), (70, 52), (24, 24)], [6, 14, 3], off_canvas=0.2)
    o = Oracle(sc)
    S_, Sp, L = o.forward(sc.params)
    g_ref = o.backward(sc.params)
    for cfg in autotune.DEFAULT_SPACE:
        _say("candidate", cfg)
        cs = CollageScene(sc, **cfg.scene_kwargs())
        cov, cov_pad, loss, grad = cs.forward_backward(cs.params_tensor())
        check_image(cov.cpu().numpy(), S_, "S")
        check_image(cov_pad.cpu().numpy(), Sp, "S_pad")
        check_loss(loss.cpu().numpy(), L)
        check_grad(grad.cpu().numpy(), g_ref)


def test_tune_skips_candidates_above_the_workspace_cap():
    """Small tiles need larger workspaces (more (tile, item) units, and per-tile arrays): the tuner
    times only the candidates whose workspace fits the cap, and the reported sizes order as expected."""
    sc = S.config3(0)
    small, large = autotune.LaunchConfig(32, -1, 0), autotune.LaunchConfig(8, -1, 0)
    _say("autotune workspace cap")
    ws_small = autotune.workspace_bytes(sc, 1024, small)
    ws_large = autotune.workspace_bytes(sc, 1024, large)
    assert ws_large > ws_small
    best, times = autotune.tune(sc, level=1024, space=[large, small], epochs=2, repeats=1, force=True,
                                max_workspace_bytes=ws_small)
    assert best == small and list(times) == [json.dumps({"bin_chunk": 0, "code_capacity": -1, "tile": 32})]
    with pytest.raises(ValueError):
        autotune.tune(sc, level=1024, space=[large], epochs=2, repeats=1, force=True, max_workspace_bytes=ws_small)
