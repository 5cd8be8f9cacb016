"""The unit pools: (screen tile, item) work units live in a pool per layout sized by the scene's unit
capacity, numbered without gaps (a tile's first unit is the count of its layout's units in earlier tiles,
an item's first map entry the count of units of earlier items), instead of one slot per item per tile.

* With the default capacity no standard workload overflows, and every output is bitwise the one of a
  scene whose pools have room for every item in every tile (the numbering does not depend on the
  capacity, and no sum depends on where a unit is stored).
* A layout whose units do not fit its pool in an epoch is reported in the status word
  COLLAGE_STATUS_UNIT_OVERFLOW, lists no units (coverage and gradient 0) and nothing is written outside
  the workspace.
* The default pools are much smaller than the dense ones on a large canvas.
"""
import numpy as np
import pytest
import torch

from paper_2406_04008_amd import _lib
from paper_2406_04008_amd import scenes as S
from paper_2406_04008_amd.collage import CollageScene

pytestmark = pytest.mark.gpu

CASES = [("config1", None, 16), ("config2", None, 8), ("config3", 512, 32), ("config3", 1024, 8),
         ("config5", 2048, 32)]


@pytest.mark.parametrize("name,level,tile", CASES, ids=[f"{c[0]}-{c[1]}-T{c[2]}" for c in CASES])
def test_default_pool_matches_the_dense_pool_bitwise(name, level, tile):
    print(f"[case] unit pool {name} level {level} tile {tile}", flush=True)
    sc = getattr(S, name)(0)
    outs = []
    for cap in (0, -1):
        cs = CollageScene(sc, level=level, tile=tile, unit_capacity=cap)
        p = cs.params_tensor()
        m, v, st = cs.new_state()
        loss = torch.empty(cs.B, _lib.LOSS_TERMS, device="cuda")
        grad = torch.empty(cs.N, 4, device="cuda")
        cs.iterate_n(p, m, v, st, 5, loss=loss, grad=grad)
        cov, cov_pad, l2, g2 = cs.forward_backward(p)
        status = cs.status()
        assert status[_lib.STATUS_UNIT_OVERFLOW] == 0, (cap, status)
        assert status[_lib.STATUS_GRAD_RANGE] == 0, (cap, status)
        outs.append((cov, cov_pad, l2, g2, p.clone(), loss.clone()))
    for a, b in zip(outs[0], outs[1]):
        assert torch.equal(a, b)


def test_overflowing_pool_is_reported():
    print("[case] unit pool overflow", flush=True)
    sc = S.config2(0)
    cs = CollageScene(sc, tile=8, unit_capacity=64)
    p = cs.params_tensor()
    cov, cov_pad, _, g = cs.forward_backward(p)
    status = cs.status()
    assert status[_lib.STATUS_UNIT_OVERFLOW] == sc.num_layouts, status
    assert float(cov.abs().max()) == 0.0 and float(cov_pad.abs().max()) == 0.0
    assert float(g.abs().max()) == 0.0
    # the same parameters with a pool that fits: none reported, and coverage is there
    ok = CollageScene(sc, tile=8)
    cov, _, _, _ = ok.forward_backward(p)
    assert ok.status()[_lib.STATUS_UNIT_OVERFLOW] == 0
    assert float(cov.max()) > 0.5


@pytest.mark.parametrize("tile,limit", [(32, 1.0), (8, 1.0)])
def test_default_pool_is_small_on_a_large_canvas(tile, limit):
    sc = S.config5(0)
    dense = CollageScene(sc, level=2048, tile=tile, unit_capacity=-1, allocate_workspace=False)
    pool = CollageScene(sc, level=2048, tile=tile, allocate_workspace=False)
    print(f"[case] workspace 2048^2 T={tile}: dense {dense.workspace_bytes / 2**30:.2f} GiB, "
          f"pool {pool.workspace_bytes / 2**30:.2f} GiB", flush=True)
    assert pool.workspace_bytes < limit * 2**30
    assert pool.workspace_bytes < 0.5 * dense.workspace_bytes
