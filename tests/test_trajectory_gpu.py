"""GPU trajectories of the larger workloads, checked step-wise against the FP64 oracle.

As for config 1 (test_config1_run_gpu.py), layouts after many epochs are not unique, so at sampled epochs
the loss terms and the gradient that the GPU epoch computed (collage_iterate, one epoch per call) are
compared with the oracle at exactly the parameters that epoch started from, to the workload's
tolerances.  Late epochs are where the items' gradients are small remainders of their pixels'
contributions, so these are the epochs that test the precision of the coverage and of its derivative.

One decision is taken in float32 on the GPU: the nearest edge of a pixel (the scan; its neighbours are
re-decided in float64).  Where another edge that is not a neighbour lies within float32 resolution of the
nearest distance, the pixel sits on a medial axis of the outline to that resolution, the loss has a kink
there, and either edge's gradient terms are a correct result; shrinking items (s near 0) have many such
pixels.  The gradient bar of each item is therefore widened by the oracle's bound on what those pixels
can change (Oracle.nearest_ambiguity at a resolution of 2^-20 (1 + |p - k t|) px, above the float32
error of the scan's distances), and is unchanged for every item without such a pixel.
"""
import numpy as np
import pytest
import torch

from oracle.oracle import Oracle
from paper_2406_04008_amd import _lib
from paper_2406_04008_amd import scenes as S
from paper_2406_04008_amd.collage import CollageScene
from tests.parity_util import check_grad, check_loss

pytestmark = pytest.mark.gpu

# distance resolution of the float32 scan: the pixel's position relative to the item's origin (rounded
# once from double) and the edge's line-frame constants carry errors of a few 2^-24 of their size
AMBIGUITY_ABS = 2.0 ** -20
AMBIGUITY_REL = 2.0 ** -20

CASES = [
    # scene, level, epochs, check every
    ("config2", None, 150, 3),
    ("config3", 128, 300, 10),
    ("config3", 512, 300, 60),
]


@pytest.mark.parametrize("name,level,epochs,every", CASES, ids=[f"{c[0]}-{c[1]}" for c in CASES])
def test_trajectory_stepwise_against_the_oracle(name, level, epochs, every):
    print(f"[case] {name} level {level}: {epochs} epochs, every {every}", flush=True)
    sc = getattr(S, name)(0)
    o = Oracle(sc, level=level)
    cs = CollageScene(sc, level=level)
    p = cs.params_tensor()
    m, v, st = cs.new_state()
    loss = torch.empty(cs.B, _lib.LOSS_TERMS, device="cuda")
    grad = torch.empty(sc.num_shapes, 4, device="cuda")
    first = last = None
    widened = 0
    for epoch in range(epochs):
        check = epoch % every == 0 or epoch == epochs - 1
        p_before = p.detach().cpu().numpy().copy() if check else None
        cs.iterate(p, m, v, st, loss=loss, grad=grad)
        if check:
            _, _, L = o.forward(p_before)
            check_loss(loss.cpu().numpy(), L, f"{name} loss at epoch {epoch}")
            slack = o.nearest_ambiguity(p_before, AMBIGUITY_ABS, AMBIGUITY_REL)
            widened += int((slack.sum(1) > 0).sum())
            check_grad(grad.cpu().numpy(), o.backward(p_before), f"{name} grad at epoch {epoch}", slack=slack)
            last = float(L.sum())
            first = last if first is None else first
    torch.cuda.synchronize()
    print(f"{name}: loss {first:.4g} -> {last:.4g}; item bars widened {widened} times", flush=True)
    assert np.all(np.isfinite(p.cpu().numpy()))
    assert last < first, (first, last)
