"""GPU parity of the team engine on trees with three and four coupling levels (the 179-bus network,
bisection trees of leaf size 24 and 12), and of the level engine on trees of one to five levels.  Each coupling column's sum is formed in one phase from the
leaf results through a precomputed row that folds in the corrections of every lower level, so these
trees check that fold through more than one level; the benchmark trees have two.

* FP64 and FP32 + FP64 refinement against the oracle (1e-10, normalised by the peak voltage), with a
  line loss and a 10 ohm fault to ground switched on and off (the rows are rebuilt after each
  switching).
* A tree with five coupling levels is refused by the team engine with a clear error.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2105_10661_amd import cases

pytestmark = pytest.mark.gpu

N_STEPS, LOSS, ON, OFF = 400, 100, 150, 300


@pytest.fixture(scope="module")
def hv():
    import torch
    from paper_2105_10661_amd import hinv
    torch.cuda.set_device(0)
    hinv.load()
    return hinv


def _net(d_th):
    net = cases.net_179()
    parent, leaf = cases.threshold_tree(net.pos, d_th)
    return dataclasses.replace(net, parent=parent, bus_leaf=leaf)


_REF = {}


def _reference(d_th):
    if d_th not in _REF:
        net = _net(d_th)
        ch = [(ON, 1, -1, 0.1), (OFF, 1, -1, -0.1)]
        _REF[d_th] = oracle.emt_run(net, N_STEPS, loss_steps=[LOSS], loss_branches=[5], solver="lu",
                                    changes=ch)[0]
    return _REF[d_th]


@pytest.mark.parametrize("d_th", [24, 12])
@pytest.mark.parametrize("prec,refine,warm", [("fp64", 0, False), ("fp32", 2, True)])
def test_team_deep_tree_with_loss_and_fault(hv, d_th, prec, refine, warm):
    import torch
    net = _net(d_th)
    print(f"[gpu] team engine, leaf size {d_th}, {prec}", flush=True)
    emt = hv.EMT(net, 1, losses=[[(LOSS, 5)]], prec=prec, max_refine=refine, warm_start=warm,
                 max_mod_rank=2, kernel_mode="team")
    V1, _ = emt.step(ON - 1)
    emt.update_line(1, -1, 0.1)
    V2, _ = emt.step(OFF - ON)
    emt.update_line(1, -1, -0.1)
    V3, _ = emt.step(N_STEPS - OFF + 1)
    V = torch.cat([V1, V2, V3])[:, 0, :].cpu().numpy()
    emt.sync_status()
    emt.close()
    ref = _reference(d_th)
    assert np.abs(V - ref).max() / np.abs(ref).max() <= 1e-10


def test_team_refuses_five_levels(hv):
    net = _net(6)
    with pytest.raises(hv.HinvError) as ex:
        hv.EMT(net, 1, kernel_mode="team")
    assert ex.value.name == "INVALID"


_RING = {}


@pytest.mark.parametrize("prec,refine,warm", [("fp64", 0, False), ("fp32", 2, True)])
def test_team_wide_ring_with_scheduled_and_dynamic_losses(hv, prec, refine, warm):
    """A 12-copy ring (2148 buses, 24 leaves): each workgroup keeps only the rows of each S^{-1} whose
    y it applies, which is what lets this tree fit the team engine in FP64.  A scheduled loss and a
    loss requested between launches add X rows to some workgroups (new needed columns)."""
    import torch
    net = cases.net_ring(12, 21)
    steps, s1, s2 = 300, 60, 180
    b1, b2 = 7, net.n_branch - 5          # a line inside copy 0, a tie line
    if "ref" not in _RING:
        _RING["ref"] = oracle.emt_run(net, steps, loss_steps=[s1, s2], loss_branches=[b1, b2], solver="sparse")[0]
    ref = _RING["ref"]
    print(f"[gpu] team engine, 12-copy ring, {prec}", flush=True)
    emt = hv.EMT(net, 1, losses=[[(s1, b1)]], prec=prec, max_refine=refine, warm_start=warm, max_mod_rank=2,
                 kernel_mode="team")
    V1, _ = emt.step(s2 - 1)
    emt.lose_line(0, b2)
    V2, _ = emt.step(steps - s2 + 1)
    V = torch.cat([V1, V2])[:, 0, :].cpu().numpy()
    emt.sync_status()
    emt.close()
    assert np.abs(V - ref).max() / np.abs(ref).max() <= 1e-10


@pytest.mark.parametrize("d_th", [90, 24, 12, 6])
@pytest.mark.parametrize("prec,refine,warm", [("fp64", 0, False), ("fp32", 2, True)])
def test_level_engine_trees_of_one_to_five_levels(hv, d_th, prec, refine, warm):
    """The level engine on bisection trees of 1 to 5 coupling levels (leaf sizes 90, 24, 12, 6): one
    barrier per apply at the top level, every other exchange as tagged values (a single-level tree keeps
    the barrier for the final values), with a line loss and a fault switched on and off."""
    import torch
    net = _net(d_th)
    print(f"[gpu] level engine, leaf size {d_th}, {prec}", flush=True)
    emt = hv.EMT(net, 1, losses=[[(LOSS, 5)]], prec=prec, max_refine=refine, warm_start=warm,
                 max_mod_rank=2, kernel_mode="level")
    V1, _ = emt.step(ON - 1)
    emt.update_line(1, -1, 0.1)
    V2, _ = emt.step(OFF - ON)
    emt.update_line(1, -1, -0.1)
    V3, _ = emt.step(N_STEPS - OFF + 1)
    V = torch.cat([V1, V2, V3])[:, 0, :].cpu().numpy()
    emt.sync_status()
    emt.close()
    ref = _reference(d_th)
    assert np.abs(V - ref).max() / np.abs(ref).max() <= 1e-10
