"""GPU parity of the panel engine (cases in panels of 16, one workgroup per leaf
per panel, leaf blocks applied to a panel on the matrix cores).

* Every case of a batch against the FP64 oracle's trajectory (1e-10,
  normalised by the peak voltage), FP64 and FP32 + FP64 refinement, with
  partial panels, rank-2 changes, a loss at step 1 and cases without losses.
* A case run in a batch equals the same case run alone bitwise: every column
  of a panel goes through the same operations (a matrix-core product's
  column depends on its own input column only).
* Identical inputs: the engine's recorded right-hand sides, solved by the
  oracle with the step's G, give the engine's recorded voltages (1e-10).
* Chunked stepping equals one launch bitwise; a loss requested between
  launches equals the same loss scheduled in advance.
* Degenerate tree (one leaf, no coupling level).
"""
import numpy as np
import pytest

import oracle
from paper_2105_10661_amd import cases

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hv():
    import torch
    from paper_2105_10661_amd import hinv
    torch.cuda.set_device(0)
    hinv.load()
    return hinv


def _peak_err(V, Vref):
    return np.abs(V - Vref).max() / np.abs(Vref).max()


# 20 cases: two panels, the second one partial
LOSSES_179 = ([[], [(1, 7)], [(40, 5)], [(10, 100), (70, 3)], [(55, 262)], [(200, 0)]]
              + [[(30 + 9 * k, (11 * k + 2) % 263)] for k in range(12)] + [[(5, 17), (5, 18)], []])


@pytest.fixture(scope="module")
def ref_179():
    net = cases.net_179()
    out = []
    for lst in LOSSES_179:
        V, _ = oracle.emt_run(net, 240, loss_steps=[s for s, _ in lst], loss_branches=[b for _, b in lst],
                              solver="lu")
        out.append(V)
    return net, out


@pytest.mark.parametrize("prec,warm", [("fp64", False), ("fp64", True), ("fp32", False), ("fp32", True)])
def test_panel_179_every_case_against_oracle(hv, ref_179, prec, warm):
    net, refs = ref_179
    print(f"[gpu] panel 179 x {len(LOSSES_179)} {prec} warm={warm}", flush=True)
    emt = hv.EMT(net, len(LOSSES_179), losses=LOSSES_179, prec=prec, max_refine=2, max_mod_rank=2,
                 warm_start=warm, kernel_mode="panel")
    V, _ = emt.step(240)
    emt.sync_status()
    Vb = V.cpu().numpy()
    errs = [_peak_err(Vb[:, k, :], refs[k]) for k in range(len(LOSSES_179))]
    print(f"[gpu] worst peak-normalised error {max(errs):.2e}", flush=True)
    assert max(errs) <= 1e-10
    if prec != "fp64":
        applies, rel = emt.stats()
        assert applies == len(LOSSES_179) * 240 * 3
        assert rel <= 1e-9
    emt.close()


def test_panel_batch_equals_alone_and_chunks(hv):
    net = cases.net_ring(8, 2)
    losses = [[(25, 40)], [], [(3, 2000), (60, 1)]]
    kw = dict(prec="fp64", max_mod_rank=2, kernel_mode="panel")
    print("[gpu] panel batch vs alone (1432 buses)", flush=True)
    emt = hv.EMT(net, len(losses), losses=losses, **kw)
    V, _ = emt.step(90)
    Vb = V.cpu().numpy()
    for k, lst in enumerate(losses):
        one = hv.EMT(net, 1, losses=[lst], **kw)
        V1, _ = one.step(90)
        assert np.array_equal(V1[:, 0, :].cpu().numpy(), Vb[:, k, :]), k
        one.close()
    # three launches of 30 steps equal one launch of 90
    ch = hv.EMT(net, len(losses), losses=losses, **kw)
    parts = [ch.step(30)[0].cpu().numpy() for _ in range(3)]
    assert np.array_equal(np.concatenate(parts), Vb)
    assert ch.next_step == 91
    ch.close()
    emt.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_panel_records_solve_their_rhs(hv, prec):
    """Per solve on identical inputs: oracle solve of the recorded b with the step's G."""
    net = cases.net_ring(4, 7)
    losses = [[(20, 33)], [(1, 500), (35, 600)]]
    emt = hv.EMT(net, 2, losses=losses, prec=prec, max_refine=2, max_mod_rank=2, kernel_mode="panel")
    V, B = emt.step(50, record_b=True)
    V, B = V.cpu().numpy(), B.cpu().numpy()
    for k, lst in enumerate(losses):
        for j in (0, 18, 19, 20, 34, 49):
            step = j + 1
            alive = np.ones(net.n_branch, np.uint8)
            for s, br in lst:
                if s <= step:
                    alive[br] = 0
            x = oracle.solve(oracle.assemble_G(net, alive), B[j, k])
            assert np.abs(V[j, k] - x).max() / np.abs(x).max() <= 1e-10, (k, j)
    emt.close()


def test_panel_dynamic_loss_equals_scheduled(hv):
    net = cases.net_ring(4, 7)
    kw = dict(prec="fp32", max_refine=2, max_mod_rank=2, kernel_mode="panel")
    ref = hv.EMT(net, 2, losses=[[(70, 11)], [(40, 3), (130, 900)]], **kw)
    Vr, _ = ref.step(200)
    dyn = hv.EMT(net, 2, losses=[[(70, 11)], [(40, 3)]], **kw)
    Va, _ = dyn.step(129)
    dyn.lose_line(1, 900)
    Vb, _ = dyn.step(71)
    import torch
    assert np.array_equal(torch.cat([Va, Vb]).cpu().numpy(), Vr.cpu().numpy())
    Vo, _ = oracle.emt_run(net, 200, loss_steps=[40, 130], loss_branches=[3, 900], solver="lu")
    assert _peak_err(Vr[:, 1, :].cpu().numpy(), Vo) <= 1e-10
    ref.close()
    dyn.close()


def test_panel_single_leaf_tree(hv):
    net = cases.small_network(40, 60, seed=9, d_th=40)
    assert net.n_leaves() == 1
    losses = [[(12, 3)], []]
    emt = hv.EMT(net, 2, losses=losses, prec="fp64", max_mod_rank=1, kernel_mode="panel")
    V, _ = emt.step(60)
    for k, lst in enumerate(losses):
        Vo, _ = oracle.emt_run(net, 60, loss_steps=[s for s, _ in lst], loss_branches=[b for _, b in lst],
                               solver="lu")
        assert _peak_err(V[:, k, :].cpu().numpy(), Vo) <= 1e-10
    emt.close()


def test_panel_refuses_what_it_cannot_hold(hv):
    # a 110-bus leaf exceeds the panel engine's 96-row limit; the automatic
    # choice falls back to the one-workgroup-per-case engine
    net = cases.small_network(110, 160, seed=4, d_th=110)
    assert net.n_leaves() == 1
    with pytest.raises(hv.HinvError) as ei:
        hv.EMT(net, 2, kernel_mode="panel")
    assert ei.value.name == "INVALID"
    emt = hv.EMT(net, 2, losses=[[], [(3, 5)]])
    V, _ = emt.step(20)
    Vo, _ = oracle.emt_run(net, 20, loss_steps=[3], loss_branches=[5], solver="lu")
    assert _peak_err(V[:, 1, :].cpu().numpy(), Vo) <= 1e-10
    emt.close()
