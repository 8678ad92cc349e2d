"""GPU parity of faults switched inside the EMT time loop (emt_update_line): the scenario of the
paper's EMT fault study, a 10 ohm fault switched on at 10 ms and off at 30 ms over 60 ms of
20 us steps on the 179-bus network (3000 steps), applied to the stored inverse by the exact local
rebuild of Algorithm 2.

* Every engine (per-kernel, fused, one workgroup per leaf with exchange or owner-computed coupling
  levels, panels of cases) against the oracle's trajectory with the same scheduled changes
  (1e-10, normalised by the peak voltage), FP64 and FP32 + FP64 refinement, for a ground fault, a
  fault across a line inside a leaf and one across a line between two leaves, with line losses
  of the cases before and during the fault.
* Four line losses active together with a fault (the general SMW path) on four engines.
* A change that makes some case's G indefinite is refused and leaves the context as it was: the
  trajectory goes on bit for bit as if the call had not been made.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2105_10661_amd import cases

pytestmark = pytest.mark.gpu

DT = 20e-6
N_STEPS, ON, OFF = 3000, 500, 1500         # 60 ms; on at 10 ms, off at 30 ms
G_FAULT = 1.0 / 10.0


@pytest.fixture(scope="module")
def hv():
    import torch
    from paper_2105_10661_amd import hinv
    torch.cuda.set_device(0)
    hinv.load()
    return hinv


def _net():
    return dataclasses.replace(cases.net_179(), dt=DT)


def _fault(net, kind):
    """(a, b) of the fault: bus 1 to ground, or across a line inside a leaf / between two leaves."""
    if kind == "ground":
        return 1, -1
    same = net.bus_leaf[net.frm] == net.bus_leaf[net.to]
    e = int(np.nonzero(same if kind == "in_leaf" else ~same)[0][3])
    return int(net.frm[e]), int(net.to[e])


def _losses(net, a, b, n_cases):
    """Line losses of the cases: none, one before the fault, one while it is on (never the faulted line)."""
    touch = {a, b}
    br = [e for e in range(net.n_branch) if int(net.frm[e]) not in touch and int(net.to[e]) not in touch]
    all_lists = [[(200, br[5])], [], [(800, br[60])]]
    return all_lists[:n_cases]


_REF = {}


def _reference(net, kind, losses):
    key = (kind, str(losses))
    if key not in _REF:
        a, b = _fault(net, kind)
        ch = [(ON, a, b, G_FAULT), (OFF, a, b, -G_FAULT)]
        _REF[key] = [oracle.emt_run(net, N_STEPS, loss_steps=[s for s, _ in lst], loss_branches=[e for _, e in lst],
                                    solver="lu", changes=ch)[0] for lst in losses]
    return _REF[key]


def _run(hv, net, kind, losses, **kw):
    import torch
    a, b = _fault(net, kind)
    emt = hv.EMT(net, len(losses), losses=losses, **kw)
    V1, _ = emt.step(ON - 1)
    on = emt.update_line(a, b, G_FAULT)
    assert emt.next_step == ON
    V2, _ = emt.step(OFF - ON)
    emt.update_line(a, b, -G_FAULT)
    V3, _ = emt.step(N_STEPS - OFF + 1)
    V = torch.cat([V1, V2, V3]).cpu().numpy()
    emt.sync_status()
    emt.close()
    return V, on


ENGINES = [("per_kernel", 1), ("fused", 1), ("team", 1), ("level", 1), ("panel", 3)]


@pytest.mark.parametrize("kind", ["ground", "in_leaf", "between_leaves"])
@pytest.mark.parametrize("mode,n_cases", ENGINES)
def test_fault_scenario_fp64(hv, mode, n_cases, kind):
    net = _net()
    a, b = _fault(net, kind)
    losses = _losses(net, a, b, n_cases)
    print(f"[gpu] fault {kind} ({a},{b}) engine={mode} cases={n_cases} fp64", flush=True)
    V, info = _run(hv, net, kind, losses, prec="fp64", max_refine=0, max_mod_rank=2, kernel_mode=mode)
    refs = _reference(net, kind, losses)
    for k, ref in enumerate(refs):
        err = np.abs(V[:, k, :] - ref).max() / np.abs(ref).max()
        assert err <= 1e-10, (k, err)
    if kind == "between_leaves":
        assert info["leaves"] == 2 and info["lca_level"] >= 1
    else:
        assert info["leaves"] == 1 and info["lca_level"] == 0


@pytest.mark.parametrize("kind", ["ground", "between_leaves"])
@pytest.mark.parametrize("mode,n_cases", [("per_kernel", 2), ("fused", 1), ("team", 1), ("level", 1), ("panel", 3)])
def test_fault_scenario_fp64_incremental(hv, mode, n_cases, kind):
    """The incremental FP64 form (warm_start): its residual takes the step's G, so the switched fault's
    conductance enters through the residual as well as through the rebuilt inverse."""
    net = _net()
    a, b = _fault(net, kind)
    losses = _losses(net, a, b, n_cases)
    print(f"[gpu] fault {kind} ({a},{b}) engine={mode} cases={n_cases} fp64 incremental", flush=True)
    V, _ = _run(hv, net, kind, losses, prec="fp64", max_refine=0, max_mod_rank=1, warm_start=True, kernel_mode=mode)
    for k, ref in enumerate(_reference(net, kind, losses)):
        err = np.abs(V[:, k, :] - ref).max() / np.abs(ref).max()
        assert err <= 1e-10, (k, err)


@pytest.mark.parametrize("mode,n_cases", [("team", 1), ("level", 1), ("panel", 3), ("fused", 1)])
def test_fault_scenario_fp32_refined(hv, mode, n_cases):
    net = _net()
    kind = "in_leaf"
    a, b = _fault(net, kind)
    losses = _losses(net, a, b, n_cases)
    print(f"[gpu] fault {kind} engine={mode} cases={n_cases} fp32", flush=True)
    V, _ = _run(hv, net, kind, losses, prec="fp32", max_refine=2, max_mod_rank=2, kernel_mode=mode)
    for k, ref in enumerate(_reference(net, kind, losses)):
        err = np.abs(V[:, k, :] - ref).max() / np.abs(ref).max()
        assert err <= 1e-10, (k, err)


@pytest.mark.parametrize("mode,n_cases", [("team", 1), ("panel", 2)])
def test_refused_change_leaves_the_run_unchanged(hv, mode, n_cases):
    """A ground conductance change of -1.5 x bus a's shunt at a bus with one line keeps the base G
    positive definite but not the case that lost that line: the call fails and is undone."""
    import torch
    net = _net()
    deg = np.bincount(np.concatenate([net.frm, net.to]), minlength=net.n_bus)
    a = int(np.nonzero(deg == 1)[0][0])
    e = int(np.nonzero((net.frm == a) | (net.to == a))[0][0])
    dg = -1.5 * 2.0 * float(net.C[a]) / net.dt
    losses = [[(50, e)], []][:n_cases]
    kw = dict(prec="fp64", max_refine=0, max_mod_rank=2, kernel_mode=mode)
    print(f"[gpu] refused change at bus {a} (line {e}) engine={mode}", flush=True)
    ref = hv.EMT(net, n_cases, losses=losses, **kw)
    Vr, _ = ref.step(200)
    emt = hv.EMT(net, n_cases, losses=losses, **kw)
    Va, _ = emt.step(120)
    with pytest.raises(hv.HinvError) as ex:
        emt.update_line(a, -1, dg)
    assert ex.value.name in ("NOT_SPD", "SINGULAR")
    assert emt.next_step == 121
    Vb, _ = emt.step(80)
    assert np.array_equal(torch.cat([Va, Vb]).cpu().numpy(), Vr.cpu().numpy())
    emt.sync_status()
    emt.close()
    ref.close()


@pytest.mark.parametrize("mode", ["team", "level", "fused", "per_kernel"])
def test_four_line_losses_and_a_fault(hv, mode):
    """Rank-4 line changes (the general SMW path, beyond the rank-2 fast paths) active together
    with a fault switched on and off, against the oracle (1e-10, FP64)."""
    import torch
    net = _net()
    a, b = _fault(net, "ground")
    br = [e for e in range(net.n_branch) if 1 not in (int(net.frm[e]), int(net.to[e]))]
    losses = [[(60, br[3]), (90, br[40]), (90, br[77]), (130, br[150])]]
    print(f"[gpu] four losses and a fault, engine={mode}", flush=True)
    emt = hv.EMT(net, 1, losses=losses, prec="fp64", max_refine=0, max_mod_rank=4, kernel_mode=mode)
    V1, _ = emt.step(99)
    emt.update_line(a, b, G_FAULT)
    V2, _ = emt.step(100)
    emt.update_line(a, b, -G_FAULT)
    V3, _ = emt.step(101)
    V = torch.cat([V1, V2, V3])[:, 0, :].cpu().numpy()
    emt.sync_status()
    emt.close()
    lst = losses[0]
    ref = oracle.emt_run(net, 300, loss_steps=[s for s, _ in lst], loss_branches=[e for _, e in lst], solver="lu",
                         changes=[(100, a, b, G_FAULT), (200, a, b, -G_FAULT)])[0]
    assert np.abs(V - ref).max() / np.abs(ref).max() <= 1e-10
