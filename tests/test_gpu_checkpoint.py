"""Checkpoint and resume of the EMT time loop (emt_state_size / emt_save_state / emt_load_state).

* Resume on a fresh handle of the same network, tree, engine and precision equals the uninterrupted
  run bitwise: scheduled losses before and after the checkpoint, a dynamic loss (emt_lose_line) and a
  base-matrix change (emt_update_line, replayed by the load) before it; every engine (per-kernel,
  one workgroup per case, panels of cases, one workgroup per leaf with exchange or owner-computed
  coupling levels), FP64 and FP32 + FP64 refinement.
* Resume on another engine, which rounds differently: the continued trajectory within 1e-10 of the
  oracle's (peak-normalised), with the same losses and change.
* Refusals leave the handle as it was: another network, a corrupt header, a short buffer, a handle
  whose own base-matrix changes diverge from the state's, more losses than max_mod_rank holds.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2105_10661_amd import cases

pytestmark = pytest.mark.gpu

N1, N2 = 200, 200            # steps before and after the checkpoint
G_FAULT = 0.05               # base-matrix change switched on at step N1 / 2


@pytest.fixture(scope="module")
def hv():
    import torch
    from paper_2105_10661_amd import hinv
    torch.cuda.set_device(0)
    hinv.load()
    return hinv


def _scenario(net, n_cases, seed):
    """Per case one scheduled loss (at a random step before or after the checkpoint), a dynamic loss
    of case 1 (case 0 if it is the only one) from step N1 / 2 + 1, and a fault across a line between
    two leaves in force from the same step."""
    rng = np.random.default_rng(seed)
    br = rng.choice(net.n_branch, n_cases + 1, replace=False)
    st = rng.integers(20, N1 + N2 - 20, n_cases)
    losses = [[(int(st[k]), int(br[k]))] for k in range(n_cases)]
    dyn = (min(1, n_cases - 1), int(br[n_cases]))
    e = int(np.nonzero(net.bus_leaf[net.frm] != net.bus_leaf[net.to])[0][2])
    fault = (int(net.frm[e]), int(net.to[e]), G_FAULT)
    return losses, dyn, fault


def _run_a(hv, net, kw, losses, dyn, fault):
    """Uninterrupted run: step to N1 / 2, change G and lose the dynamic line, step to N1, save, step N2."""
    import torch
    a = hv.EMT(net, len(losses), losses=losses, **kw)
    Va1, _ = a.step(N1 // 2)
    a.update_line(*fault)
    a.lose_line(*dyn)
    Va2, _ = a.step(N1 - N1 // 2)
    state = a.save_state()
    Va3, _ = a.step(N2)
    torch.cuda.synchronize()
    a.sync_status()
    a.close()
    return torch.cat([Va1, Va2]).cpu().numpy(), state, Va3.cpu().numpy()


ENGINES = [("per_kernel", 3), ("fused", 3), ("panel", 20), ("team", 1), ("level", 1)]


RESUME_CASES = ([(e, n, "fp64", False, 0) for e, n in ENGINES] + [(e, n, "fp32", True, 2) for e, n in ENGINES]
                # the incremental FP64 form (v carries over from step to step); the panel's incremental layout
                # takes one change per case, this scenario two
                + [(e, n, "fp64", True, 0) for e, n in ENGINES if e in ("per_kernel", "fused", "team", "level")])


@pytest.mark.parametrize("engine,n_cases,prec,warm,refine", RESUME_CASES)
def test_resume_is_bitwise(hv, engine, n_cases, prec, warm, refine):
    import torch
    net = cases.net_ring(8, 4) if engine in ("panel", "team", "level") else cases.net_179()
    losses, dyn, fault = _scenario(net, n_cases, 11)
    kw = dict(prec=prec, max_refine=refine, rel_tol=1e-7, warm_start=warm, max_mod_rank=2, kernel_mode=engine)
    print(f"[gpu] checkpoint {engine} {prec}: {n_cases} cases, {net.n_bus} buses", flush=True)
    _, state, Va3 = _run_a(hv, net, kw, losses, dyn, fault)
    b = hv.EMT(net, n_cases, losses=losses, **kw)
    b.load_state(state)
    assert b.next_step == N1 + 1
    Vb3, _ = b.step(N2)
    torch.cuda.synchronize()
    b.sync_status()
    b.close()
    assert np.array_equal(Va3, Vb3.cpu().numpy())


def _oracle(net, losses, dyn, fault, k):
    ls = [s for s, _ in losses[k]]
    lb = [e for _, e in losses[k]]
    if k == dyn[0]:
        ls.append(N1 // 2 + 1)
        lb.append(dyn[1])
    V, _ = oracle.emt_run(net, N1 + N2, loss_steps=ls, loss_branches=lb, solver="inv",
                          changes=[(N1 // 2 + 1, fault[0], fault[1], fault[2])])
    return V


@pytest.mark.parametrize("src,dst", [("panel", "fused"), ("fused", "per_kernel"), ("team", "level")])
def test_resume_on_another_engine(hv, src, dst):
    """The state carries no engine-specific layout: rows and branches are in the network's order."""
    net = cases.net_ring(8, 4)
    n_cases = 1 if src == "team" else 17
    losses, dyn, fault = _scenario(net, n_cases, 12)
    kw = dict(prec="fp64", max_refine=0, rel_tol=1e-7, max_mod_rank=2)
    print(f"[gpu] checkpoint {src} -> {dst}: {n_cases} cases", flush=True)
    Va12, state, Va3 = _run_a(hv, net, dict(kw, kernel_mode=src), losses, dyn, fault)
    b = hv.EMT(net, n_cases, losses=losses, kernel_mode=dst, **kw)
    b.load_state(state)
    Vb3, _ = b.step(N2)
    b.sync_status()
    Vb3 = Vb3.cpu().numpy()
    b.close()
    for k in sorted({0, dyn[0], n_cases - 1}):
        ref = _oracle(net, losses, dyn, fault, k)
        peak = np.abs(ref).max()
        assert np.abs(Va12[:, k] - ref[:N1]).max() / peak <= 1e-10
        assert np.abs(Vb3[:, k] - ref[N1:]).max() / peak <= 1e-10, k


def test_refusals_leave_the_handle_unchanged(hv):
    import torch
    net = cases.net_179()
    losses, dyn, fault = _scenario(net, 2, 13)
    kw = dict(prec="fp64", max_mod_rank=2, kernel_mode="fused")
    _, state, Va3 = _run_a(hv, net, kw, losses, dyn, fault)
    b = hv.EMT(net, 2, losses=losses, **kw)
    bad = state.copy()
    bad[0] ^= 0xFF
    other = dataclasses.replace(net, R=net.R * 1.01)
    o = hv.EMT(other, 2, losses=losses, **kw)
    for what, call in (("magic", lambda: b.load_state(bad)),
                       ("short", lambda: b.load_state(state[:-8])),
                       ("network", lambda: o.load_state(state))):
        with pytest.raises(hv.HinvError) as e:
            call()
        assert e.value.name == "INVALID", what
    o.close()
    # a handle with a base-matrix change the state does not have
    c = hv.EMT(net, 2, losses=losses, **kw)
    c.update_line(fault[0], fault[1], 2 * fault[2])
    with pytest.raises(hv.HinvError) as e:
        c.load_state(state)
    assert e.value.name == "INVALID"
    c.close()
    # rank: the state's case 1 holds two losses; a handle of max_mod_rank 1 cannot take them
    d = hv.EMT(net, 2, losses=[[], []], prec="fp64", max_mod_rank=1, kernel_mode="fused")
    with pytest.raises(hv.HinvError) as e:
        d.load_state(state)
    assert e.value.name == "RANK_LIMIT"
    d.close()
    assert b.next_step == 1
    b.load_state(state)
    Vb3, _ = b.step(N2)
    torch.cuda.synchronize()
    b.close()
    assert np.array_equal(Va3, Vb3.cpu().numpy())


@pytest.mark.parametrize("engine", ["fused", "panel"])
def test_change_of_g_after_dynamic_losses(hv, engine):
    """A change of G reloads every case's line losses; with dynamic losses added, the changes outnumber
    the columns the handle's scratch was sized for at creation (one per scheduled loss), so they are
    formed in groups.  Trajectories against the oracle, 1e-10."""
    import torch
    net = cases.net_ring(8, 4)
    n_cases = 17
    losses, _, fault = _scenario(net, n_cases, 14)
    rng = np.random.default_rng(15)
    dyn = [(int(k), int(b)) for k, b in zip((0, 5, 16), rng.choice(net.n_branch, 3, replace=False))
           if all(b != e for _, e in losses[k])]
    print(f"[gpu] change of G after {len(dyn)} dynamic losses ({engine})", flush=True)
    emt = hv.EMT(net, n_cases, losses=losses, prec="fp64", max_mod_rank=2, kernel_mode=engine)
    V1, _ = emt.step(N1 // 2)
    for k, b in dyn:
        emt.lose_line(k, b)
    emt.update_line(*fault)
    V2, _ = emt.step(N2)
    torch.cuda.synchronize()
    emt.sync_status()
    V = torch.cat([V1, V2]).cpu().numpy()
    emt.close()
    for k, b in dyn:
        ls = [s for s, _ in losses[k]] + [N1 // 2 + 1]
        lb = [e for _, e in losses[k]] + [b]
        ref, _ = oracle.emt_run(net, N1 // 2 + N2, loss_steps=ls, loss_branches=lb, solver="inv",
                                changes=[(N1 // 2 + 1, fault[0], fault[1], fault[2])])
        assert np.abs(V[:, k] - ref).max() / np.abs(ref).max() <= 1e-10, k


def test_three_phase_batch_with_more_changes_than_cases(hv):
    """Three-phase: each lost line is three changes, so ten cases with one loss each hold thirty
    changes against a scratch of ten columns.  Every case against the oracle's three-phase loop."""
    import torch
    net = cases.net_ring_fine(2, 6)
    rng = np.random.default_rng(16)
    br = rng.choice(net.n_branch, 10, replace=False)
    st = rng.integers(20, 150, 10)
    losses = [[(int(s), int(b))] for s, b in zip(st, br)]
    print("[gpu] three-phase batch of 10 cases, 30 changes", flush=True)
    emt = hv.EMT(net, 10, losses=losses, prec="fp64", max_mod_rank=3, mutual=cases.MUTUAL_RATIO,
                 kernel_mode="fused")
    V, _ = emt.step(200)
    torch.cuda.synchronize()
    emt.sync_status()
    V = V.cpu().numpy()
    emt.close()
    for k in (0, 4, 9):
        ref, _ = oracle.emt_run3(net, 200, cases.MUTUAL_RATIO, loss_steps=[int(st[k])], loss_branches=[int(br[k])])
        assert np.abs(V[:, k] - ref).max() / np.abs(ref).max() <= 1e-10, k
