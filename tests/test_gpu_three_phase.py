"""GPU parity on three-phase networks (each bus three rows, lines with mutual coupling between their
phases; the library's G from emt_network3_csr, the oracle's from assemble_G3): the exact hierarchical
inverse against the oracle's inverse (1e-12), FP32 storage with FP64 refinement (1e-10 per solve),
sampled solves at 2148 rows, the comparison baseline (sparse Cholesky) and the paper's approximation on
a three-phase tree."""
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


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def _solve_rows(X, B, G):
    Xo = oracle.solve(G, B)
    return (np.abs(X - Xo).max(1) / np.abs(Xo).max(1)).max()


def test_three_phase_inverse_179(hv):
    import torch
    net = cases.net_ring_fine(1, 1)
    rp, ci, cv = hv.network3_csr(net, cases.MUTUAL_RATIO)
    n = 3 * net.n_bus
    leaf = cases.phase_rows(net.bus_leaf)
    print(f"[gpu] three-phase inverse, {n} rows", flush=True)
    H = hv.Hierarchy(rp, ci, cv, net.parent, leaf, max_nrhs=n)
    V = H.solve(torch.eye(n, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    G3 = oracle.assemble_G3(net, cases.MUTUAL_RATIO)
    assert _rel(V.cpu().numpy().T, oracle.inverse(G3)) <= 1e-12
    info = H.info()
    assert info["n"] == n and info["max_leaf"] <= 128
    H.close()


@pytest.mark.parametrize("prec,refine", [("fp64", 0), ("fp32", 2)])
def test_three_phase_solves_2148_rows(hv, prec, refine):
    import torch
    net = cases.net_ring_fine(4, 7)
    rp, ci, cv = hv.network3_csr(net, cases.MUTUAL_RATIO)
    leaf = cases.phase_rows(net.bus_leaf)
    print(f"[gpu] three-phase solves, {3 * net.n_bus} rows, {prec}", flush=True)
    H = hv.Hierarchy(rp, ci, cv, net.parent, leaf, max_nrhs=4, prec=prec, max_refine=refine, rel_tol=1e-9)
    B = np.random.default_rng(12).standard_normal((4, 3 * net.n_bus))
    X = H.solve(torch.tensor(B, device="cuda")).cpu().numpy()
    H.sync_status()
    H.close()
    assert _solve_rows(X, B, oracle.assemble_G3(net, cases.MUTUAL_RATIO)) <= (1e-12 if prec == "fp64" else 1e-10)


def test_three_phase_cholesky_baseline(hv):
    import torch
    net = cases.net_ring_fine(4, 7)
    rp, ci, cv = hv.network3_csr(net, cases.MUTUAL_RATIO)
    print(f"[gpu] three-phase cholesky baseline, {3 * net.n_bus} rows", flush=True)
    C = hv.Chol(rp, ci, cv)
    B = np.random.default_rng(13).standard_normal((3, 3 * net.n_bus))
    X = C.solve(torch.tensor(B, device="cuda")).cpu().numpy()
    C.close()
    assert _solve_rows(X, B, oracle.assemble_G3(net, cases.MUTUAL_RATIO)) <= 1e-12


def test_three_phase_paper_approximation(hv):
    import torch
    net = cases.net_ring_fine(1, 1)
    rp, ci, cv = hv.network3_csr(net, cases.MUTUAL_RATIO)
    n = 3 * net.n_bus
    leaf = cases.phase_rows(net.bus_leaf)
    H = hv.Hierarchy(rp, ci, cv, net.parent, leaf, max_nrhs=n, coupling="paper", max_refine=0)
    V = H.solve(torch.eye(n, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    ref = oracle.paper_inverse(oracle.assemble_G3(net, cases.MUTUAL_RATIO), net.parent, leaf)
    assert _rel(V.cpu().numpy().T, ref) <= 1e-12
    H.close()


# ---------------------------------------------------------------------------
# Three-phase EMT time loop (emt3_create): 3x3 line companions and histories, losses of whole lines

@pytest.fixture(scope="module")
def ring3():
    """2-copy ring (358 buses, 1074 rows), mutual 0.3: oracle trajectories (dense LU, re-factorised at
    the loss) of a tie-line loss, a loss inside a copy, and an unbalanced drive with a loss."""
    net = cases.net_ring_fine(2, 21)
    n_steps = 3000
    runs = {"tie": ((1000, 528), oracle.BALANCED), "inner": ((1500, 40), oracle.BALANCED),
            "unbalanced": ((700, 300), (0.0, -1.9, 2.6))}
    print(f"[gpu] three-phase oracle runs, {3 * net.n_bus} rows x {n_steps} steps", flush=True)
    refs = {k: oracle.emt_run3(net, n_steps, cases.MUTUAL_RATIO, loss_steps=[ls[0]], loss_branches=[ls[1]],
                               shift=sh)[0] for k, (ls, sh) in runs.items()}
    return net, n_steps, runs, refs


@pytest.mark.timeout(600)
@pytest.mark.parametrize("engine", ["per_kernel", "fused"])
@pytest.mark.parametrize("prec,warm,refine", [("fp64", False, 0), ("fp32", True, 2)])
def test_three_phase_emt_ring_trajectories(hv, ring3, prec, warm, refine, engine):
    """Balanced cases batched (one tie-line loss, one loss inside a copy), the unbalanced one alone;
    every trajectory against the oracle, peak-normalised, 1e-10; one launch per phase and one
    workgroup per case."""
    import torch
    net, n_steps, runs, refs = ring3
    groups = [(["tie", "inner"], None), (["unbalanced"], runs["unbalanced"][1])]
    for names, shift in groups:
        print(f"[gpu] three-phase EMT {prec} {engine}: {names}", flush=True)
        emt = hv.EMT(net, len(names), losses=[[runs[k][0]] for k in names], prec=prec, max_refine=refine,
                     rel_tol=1e-7, warm_start=warm, max_mod_rank=3, mutual=cases.MUTUAL_RATIO, shift=shift,
                     kernel_mode=engine)
        assert emt.n == 3 * net.n_bus
        V = torch.empty((n_steps, len(names), emt.n), dtype=torch.float64, device="cuda")
        for c0 in range(0, n_steps, 500):
            emt.step(500, v_out=V[c0:c0 + 500])
        emt.sync_status()
        emt.close()
        Vh = V.cpu().numpy()
        for j, k in enumerate(names):
            err = np.abs(Vh[:, j, :] - refs[k]).max() / np.abs(refs[k]).max()
            print(f"[gpu]   {k}: {err:.2e}", flush=True)
            assert err <= 1e-10, (k, err)


def test_three_phase_lose_line_now_equals_scheduled(hv, ring3):
    """emt_lose_line on a three-phase handle (line index, all phases, rank 3) at the step a scheduled
    loss takes effect gives the same trajectory."""
    import torch
    net, n_steps, runs, refs = ring3
    (ls, line), _ = runs["tie"]
    print("[gpu] three-phase emt_lose_line", flush=True)
    a = hv.EMT(net, 1, losses=[[(ls, line)]], max_mod_rank=3, mutual=cases.MUTUAL_RATIO, kernel_mode="fused")
    b = hv.EMT(net, 1, max_mod_rank=3, mutual=cases.MUTUAL_RATIO, kernel_mode="fused")
    Va, _ = a.step(ls + 200)
    Vb1, _ = b.step(ls - 1)
    b.lose_line(0, line)
    Vb2, _ = b.step(201)
    torch.cuda.synchronize()
    Vb = torch.cat([Vb1, Vb2]).cpu().numpy()
    assert np.abs(Va.cpu().numpy() - Vb).max() <= 1e-13 * np.abs(refs["tie"]).max()
    assert np.abs(Vb[:, 0, :] - refs["tie"][:ls + 200]).max() <= 1e-10 * np.abs(refs["tie"]).max()
    with pytest.raises(hv.HinvError):
        b.lose_line(0, line)                  # already lost
    with pytest.raises(hv.HinvError):
        b.lose_line(0, 3)                     # rank 3 holds one line
    a.close()
    b.close()
