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
