"""GPU parity at the benchmark configurations' full sizes.

The 11456-bus (8x8 torus) network runs on the level engine (its coupling
levels do not fit every workgroup's LDS, so they are computed by the owners
of their columns) and on the per-kernel engine; the oracle there is the library sparse LU of G (SuperLU), pinned
against the dense LU on the 179-bus network.  The 256-case contingency batch
runs on the one-workgroup-per-case engine and on the panel engine; sampled
cases are checked against full oracle trajectories and against the same case
run alone on the same engine (bitwise).
Tolerance: 1e-10 relative (per solve: per-vector infinity norm; trajectories:
normalised by the peak voltage).
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


@pytest.mark.parametrize("shape", [(8, 8), (4, 8)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_torus_per_solve_random(hv, shape, prec):
    import torch
    net = cases.net_torus(*shape, seed=3)
    print(f"[gpu] torus {shape} {prec} per-solve", flush=True)
    H = hv.Hierarchy.from_network(net, prec=prec, max_refine=3, max_nrhs=4, rel_tol=1e-9)
    info = H.info()
    assert info["n"] == net.n_bus and info["n_leaves"] == net.n_leaves()
    B = np.random.default_rng(11).standard_normal((4, net.n_bus))
    X = H.solve(torch.tensor(B, device="cuda")).cpu().numpy()
    solve = oracle.sparse_solver(net)
    for k in range(4):
        ref = solve(B[k])
        assert np.abs(X[k] - ref).max() / np.abs(ref).max() <= 1e-10
    H.close()


@pytest.mark.parametrize("prec,mode", [("fp64", "auto"), ("fp32", "auto"), ("fp64", "per_kernel")])
def test_torus_11456_trajectory_with_loss(hv, prec, mode):
    net = cases.net_torus(8, 8, seed=3)
    steps = 300
    loss = (120, 4321)
    print(f"[gpu] 11456 trajectory {prec} {mode}", flush=True)
    Vref, _ = oracle.emt_run(net, steps, loss_steps=[loss[0]], loss_branches=[loss[1]], solver="sparse")
    emt = hv.EMT(net, 1, losses=[[loss]], prec=prec, max_refine=2, rel_tol=1e-9, kernel_mode=mode)
    V, _ = emt.step(steps)
    Vg = V[:, 0, :].cpu().numpy()
    assert np.abs(Vg - Vref).max() / np.abs(Vref).max() <= 1e-10
    emt.close()


@pytest.mark.parametrize("mode,prec,warm", [("fused", "fp32", True), ("fused", "fp64", True), ("panel", "fp32", True),
                                            ("panel", "fp32", False), ("panel", "fp64", False), ("panel", "fp64", True)])
def test_contingency_batch_256(hv, mode, prec, warm):
    base, bcases = cases.cases_c4(n_cases=256, n_steps=1200, step_range=(1, 900))
    losses = [list(zip(c.loss_steps.tolist(), c.loss_branches.tolist())) for c in bcases]
    print(f"[gpu] 256-case batch {mode} {prec} warm={warm}", flush=True)
    kw = dict(prec=prec, max_refine=2, rel_tol=1e-9, warm_start=warm, max_mod_rank=1, kernel_mode=mode)
    emt = hv.EMT(base, 256, losses=losses, **kw)
    V, _ = emt.step(1200)
    Vb = V.cpu().numpy()
    for k in (0, 77, 200, 255):
        st, br = losses[k][0]
        Vref, _ = oracle.emt_run(base, 1200, loss_steps=[st], loss_branches=[br], solver="inv")
        assert np.abs(Vb[:, k, :] - Vref).max() / np.abs(Vref).max() <= 1e-10, k
    emt.sync_status()
    for k in (3, 130):
        one = hv.EMT(base, 1, losses=[losses[k]], **kw)
        V1, _ = one.step(1200)
        assert np.array_equal(V1[:, 0, :].cpu().numpy(), Vb[:, k, :]), k
        one.close()
    emt.close()
