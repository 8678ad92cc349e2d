"""The allocation-free solve (hinv_solve_noalloc) against the workspace solve (hinv_solve).

Both run the same kernels with the same launch shapes on the same stored inverse; only the per-call
temporaries differ (the library's static device scratch instead of the handle's workspace), so the
results must agree bit for bit.  Each result is also checked against the FP64 oracle (dense LU of the
changed G) at 1e-10.  Two calls in a row, the second with fewer right-hand sides, then a call on a
smaller network: the scratch keeps the previous call's contents, which must not leak into a result.
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


def _check_calls(hv, net, lost, prec, sizes, seed):
    import torch
    g = oracle.branch_conductance(net)
    H = hv.Hierarchy.from_network(net, prec=prec, max_refine=2, max_nrhs=max(sizes), rel_tol=1e-9)
    alive = np.ones(net.n_branch, bool)
    for e in lost:
        H.modify_line(int(net.frm[e]), int(net.to[e]), -float(g[e]))
        alive[e] = False
    G = oracle.assemble_G(net, alive)
    rng = np.random.default_rng(seed)
    for k in sizes:
        print(f"[gpu] noalloc {net.n_bus} buses {prec} nrhs {k}", flush=True)
        B = rng.standard_normal((k, net.n_bus))
        X = torch.tensor(B, device="cuda")
        ref = H.solve(X)
        out = torch.full_like(X, float("nan"))
        H.solve_noalloc(X, out)          # hinv_solve_noalloc through the C ABI
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
        xo = oracle.solve(G, B)
        o = out.cpu().numpy()
        err = (np.abs(o - xo).max(1) / np.abs(xo).max(1)).max()
        assert err <= 1e-10, err
    H.sync_status()
    H.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_equals_workspace_solve(hv, prec):
    _check_calls(hv, cases.net_ring(8, 2), [5, 2110], prec, [40, 3], seed=1)
    _check_calls(hv, cases.net_179(), [17], prec, [2], seed=2)


def test_noalloc_rejects_oversize(hv):
    import torch
    net = cases.net_179()
    H = hv.Hierarchy.from_network(net, max_nrhs=1)
    X = torch.zeros((1 << 16, net.n_bus), dtype=torch.float64, device="cuda")   # 8 * 65536 * 4 * 179 B > 32 MiB
    with pytest.raises(hv.HinvError) as e:
        H.solve_noalloc(X, torch.empty_like(X))
    assert e.value.status == 1 and "scratch" in str(e.value)
    H.close()
