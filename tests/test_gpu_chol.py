"""GPU parity of the comparison baseline (sparse Cholesky of G, triangular solves on the GPU): solves
against the oracle's dense LU within 1e-12 (relative, per right-hand side), several right-hand sides in
one launch, and the reported counts."""
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


@pytest.mark.parametrize("name", ["c1-179", "ring4-716", "ring8-1432"])
def test_cholesky_solves_match_oracle(hv, name):
    import torch
    net = {"c1-179": cases.net_179(), "ring4-716": cases.net_ring(4, 7), "ring8-1432": cases.net_ring(8, 2)}[name]
    print(f"[gpu] cholesky baseline {name}", flush=True)
    C = hv.Chol.from_network(net)
    B = np.random.default_rng(4).standard_normal((5, net.n_bus))
    X = C.solve(torch.tensor(B, device="cuda")).cpu().numpy()
    Xo = oracle.solve(oracle.assemble_G(net), B)
    assert (np.abs(X - Xo).max(1) / np.abs(Xo).max(1)).max() <= 1e-12
    info = C.info()
    rp, _, _ = hv.network_csr(net)
    assert info["n"] == net.n_bus
    assert info["nnz_l"] >= (rp[-1] + net.n_bus) // 2
    assert info["solve_flops"] == 4.0 * (info["nnz_l"] - net.n_bus) + 2.0 * net.n_bus
    assert info["fwd_levels"] >= 1 and info["bwd_levels"] >= 1
    C.close()


def test_hierarchy_flop_counts_by_hand(hv):
    """hinv_get_info's FLOP counts on a two-leaf tree with one cut line, counted by hand."""
    net = cases.small_network(12, 16, seed=6)
    rp, ci, cv = hv.network_csr(net)
    leaf = np.where(np.arange(12) < 5, 1, 2).astype(np.int32)
    parent = np.array([-1, 0, 0], np.int32)
    G = oracle.assemble_G(net)
    cut = [(a, b) for a in range(5) for b in range(5, 12) if G[a, b] != 0.0]
    H = hv.Hierarchy(rp, ci, cv, parent, leaf)
    info = H.info()
    H.close()
    m = 2 * len(cut)
    n1, n2 = 5, 7
    apply = 2 * n1 ** 2 + 2 * n2 ** 2 + m + 2 * m ** 2 + 2 * n1 * len(cut) + 2 * n2 * len(cut)
    build = 2 * n1 ** 3 + 2 * n2 ** 3 + m ** 2 + 2 * m ** 3 + len(cut) * (n1 + n2)
    assert info["n_cols"] == m and info["apply_flops"] == apply and info["build_flops"] == build
