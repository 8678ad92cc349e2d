"""C-ABI checks that need no GPU: symbols, host-side validation, G assembly.

The workspace-size and CSR calls run only host code (no HIP call), so they
can be exercised here; everything that launches kernels is in the gpu tests.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2105_10661_amd import cases

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def hv():
    from paper_2105_10661_amd import hinv
    if not os.path.exists(hinv.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    hinv.load()
    return hinv


def _declared():
    txt = open(os.path.join(ROOT, "include", "hinv.h")).read()
    return sorted(set(re.findall(r"^\s*(?:hinv_status|const char\*)\s+(\w+)\s*\(", txt, re.M)))


def test_exports_every_declared_symbol(hv):
    lib = ctypes.CDLL(hv.LIB_PATH)
    names = _declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(hv.EXPORTS)


def _arrays(rp, ci, cv, parent, leaf):
    c = np.ascontiguousarray
    return [c(rp, np.int32), c(ci, np.int32), c(cv, np.float64), c(parent, np.int32), c(leaf, np.int32)]


def _ws_size(hv, rp, ci, cv, parent, leaf, **opt):
    lib = hv.load()
    arrs = _arrays(rp, ci, cv, parent, leaf)
    csr = hv._CSR(len(arrs[0]) - 1, hv._ptr(arrs[0]), hv._ptr(arrs[1]), hv._ptr(arrs[2]))
    tree = hv._Tree(len(arrs[3]), hv._ptr(arrs[3]), hv._ptr(arrs[4]))
    o = dict(prec="fp64", rel_tol=1e-13, max_refine=2, max_mod_rank=2, max_nrhs=1)
    o.update(opt)
    op = hv._options(**o)
    nb = ctypes.c_size_t(0)
    st = lib.hinv_workspace_size(ctypes.byref(csr), ctypes.byref(tree), ctypes.byref(op), ctypes.byref(nb))
    return st, nb.value


def test_library_assembles_the_oracle_G(hv):
    for net in (cases.net_179(), cases.net_ring(8, 2), cases.small_network(9, 14, seed=2)):
        rp, ci, cv = hv.network_csr(net)
        n = net.n_bus
        G = np.zeros((n, n))
        for r in range(n):
            G[r, ci[rp[r]:rp[r + 1]]] = cv[rp[r]:rp[r + 1]]
        Go = oracle.assemble_G(net)
        assert np.array_equal(G != 0, Go != 0)
        assert np.abs(G - Go).max() <= 4 * np.finfo(float).eps * np.abs(Go).max()


def test_workspace_size_accepts_config_networks(hv):
    for net in (cases.net_179(), cases.net_ring(8, 2)):
        rp, ci, cv = hv.network_csr(net)
        st, nb = _ws_size(hv, rp, ci, cv, net.parent, net.bus_leaf)
        assert st == 0 and nb > 0
        st32, nb32 = _ws_size(hv, rp, ci, cv, net.parent, net.bus_leaf, prec="fp32")
        assert st32 == 0 and nb32 > nb


def test_rejects_bad_inputs(hv):
    net = cases.net_179()
    rp, ci, cv = hv.network_csr(net)
    P, L = net.parent.copy(), net.bus_leaf.copy()
    INVALID, NOT_SPD = 1, 2
    # asymmetric value
    cv2 = cv.copy()
    r = 5
    j = rp[r] + (1 if ci[rp[r]] == r else 0)
    cv2[j] *= 1.5
    assert _ws_size(hv, rp, ci, cv2, P, L)[0] == INVALID
    # non-positive diagonal
    cv3 = cv.copy()
    d = [e for e in range(rp[3], rp[4]) if ci[e] == 3][0]
    cv3[d] = -1.0
    assert _ws_size(hv, rp, ci, cv3, P, L)[0] == NOT_SPD
    # column out of range
    ci2 = ci.copy()
    ci2[-1] = net.n_bus
    assert _ws_size(hv, rp, ci2, cv, P, L)[0] == INVALID
    # two roots
    P2 = P.copy()
    P2[1] = -1
    assert _ws_size(hv, rp, ci, cv, P2, L)[0] == INVALID
    # cycle
    P3 = P.copy()
    P3[0] = 3
    assert _ws_size(hv, rp, ci, cv, P3, L)[0] == INVALID
    # bus assigned to an internal node
    L2 = L.copy()
    L2[0] = 0
    assert _ws_size(hv, rp, ci, cv, P, L2)[0] == INVALID
    # leaf larger than the limit: one leaf for 179 buses
    assert _ws_size(hv, rp, ci, cv, np.array([-1], np.int32), np.zeros(179, np.int32))[0] == INVALID
    # options
    assert _ws_size(hv, rp, ci, cv, P, L, prec=7)[0] == INVALID
    assert _ws_size(hv, rp, ci, cv, P, L, max_nrhs=0)[0] == INVALID
    assert _ws_size(hv, rp, ci, cv, P, L, max_mod_rank=99)[0] == INVALID
    msg = hv.load().hinv_last_error().decode()
    assert "max_mod_rank" in msg


def test_emt_validation(hv):
    lib = hv.load()
    net = cases.net_179()
    na = hv._NetArrays(net)
    ptr, st, br = hv._case_arrays(2, [[(5, 3)], [(7, 3), (9, 3)]])      # case 1 loses branch 3 twice
    cs = hv._Cases(2, hv._ptr(ptr), hv._ptr(st), hv._ptr(br))
    op = hv._options("fp64", 1e-13, 2, 2, 1)
    nb = ctypes.c_size_t(0)
    assert lib.emt_workspace_size(ctypes.byref(na.s), ctypes.byref(na.tree), ctypes.byref(op), ctypes.byref(cs),
                                  ctypes.byref(nb)) == 1
    ptr, st, br = hv._case_arrays(2, [[(5, 3)], [(7, 4), (9, 3)]])
    cs = hv._Cases(2, hv._ptr(ptr), hv._ptr(st), hv._ptr(br))
    assert lib.emt_workspace_size(ctypes.byref(na.s), ctypes.byref(na.tree), ctypes.byref(op), ctypes.byref(cs),
                                  ctypes.byref(nb)) == 0
    op1 = hv._options("fp64", 1e-13, 2, 1, 1)                          # rank limit 1 < 2 losses
    assert lib.emt_workspace_size(ctypes.byref(na.s), ctypes.byref(na.tree), ctypes.byref(op1), ctypes.byref(cs),
                                  ctypes.byref(nb)) == 7
    bad = cases.net_179()
    bad.to = bad.to.copy()
    bad.to[0] = bad.frm[0]                                             # self loop
    nb2 = hv._NetArrays(bad)
    assert lib.emt_workspace_size(ctypes.byref(nb2.s), ctypes.byref(nb2.tree), ctypes.byref(op), ctypes.byref(cs),
                                  ctypes.byref(nb)) == 1


def _chol_ws(hv, rp, ci, cv):
    lib = hv.load()
    c = np.ascontiguousarray
    a = [c(rp, np.int32), c(ci, np.int32), c(cv, np.float64)]
    csr = hv._CSR(len(a[0]) - 1, hv._ptr(a[0]), hv._ptr(a[1]), hv._ptr(a[2]))
    nb = ctypes.c_size_t(0)
    return lib.chol_workspace_size(ctypes.byref(csr), ctypes.byref(nb)), nb.value


def test_cholesky_baseline_host_factorization(hv):
    """The comparison baseline's host factorization: sizes an SPD G, rejects an indefinite one."""
    net = cases.net_179()
    rp, ci, cv = hv.network_csr(net)
    st, nb = _chol_ws(hv, rp, ci, cv)
    assert st == 0 and nb > 8 * rp[-1]
    st, _ = _chol_ws(hv, np.array([0, 2, 4]), np.array([0, 1, 0, 1]), np.array([1.0, 2.0, 2.0, 1.0]))
    assert hv.STATUS[st] == "NOT_SPD"
    st, _ = _chol_ws(hv, np.array([0, 0]), np.array([], np.int32), np.array([]))
    assert hv.STATUS[st] == "INVALID"


def test_three_phase_G_matches_oracle(hv):
    """The library's three-phase G (closed-form 3x3 companions) against the oracle's (3x3 inverse)."""
    net = cases.net_ring_fine(2, 5)
    rp, ci, cv = hv.network3_csr(net, cases.MUTUAL_RATIO)
    n = 3 * net.n_bus
    G = np.zeros((n, n))
    for r in range(n):
        G[r, ci[rp[r]:rp[r + 1]]] = cv[rp[r]:rp[r + 1]]
    ref = oracle.assemble_G3(net, cases.MUTUAL_RATIO)
    assert np.abs(G - ref).max() <= 1e-14 * np.abs(ref).max()
    lib = hv.load()
    na = hv._NetArrays(net)
    nnz = ctypes.c_int64(0)
    assert hv.STATUS[lib.emt_network3_csr(ctypes.byref(na.s), 0.5, None, None, None, ctypes.byref(nnz))] == "INVALID"


def test_emt3_validation(hv):
    """emt3_workspace_size (host only): a line loss takes three of max_mod_rank, the three-phase loop
    runs on the per-kernel engine only, and the mutual ratio and phase shifts are checked."""
    lib = hv.load()
    net = cases.net_ring_fine(2, 5)
    na = hv._NetArrays(net)
    nb = ctypes.c_size_t(0)

    def size(losses, rank, mode="auto", mutual=cases.MUTUAL_RATIO, shift=None):
        ptr, st, br = hv._case_arrays(2, losses)
        cs = hv._Cases(2, hv._ptr(ptr), hv._ptr(st), hv._ptr(br))
        op = hv._options("fp64", 1e-9, 2, rank, 1, False, mode)
        sh = None if shift is None else np.ascontiguousarray(shift, np.float64)
        return hv.STATUS[lib.emt3_workspace_size(ctypes.byref(na.s), float(mutual), hv._ptr(sh), ctypes.byref(na.tree),
                                                 ctypes.byref(op), ctypes.byref(cs), ctypes.byref(nb))]

    assert size([[(5, 3)], []], 3) == "OK" and nb.value > 0
    assert size([[(5, 3)], []], 2) == "RANK_LIMIT"                    # one line loss = rank 3
    assert size([[(5, 3), (9, 4)], [(7, 10)]], 6) == "OK"
    assert size([[(5, 3), (9, 4)], [(7, 10)]], 5) == "RANK_LIMIT"
    assert size([[(5, net.n_branch)], []], 3) == "INVALID"           # lines, not phase branches
    assert size([[(5, 3)], []], 3, mode="panel") == "INVALID"
    assert size([[(5, 3)], []], 3, mode="per_kernel") == "OK"
    assert size([[(5, 3)], []], 3, mode="fused") == "OK"
    assert size(None, 3, mutual=0.5) == "INVALID"
    assert size(None, 3, shift=[0.0, np.nan, 1.0]) == "INVALID"
    assert size(None, 3, shift=[0.0, 0.0, 0.0]) == "OK"
    big = cases.net_ring(2, 5)                                        # 45-bus leaves: 135 rows > 128
    nbig = hv._NetArrays(big)
    ptr, st, br = hv._case_arrays(1, None)
    cs = hv._Cases(1, hv._ptr(ptr), hv._ptr(st), hv._ptr(br))
    op = hv._options("fp64", 1e-9, 2, 3, 1)
    assert hv.STATUS[lib.emt3_workspace_size(ctypes.byref(nbig.s), 0.3, None, ctypes.byref(nbig.tree),
                                             ctypes.byref(op), ctypes.byref(cs), ctypes.byref(nb))] == "INVALID"
