"""GPU parity of the build's largest capacitance-inversion path (order above 1024: S assembled by
``k_fill_s``, inverted by one launch pair per pivot step), which no benchmark tree reaches: two
128-bus leaves joined by 600 distinct lines, so the root has 1200 coupling columns.

* The exact inverse against the oracle's (1e-12, relative max-norm).
* A line update at the root equals a fresh build of the changed G bit for bit.
* The paper's approximation (S^{-1} replaced by C on that path) against the oracle's Algorithm 1.
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


def _two_halves(n_half=128, n_cross=600, seed=3):
    rng = np.random.default_rng(seed)
    frm, to = [], []
    for base in (0, n_half):
        for i in range(1, n_half):                 # a random tree inside each half
            frm.append(base + i)
            to.append(base + int(rng.integers(i)))
    pairs = set()
    while len(pairs) < n_cross:
        pairs.add((int(rng.integers(n_half)), n_half + int(rng.integers(n_half))))
    for a, b in sorted(pairs):
        frm.append(a)
        to.append(b)
    nb = len(frm)
    return cases.Network(
        name="two 128-bus halves, 600 cross lines", n_bus=2 * n_half,
        frm=np.asarray(frm, np.int32), to=np.asarray(to, np.int32),
        R=rng.uniform(0.5, 5.0, nb), L=rng.uniform(1e-3, 1e-2, nb), C=rng.uniform(1e-6, 1e-5, 2 * n_half),
        src_bus=np.zeros(0, np.int32), src_amp=np.zeros(0), src_phase=np.zeros(0),
        parent=np.array([-1, 0, 0], np.int32),
        bus_leaf=np.repeat(np.array([1, 2], np.int32), n_half))


def _inverse(H, n):
    import torch
    V = H.solve(torch.eye(n, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    return V.cpu().numpy().T


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def test_root_of_order_1200(hv):
    net = _two_halves()
    n = net.n_bus
    rp, ci, cv = hv.network_csr(net)
    print("[gpu] build with a root of order 1200", flush=True)
    H = hv.Hierarchy(rp, ci, cv, net.parent, net.bus_leaf, max_nrhs=n)
    assert H.info()["max_cols"] == 1200
    G = oracle.assemble_G(net)
    Gi = _inverse(H, n)
    assert _rel(Gi, oracle.inverse(G)) <= 1e-12
    # a line at the root: local rebuild == fresh build
    g = oracle.branch_conductance(net)
    e = net.n_branch - 7
    a, b, dg = int(net.frm[e]), int(net.to[e]), -0.5 * float(g[e])
    info = H.update_line(a, b, dg)
    assert info["lca_level"] == 1 and info["nodes"] == 1
    cv2 = cv.copy()
    for r, c, d in ((a, a, dg), (b, b, dg), (a, b, -dg), (b, a, -dg)):
        cv2[rp[r] + int(np.nonzero(ci[rp[r]:rp[r + 1]] == c)[0][0])] += d
    F = hv.Hierarchy(rp, ci, cv2, net.parent, net.bus_leaf, max_nrhs=n)
    Gu = _inverse(H, n)
    assert np.array_equal(Gu, _inverse(F, n))
    w = np.zeros(n)
    w[a], w[b] = 1.0, -1.0
    assert _rel(Gu, oracle.inverse(G + dg * np.outer(w, w))) <= 1e-12
    H.close()
    F.close()


def test_root_of_order_1200_paper_mode(hv):
    net = _two_halves()
    n = net.n_bus
    rp, ci, cv = hv.network_csr(net)
    H = hv.Hierarchy(rp, ci, cv, net.parent, net.bus_leaf, max_nrhs=n, coupling="paper", max_refine=0)
    ref = oracle.paper_inverse(oracle.assemble_G(net), net.parent, net.bus_leaf)
    assert _rel(_inverse(H, n), ref) <= 1e-12
    H.close()
