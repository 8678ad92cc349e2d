"""Pins of the FP64 oracle against things other than itself.

Each check ties one part of the oracle to the mathematics: library routines
(numpy / scipy), an independent state-space formulation of the same circuit,
closed-form solutions, conservation identities and structural properties of
G.  A plausible slip in the oracle (wrong sign of a history term, a dropped
conductance, a transposed incidence, a wrong initial condition, a swapped
pivot) fails at least one of them.
"""
import numpy as np
import pytest
import scipy.linalg

import oracle
from paper_2105_10661_amd import cases


def _net_from(n_bus, frm, to, R, L, C, src_bus, amp, phase, dt, freq=60.0):
    parent, bus_leaf = np.array([-1], np.int32), np.zeros(n_bus, np.int32)
    return cases.Network(name="hand", n_bus=n_bus, frm=np.asarray(frm, np.int32), to=np.asarray(to, np.int32),
                         R=np.asarray(R, float), L=np.asarray(L, float), C=np.asarray(C, float),
                         src_bus=np.asarray(src_bus, np.int32), src_amp=np.asarray(amp, float),
                         src_phase=np.asarray(phase, float), parent=parent, bus_leaf=bus_leaf, dt=dt, freq=freq)


# --------------------------------------------------------------------------
# G: structure (Section II: real, symmetric conductance matrix)
# --------------------------------------------------------------------------

def test_G_structure_179():
    net = cases.net_179()
    G = oracle.assemble_G(net)
    assert np.array_equal(G, G.T)
    off = G - np.diag(np.diag(G))
    assert (off <= 0).all()
    # each branch touches exactly 4 entries: count the off-diagonal non-zeros
    assert np.count_nonzero(off) == 2 * net.n_branch
    # row sums: branch terms cancel, leaving the shunt conductance 2C/dt
    rs = G.sum(1)
    assert np.allclose(rs, 2 * net.C / net.dt, rtol=0, atol=1e-15 * np.abs(G).max() * 8)
    np.linalg.cholesky(G)                      # SPD (library Cholesky succeeds)
    # the sparse assembly is the same matrix
    Gs = oracle.sparse_G(net).toarray()
    assert np.array_equal(Gs != 0, G != 0)
    assert np.abs(Gs - G).max() <= 4 * np.finfo(float).eps * np.abs(G).max()


def test_G_removed_branch_is_rank_one_change():
    net = cases.net_179()
    e = 17
    alive = np.ones(net.n_branch, np.uint8)
    alive[e] = 0
    G = oracle.assemble_G(net)
    Gp = oracle.assemble_G(net, alive)
    D = G - Gp
    a, b = net.frm[e], net.to[e]
    nz = np.argwhere(D != 0)
    assert sorted(map(tuple, nz)) == sorted([(a, a), (a, b), (b, a), (b, b)])
    assert np.linalg.matrix_rank(D) == 1


# --------------------------------------------------------------------------
# LU solve / explicit inverse (Eq. (2)) against library routines
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 7, 64, 200])
def test_lu_solve_matches_numpy(n):
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n)) + 0.1 * np.eye(n)     # general matrix: pivoting matters
    b = rng.standard_normal(n)
    x = oracle.solve(A, b)
    xr = np.linalg.solve(A, b)
    assert np.abs(x - xr).max() <= 1e-10 * max(1.0, np.abs(xr).max())


def test_lu_needs_pivoting():
    A = np.array([[0.0, 2.0, 1.0], [1.0, 0.0, 0.0], [3.0, 1.0, 0.0]])
    b = np.array([1.0, 2.0, 3.0])
    np.testing.assert_allclose(oracle.solve(A, b), np.linalg.solve(A, b), rtol=1e-14)
    with pytest.raises(np.linalg.LinAlgError):
        oracle.solve(np.zeros((3, 3)), b)


def test_solve_many_rows():
    net = cases.net_179()
    G = oracle.assemble_G(net)
    B = np.random.default_rng(0).standard_normal((5, net.n_bus))
    X = oracle.solve(G, B)
    np.testing.assert_allclose(X, scipy.linalg.solve(G, B.T, assume_a="pos").T, rtol=1e-10, atol=0)


def test_inverse_properties_179():
    net = cases.net_179()
    G = oracle.assemble_G(net)
    Gi = oracle.inverse(G)
    n = net.n_bus
    kappa = np.linalg.cond(G)
    assert np.abs(G @ Gi - np.eye(n)).max() <= 50 * kappa * np.finfo(float).eps
    assert np.abs(Gi - Gi.T).max() <= 1e-12 * np.abs(Gi).max()
    # G is an irreducible Stieltjes matrix (connected network): G^{-1} > 0 entrywise
    assert Gi.min() > 0
    np.testing.assert_allclose(Gi, np.linalg.inv(G), rtol=1e-10, atol=0)


def test_sparse_solver_matches_dense():
    net = cases.net_179()
    G = oracle.assemble_G(net)
    b = np.random.default_rng(1).standard_normal(net.n_bus)
    x1 = oracle.sparse_solver(net)(b)
    x2 = oracle.solve(G, b)
    assert np.abs(x1 - x2).max() <= 1e-12 * np.abs(x2).max()


# --------------------------------------------------------------------------
# Time loop (Eq. (1)) against closed forms and an independent formulation
# --------------------------------------------------------------------------

def test_capacitor_only_bus_is_trapezoidal_sum():
    """No branches: C dv/dt = u; trapezoid gives v_n = sum_k dt/(2C) (u_k + u_{k-1})."""
    dt, C, A, ph, f = 1e-4, 3e-6, 1.7, 0.4, 60.0
    net = _net_from(1, [], [], [], [], [C], [0], [A], [ph], dt, f)
    V, _ = oracle.emt_run(net, 200)
    t = np.arange(0, 201) * dt
    u = A * np.sin(2 * np.pi * f * t + ph)
    ref = np.cumsum(dt / (2 * C) * (u[1:] + u[:-1]))
    np.testing.assert_allclose(V[:, 0], ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def _state_space_run(net, n_steps, loss_steps=(), loss_branches=()):
    """Independent check: trapezoidal (Tustin) rule on the state x = (bus voltages, branch currents).

    C_a dv_a/dt = u_a - sum_e A[a,e] i_e ;  L_e di_e/dt = v_from - v_to - R_e i_e.
    x_n = x_{n-1} + dt/2 (f_n(x_n) + f_{n-1}(x_{n-1})), a lost branch's current
    is held at zero from its loss step on.  Start: x_0 = 0.
    """
    n, m, dt = net.n_bus, net.n_branch, net.dt
    A = np.zeros((n, m))
    A[net.frm, np.arange(m)] = 1.0
    A[net.to, np.arange(m)] = -1.0
    dead_from = np.full(m, 1 << 60)
    for s, e in zip(loss_steps, loss_branches):
        dead_from[e] = s

    def jac(step):
        alive = (dead_from > step).astype(float)
        K = np.zeros((n + m, n + m))
        K[:n, n:] = -(A * alive) / net.C[:, None]
        K[n:, :n] = (A.T / net.L[:, None]) * alive[:, None]
        K[n:, n:] = np.diag(-net.R / net.L * alive)
        return K, alive

    def src(step):
        u = np.zeros(n + m)
        t = step * dt
        np.add.at(u, net.src_bus, net.src_amp * np.sin(2 * np.pi * net.freq * t + net.src_phase))
        u[:n] /= net.C
        return u

    x = np.zeros(n + m)
    out = np.zeros((n_steps, n))
    Kp, _ = jac(0)
    for step in range(1, n_steps + 1):
        K, alive = jac(step)
        rhs = x + dt / 2 * (Kp @ x + src(step - 1) + src(step))
        M = np.eye(n + m) - dt / 2 * K
        dead = np.where(alive == 0)[0] + n          # algebraic rows: i_e = 0
        M[dead, :] = 0.0
        M[dead, dead] = 1.0
        rhs[dead] = 0.0
        x = np.linalg.solve(M, rhs)
        out[step - 1] = x[:n]
        Kp = K
    return out


def test_matches_state_space_trapezoid_small():
    net = cases.small_network(7, 10, seed=3)
    V, _ = oracle.emt_run(net, 600, solver="lu")
    ref = _state_space_run(net, 600)
    assert np.abs(V - ref).max() <= 1e-9 * np.abs(ref).max()


def test_matches_state_space_trapezoid_with_line_loss():
    net = cases.small_network(8, 12, seed=5)
    V, _ = oracle.emt_run(net, 500, loss_steps=[137], loss_branches=[4], solver="inv")
    ref = _state_space_run(net, 500, loss_steps=[137], loss_branches=[4])
    assert np.abs(V - ref).max() <= 1e-9 * np.abs(ref).max()
    # the loss visibly changes the trajectory (the check is not vacuous)
    V0, _ = oracle.emt_run(net, 500, solver="inv")
    assert np.abs(V0 - ref).max() > 1e-3 * np.abs(ref).max()


def test_converges_to_continuous_solution_second_order():
    """2-bus R-L-C circuit with a 60 Hz source: error vs the exact ODE solution shrinks ~4x per dt/2."""
    R, L, C0, C1, A, ph, f = 1.0, 1e-2, 1e-3, 2e-3, 1.3, 0.7, 60.0
    T = 0.02
    w = 2 * np.pi * f
    # exact: augmented linear system z = (v0, v1, i, sin, cos), z' = M z
    M = np.array([[0, 0, -1 / C0, A / C0, 0],
                  [0, 0, 1 / C1, 0, 0],
                  [1 / L, -1 / L, -R / L, 0, 0],
                  [0, 0, 0, 0, w],
                  [0, 0, 0, -w, 0]], float)
    z0 = np.array([0, 0, 0, np.sin(ph), np.cos(ph)])
    exact = (scipy.linalg.expm(M * T) @ z0)[:2]
    errs = []
    for dt in (2e-4, 1e-4, 5e-5, 2.5e-5):
        net = _net_from(2, [0], [1], [R], [L], [C0, C1], [0], [A], [ph], dt, f)
        V, _ = oracle.emt_run(net, int(round(T / dt)), solver="lu")
        errs.append(np.abs(V[-1] - exact).max())
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(ratios > 3.6) and np.all(ratios < 4.4), (errs, ratios)


def test_discrete_charge_balance_across_loss():
    """Summing KCL over all buses: (2/dt) sum_a C_a (v_a^n - v_a^{n-1}) = sum_a (i_in^n + i_in^{n-1})."""
    case = cases.case_c1(n_steps=400)
    net = case.net
    V, _ = oracle.emt_run(net, 400, loss_steps=[150], loss_branches=[33])
    Vp = np.vstack([np.zeros(net.n_bus), V])
    lhs = (2 / net.dt) * ((Vp[1:] - Vp[:-1]) * net.C).sum(1)
    t = np.arange(0, 401) * net.dt
    u = np.array([oracle.source_current(net, tt).sum() for tt in t])
    rhs = u[1:] + u[:-1]
    scale = (2 / net.dt) * (np.abs(Vp[1:] - Vp[:-1]) * net.C).sum(1) + np.abs(rhs)
    assert np.all(np.abs(lhs - rhs) <= 1e-9 * scale.max())


def test_kcl_residual_every_step():
    case = cases.case_c1(n_steps=200)
    net = case.net
    V, B = oracle.emt_run(net, 200, record_b=True, solver="inv")
    G = oracle.assemble_G(net)
    r = B - V @ G.T
    assert np.abs(r).max() <= 1e-9 * np.abs(G).max() * np.abs(V).max()


def test_solver_variants_agree_fp64_floor():
    """LU vs explicit inverse vs sparse LU on the 179-bus network, 1000 steps, with a loss."""
    case = cases.case_c1()
    net = case.net
    kw = dict(loss_steps=[400], loss_branches=[100])
    Vi, _ = oracle.emt_run(net, 1000, solver="inv", **kw)
    Vl, _ = oracle.emt_run(net, 1000, solver="lu", **kw)
    Vs, _ = oracle.emt_run(net, 1000, solver="sparse", **kw)
    peak = np.abs(Vl).max()
    assert np.abs(Vi - Vl).max() <= 1e-11 * peak
    assert np.abs(Vs - Vl).max() <= 1e-11 * peak


def test_generator_is_deterministic():
    a = cases.net_ring(8, 2)
    b = cases.net_ring(8, 2)
    for k in ("frm", "to", "R", "L", "C", "src_bus", "src_amp", "src_phase", "parent", "bus_leaf"):
        assert np.array_equal(getattr(a, k), getattr(b, k))
    c = cases.net_ring(8, 3)
    k = 8 * cases.BASE_BRANCHES                 # copies share the topology; tie lines are drawn
    assert not np.array_equal(a.R, c.R) and np.array_equal(a.frm[:k], c.frm[:k])


# ---------------------------------------------------------------------------
# The paper's approximate inverse (Section III.A-B, Algorithm 1)

def _two_leaf_tree(n, split):
    parent = np.array([-1, 0, 0], np.int32)
    leaf = np.where(np.arange(n) < split, 1, 2).astype(np.int32)
    return parent, leaf


def test_paper_inverse_two_by_two_closed_form():
    a, b, d = 3.0, -0.7, 2.5
    G = np.array([[a, b], [b, d]])
    parent, leaf = _two_leaf_tree(2, 1)
    Gt = oracle.paper_inverse(G, parent, leaf)
    ref = np.array([[1 / a, -b / (a * d)], [-b / (a * d), 1 / d]])
    assert np.abs(Gt - ref).max() <= 1e-15


def test_paper_inverse_zeroes_the_off_diagonal_blocks_of_G_times_it():
    """Eq. (5)-(6): M is chosen so that G G~^{-1} has zero off-diagonal blocks; the diagonal blocks
    are I + H M^T and I + H^T M (Eq. (5) with the product written out; the paper prints I + M H^T)."""
    net = cases.small_network(14, 24, seed=5)
    G = oracle.assemble_G(net)
    for split in (5, 7, 9):
        parent, leaf = _two_leaf_tree(14, split)
        Gt = oracle.paper_inverse(G, parent, leaf)
        P = G @ Gt
        H = G[:split, split:]
        M = Gt[:split, split:]
        assert np.abs(P[:split, split:]).max() <= 1e-13
        assert np.abs(P[split:, :split]).max() <= 1e-13
        assert np.abs(P[:split, :split] - (np.eye(split) + H @ M.T)).max() <= 1e-13
        assert np.abs(P[split:, split:] - (np.eye(14 - split) + H.T @ M)).max() <= 1e-13
        assert np.abs(P - np.eye(14)).max() > 1e-6          # not the exact inverse
        # the diagonal blocks are the leaves' exact inverses (Eq. (4))
        assert _relerr(Gt[:split, :split], np.linalg.inv(G[:split, :split])) <= 1e-13


def test_paper_inverse_exact_special_cases():
    net = cases.small_network(12, 18, seed=2)
    G = oracle.assemble_G(net)
    # one leaf: direct inversion
    Gt = oracle.paper_inverse(G, np.array([-1]), np.zeros(12, np.int32))
    assert _relerr(Gt, np.linalg.inv(G)) <= 1e-13
    # uncoupled children: block-diagonal G is inverted exactly
    Gb = G.copy()
    Gb[:6, 6:] = 0.0
    Gb[6:, :6] = 0.0
    parent, leaf = _two_leaf_tree(12, 6)
    assert _relerr(oracle.paper_inverse(Gb, parent, leaf), np.linalg.inv(Gb)) <= 1e-13


def test_paper_inverse_recursion_uses_the_childrens_approximations():
    """Algorithm 1: a node's diagonal blocks are its children's *approximate* inverses, built the same
    way on the child's own subtree; brute force on a three-level binary tree."""
    net = cases.small_network(16, 30, seed=7)
    G = oracle.assemble_G(net)
    parent, leaf = cases.threshold_tree(net.pos, 4)
    Gt = oracle.paper_inverse(G, parent, leaf)
    kids = [t for t, p in enumerate(parent) if p == 0]
    assert len(kids) == 2
    for c in kids:
        sub = [t for t in range(len(parent)) if _under(parent, t, c)]
        idx = {t: k for k, t in enumerate(sub)}
        sp = np.array([-1 if t == c else idx[parent[t]] for t in sub], np.int32)
        buses = np.nonzero(np.isin(leaf, sub))[0]
        sl = np.array([idx[leaf[a]] for a in buses], np.int32)
        Gc = oracle.paper_inverse(G[np.ix_(buses, buses)], sp, sl)
        assert _relerr(Gt[np.ix_(buses, buses)], Gc) <= 1e-15
        # and that child's approximation differs from its exact inverse (it has a cut of its own)
        assert _relerr(Gc, np.linalg.inv(G[np.ix_(buses, buses)])) > 1e-9


def _relerr(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def _under(parent, t, c):
    while t >= 0:
        if t == c:
            return True
        t = parent[t]
    return False


def test_paper_inverse_error_falls_with_the_leaf_size():
    """Section V.A, Fig. 5: the error of G~^{-1} falls as the leaf threshold grows, and vanishes once
    one leaf holds the network (trend only; the paper's values are for data not available here)."""
    net = cases.net_179()
    G = oracle.assemble_G(net)
    Gi = np.linalg.inv(G)
    errs = []
    for d_th in (4, 16, 64, 179):
        parent, leaf = cases.threshold_tree(net.pos, d_th)
        Gt = oracle.paper_inverse(G, parent, leaf)
        errs.append(np.linalg.norm(Gt - Gi) / np.linalg.norm(Gi))
    assert errs[0] > errs[1] > errs[2] and errs[3] <= 1e-13


# ---------------------------------------------------------------------------
# Three-phase G (Section III.A)

def test_G3_without_mutual_coupling_is_three_copies_of_G():
    net = cases.small_network(9, 14, seed=3)
    G = oracle.assemble_G(net)
    G3 = oracle.assemble_G3(net, 0.0)
    assert _relerr(G3, np.kron(G, np.eye(3))) <= 1e-15


def test_G3_structure():
    net = cases.net_179()
    G3 = oracle.assemble_G3(net, cases.MUTUAL_RATIO)
    assert np.abs(G3 - G3.T).max() <= 1e-15 * np.abs(G3).max()        # symmetric up to the 3x3 inverses' rounding
    shunt = np.repeat(2.0 * net.C / net.dt, 3)
    assert np.abs(G3.sum(1) - shunt).max() <= 1e-12 * np.abs(G3).max()
    np.linalg.cholesky(G3)
    assert (np.abs(G3[0::3, 1::3]) > 0).any()            # phases are coupled


def test_G3_two_bus_line_sequence_eigenvalues():
    """One line between two buses with equal shunts: the eigenvalues of G3 are the shunt conductance
    (three common modes) and gC + 2/(R + (2L/dt)(1 + 2mu)) (zero sequence), gC + 2/(R + (2L/dt)(1 - mu))
    (twice: positive and negative sequence)."""
    R, L, C, dt, mu = 0.8, 2e-3, 3e-6, 5e-5, 0.3
    net = cases.Network(name="2-bus line", n_bus=2, frm=np.array([0], np.int32), to=np.array([1], np.int32),
                        R=np.array([R]), L=np.array([L]), C=np.array([C, C]), src_bus=np.zeros(0, np.int32),
                        src_amp=np.zeros(0), src_phase=np.zeros(0), parent=np.array([-1], np.int32),
                        bus_leaf=np.zeros(2, np.int32), dt=dt)
    gc, zl = 2.0 * C / dt, 2.0 * L / dt
    ref = np.sort([gc] * 3 + [gc + 2.0 / (R + zl * (1 + 2 * mu))] + [gc + 2.0 / (R + zl * (1 - mu))] * 2)
    ev = np.sort(np.linalg.eigvalsh(oracle.assemble_G3(net, mu)))
    assert np.abs(ev - ref).max() <= 1e-12 * ref.max()


# --------------------------------------------------------------------------
# Three-phase time loop (3x3 line companions, Section III.A's three rows per bus)
# --------------------------------------------------------------------------

def _shifted(net, **kw):
    import dataclasses
    return dataclasses.replace(net, **kw)


def test_three_phase_without_mutual_is_three_single_phase_runs():
    """mutual = 0: phase p is the single-phase network driven by the sources shifted by shift[p]; the
    lost line is lost in every phase."""
    net = cases.small_network(8, 12, seed=5)
    V3, _ = oracle.emt_run3(net, 300, 0.0, loss_steps=[137], loss_branches=[4])
    for p in range(3):
        net_p = _shifted(net, src_phase=net.src_phase + oracle.BALANCED[p])
        V1, _ = oracle.emt_run(net_p, 300, loss_steps=[137], loss_branches=[4], solver="lu")
        assert np.abs(V3[:, p::3] - V1).max() <= 1e-11 * np.abs(V1).max()


@pytest.mark.parametrize("n_bus,n_branch,loss", [(2, 1, None), (7, 10, (120, 3))])
def test_three_phase_sequence_decoupling(n_bus, n_branch, loss):
    """Lines with mutual inductance mu L between phases: a zero-sequence drive (equal currents in the
    three phases) sees the inductance L (1 + 2 mu) in every phase, a positive- or negative-sequence drive
    (currents summing to zero) sees L (1 - mu).  Each is a single-phase run with that inductance; on the
    two-bus line and on a meshed network with a line lost mid-run."""
    mu = 0.3
    if n_bus == 2:
        net = _net_from(2, [0], [1], [0.7], [2e-3], [3e-6, 5e-6], [0], [1.3], [0.4], 5e-5)
    else:
        net = cases.small_network(n_bus, n_branch, seed=11)
    kw = dict(loss_steps=[loss[0]], loss_branches=[loss[1]]) if loss else {}
    zero = (0.0, 0.0, 0.0)
    negative = (0.0, 2.0 * np.pi / 3.0, -2.0 * np.pi / 3.0)
    for shift, ratio in ((zero, 1 + 2 * mu), (oracle.BALANCED, 1 - mu), (negative, 1 - mu)):
        V3, _ = oracle.emt_run3(net, 400, mu, shift=shift, **kw)
        for p in range(3):
            net_p = _shifted(net, L=net.L * ratio, src_phase=net.src_phase + shift[p])
            V1, _ = oracle.emt_run(net_p, 400, solver="lu", **kw)
            assert np.abs(V3[:, p::3] - V1).max() <= 1e-11 * np.abs(V1).max(), (shift, p)
    # and the modes really differ (the check is not vacuous)
    Vz, _ = oracle.emt_run3(net, 400, mu, shift=zero, **kw)
    Vz0, _ = oracle.emt_run3(net, 400, 0.0, shift=zero, **kw)
    assert np.abs(Vz - Vz0).max() > 1e-3 * np.abs(Vz0).max()


def test_three_phase_charge_balance_across_loss():
    """Summing KCL over all buses, phase by phase (lines only move charge between buses):
    (2/dt) sum_a C_a (v_ap^n - v_ap^{n-1}) = sum_a (i_in,ap^n + i_in,ap^{n-1}), across a line loss."""
    net = cases.net_ring_fine(1, 1)
    n_steps = 300
    V, _ = oracle.emt_run3(net, n_steps, cases.MUTUAL_RATIO, loss_steps=[120], loss_branches=[40], solver="inv")
    Vp = np.vstack([np.zeros(3 * net.n_bus), V])
    t = np.arange(0, n_steps + 1) * net.dt
    u = np.array([oracle.source_current3(net, tt).sum(0) for tt in t])       # (steps + 1, 3)
    for p in range(3):
        d = (Vp[1:, p::3] - Vp[:-1, p::3]) * net.C
        lhs = (2 / net.dt) * d.sum(1)
        rhs = u[1:, p] + u[:-1, p]
        scale = (2 / net.dt) * np.abs(d).sum(1).max() + np.abs(rhs).max()
        assert np.all(np.abs(lhs - rhs) <= 1e-9 * scale)


def _state_space_run3(net, mu, n_steps, shift, loss_steps=(), loss_branches=()):
    """Independent check: the trapezoidal (Tustin) rule on the state (3 n bus voltages, 3 m line
    currents): C_a dv_a/dt = u_a - sum_e A[a,e] i_e per phase; L_e di_e/dt = v_from - v_to - R_e i_e
    with the 3x3 inductance matrix L_e = L[e] ((1 - mu) I + mu J).  A lost line's currents are held at
    zero from its loss step on."""
    n, m, dt = net.n_bus, net.n_branch, net.dt
    N, M3 = 3 * n, 3 * m
    Ainc = np.zeros((N, M3))
    for e in range(m):
        for p in range(3):
            Ainc[3 * net.frm[e] + p, 3 * e + p] = 1.0
            Ainc[3 * net.to[e] + p, 3 * e + p] = -1.0
    Linv = np.zeros((M3, M3))
    J = np.ones((3, 3))
    for e in range(m):
        Linv[3 * e:3 * e + 3, 3 * e:3 * e + 3] = np.linalg.inv(net.L[e] * ((1 - mu) * np.eye(3) + mu * J))
    Rd = np.diag(np.repeat(net.R, 3))
    Cd = np.repeat(net.C, 3)
    dead_from = np.full(m, 1 << 60)
    for s, e in zip(loss_steps, loss_branches):
        dead_from[e] = s

    def jac(step):
        alive = np.repeat((dead_from > step).astype(float), 3)
        K = np.zeros((N + M3, N + M3))
        K[:N, N:] = -(Ainc * alive) / Cd[:, None]
        K[N:, :N] = (Linv @ Ainc.T) * alive[:, None]
        K[N:, N:] = -(Linv @ Rd) * alive[:, None]
        return K, alive

    def src(step):
        u = np.zeros(N + M3)
        u[:N] = oracle.source_current3(net, step * dt, shift).ravel() / Cd
        return u

    x = np.zeros(N + M3)
    out = np.zeros((n_steps, N))
    Kp, _ = jac(0)
    for step in range(1, n_steps + 1):
        K, alive = jac(step)
        rhs = x + dt / 2 * (Kp @ x + src(step - 1) + src(step))
        Mx = np.eye(N + M3) - dt / 2 * K
        dead = np.where(alive == 0)[0] + N
        Mx[dead, :] = 0.0
        Mx[dead, dead] = 1.0
        rhs[dead] = 0.0
        x = np.linalg.solve(Mx, rhs)
        out[step - 1] = x[:N]
        Kp = K
    return out


def test_three_phase_matches_state_space_trapezoid_unbalanced():
    """Unbalanced drive (phase shifts 0, -1.9, 2.6 rad, so every sequence is excited), mutual 0.3, a
    line lost at step 150: the nodal loop with 3x3 companions against the state-space Tustin rule."""
    net = cases.small_network(7, 10, seed=3)
    shift = (0.0, -1.9, 2.6)
    V, _ = oracle.emt_run3(net, 400, 0.3, loss_steps=[150], loss_branches=[2], shift=shift)
    ref = _state_space_run3(net, 0.3, 400, shift, loss_steps=[150], loss_branches=[2])
    assert np.abs(V - ref).max() <= 1e-9 * np.abs(ref).max()
    V0, _ = oracle.emt_run3(net, 400, 0.3, shift=shift)
    assert np.abs(V0 - ref).max() > 1e-3 * np.abs(ref).max()


def test_three_phase_kcl_residual_every_step():
    net = cases.small_network(9, 14, seed=7)
    V, B = oracle.emt_run3(net, 200, 0.3, loss_steps=[80], loss_branches=[5], record_b=True)
    for lo, hi, alive in ((0, 79, None), (79, 200, np.arange(net.n_branch) != 5)):
        G3 = oracle.assemble_G3(net, 0.3, alive)
        r = B[lo:hi] - V[lo:hi] @ G3.T
        assert np.abs(r).max() <= 1e-9 * np.abs(G3).max() * np.abs(V).max()


# --------------------------------------------------------------------------
# Faults switched in the time loop: memoryless conductances (Section IV.A's
# fault-on stage, the Section V.C scenario)
# --------------------------------------------------------------------------

def _with_resistor(net, a, b, r):
    """The network plus one branch of resistance r and no inductance between buses a and b."""
    import dataclasses
    return dataclasses.replace(net, frm=np.append(net.frm, a).astype(np.int32),
                               to=np.append(net.to, b).astype(np.int32),
                               R=np.append(net.R, r), L=np.append(net.L, 0.0))


def test_fault_on_equals_a_pure_resistance_branch():
    """A branch with L = 0 is a resistor (its trapezoidal history stays zero), so a fault of 10 ohm
    switched on at step 1 is the network with that branch."""
    net = cases.case_c1(n_steps=300).net
    a, b, rf = 7, 150, 10.0
    Vf, _ = oracle.emt_run(net, 300, changes=[(1, a, b, 1.0 / rf)])
    Vr, _ = oracle.emt_run(_with_resistor(net, a, b, rf), 300)
    V0, _ = oracle.emt_run(net, 300)
    peak = np.abs(Vr).max()
    assert np.abs(Vf - Vr).max() <= 1e-12 * peak
    assert np.abs(Vf - V0).max() > 1e-3 * peak          # the fault matters


def test_fault_off_equals_losing_that_branch():
    net = cases.case_c1(n_steps=300).net
    a, b, rf, off = 12, 40, 10.0, 170
    Vf, _ = oracle.emt_run(net, 300, changes=[(1, a, b, 1.0 / rf), (off, a, b, -1.0 / rf)])
    Vr, _ = oracle.emt_run(_with_resistor(net, a, b, rf), 300, loss_steps=[off], loss_branches=[net.n_branch])
    assert np.abs(Vf - Vr).max() <= 1e-12 * np.abs(Vr).max()


def test_ground_fault_charge_balance():
    """Summing KCL over all buses with a ground fault of conductance g_f at bus a, on for steps
    [s1, s2): (2/dt) sum C (v^n - v^{n-1}) = sum (i_in^n + i_in^{n-1}) - (i_f^n + i_f^{n-1}),
    i_f^n = g_f v_a^n while on and 0 otherwise.  Holds only if the fault enters G as g_f e_a e_a^T
    with no history current, including across both switching steps."""
    net = cases.case_c1(n_steps=400).net
    a, gf, s1, s2 = 33, 0.1, 120, 260
    V, _ = oracle.emt_run(net, 400, changes=[(s1, a, -1, gf), (s2, a, -1, -gf)])
    V0, _ = oracle.emt_run(net, 400)
    assert np.array_equal(V[:s1 - 1], V0[:s1 - 1])          # steps before the fault
    Vp = np.vstack([np.zeros(net.n_bus), V])
    steps = np.arange(0, 401)
    i_f = np.where((steps >= s1) & (steps < s2), gf * Vp[:, a], 0.0)
    lhs = (2 / net.dt) * ((Vp[1:] - Vp[:-1]) * net.C).sum(1)
    u = np.array([oracle.source_current(net, n * net.dt).sum() for n in steps])
    rhs = u[1:] + u[:-1] - (i_f[1:] + i_f[:-1])
    scale = (2 / net.dt) * (np.abs(Vp[1:] - Vp[:-1]) * net.C).sum(1) + np.abs(u[1:]) + np.abs(u[:-1])
    assert np.all(np.abs(lhs - rhs) <= 1e-9 * scale.max())
    assert np.abs(V[s1:s2, a]).max() < 0.5 * np.abs(V0[s1:s2, a]).max()


def test_bolted_ground_fault_holds_the_bus_at_zero():
    """As the fault conductance grows, v_a at the fault-on steps falls like 1/g_f."""
    net = cases.case_c1(n_steps=200).net
    a, s1 = 90, 60
    va = [np.abs(oracle.emt_run(net, 200, changes=[(s1, a, -1, gf)])[0][s1 - 1:, a]).max() for gf in (1e4, 1e7)]
    ratio = va[0] / va[1]
    assert 5e2 < ratio < 2e3
