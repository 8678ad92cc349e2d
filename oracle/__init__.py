"""FP64 CPU oracle for the EMT network solution — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never calls it and the
two share no code; only the seeded input generator feeds both.

What is computed, and where the paper defines it:

* ``assemble_G``: the nodal conductance matrix G of the network (Section II,
  Eq. (1)), with trapezoidal companion models: a series R-L branch is the
  conductance g = 1/(R + 2L/dt) between its buses, a shunt capacitor C the
  conductance 2C/dt to ground (the paper only says "discretized by numerical
  integration"; trapezoidal is the EMTP standard it cites).
* ``solve`` / ``inverse``: v = G^{-1} i (Eq. (2)) by LU with partial pivoting
  (the LU-based solver of the paper's Introduction and Section V.C) and by an
  explicit inverse built from G X = I.  ``sparse_solver`` is a library sparse
  direct solve (SuperLU) used where the dense inverse does not fit.
* ``assemble_G3``: the three-phase G (each bus three rows, Section III.A)
  with the mutual inductance of a line between its phases; ``emt_run3`` the
  time loop of Eq. (1) on it, with 3x3 line companions.
* ``paper_inverse``: the paper's approximate hierarchical inverse G~^{-1}
  (Section III.A-B, Eq. (3)-(8), Algorithm 1): leaves inverted directly, every
  internal node's diagonal blocks are its children's approximate inverses and
  its off-diagonal blocks M = -G~_i^{-1} H_ij G~_j^{-1} (Eq. (8)).  A node with
  more than two children takes Eq. (8) for every pair of children (for the
  binary trees of the paper's Section III.B this is Algorithm 1 as printed).
* ``emt_run``: the time loop of Eq. (1): at step n, G_n v_n = i_in(t_n) + i_his
  with the history currents of the trapezoidal companions.  A lost line is
  handled by full re-assembly and re-factorisation of G (the paper's
  Section IV problem, solved here the plain way).

Readings where the paper is silent (listed in the design notes as well):
  - companion models: trapezoidal, history recursions below;
  - start: v = 0, branch currents 0, capacitor currents consistent with KCL at
    t = 0, i.e. the shunt history at step 1 is -i_in(0);
  - a branch lost at step s carries no current from step s on: it is absent
    from G_s and its history is zero; capacitor histories are untouched;
  - sources are amp*sin(2*pi*f*t + phase), t_n = n*dt;
  - three-phase networks: every line has the same ratio of mutual to self
    inductance between its phases (a transposed line), shunts are per phase
    to ground, a source drives phase p of its bus with its phase plus
    shift[p] (balanced by default: 0, -120, +120 degrees), and a lost line
    loses all three phases.

Parity unpinned: nothing here.  Every function is pinned by the
``tests/test_oracle_*.py`` checks against closed forms, an independent
state-space formulation, conservation identities and library routines.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "emt_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C part of the oracle (gcc, OpenMP) next to its source."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.orc_assemble.argtypes = [ctypes.c_int, ctypes.c_int, ip, ip, dp, dp, dp, ctypes.c_double,
                                     ctypes.c_void_p, dp]
        lib.orc_lu_factor.argtypes = [ctypes.c_int, dp, ip]
        lib.orc_lu_solve.argtypes = [ctypes.c_int, dp, ip, dp]
        lib.orc_solve.argtypes = [ctypes.c_int, dp, dp, dp]
        lib.orc_solve_many.argtypes = [ctypes.c_int, dp, ctypes.c_int, dp, dp]
        lib.orc_inverse.argtypes = [ctypes.c_int, dp, dp]
        lib.orc_matvec.argtypes = [ctypes.c_int, dp, dp, dp]
        lib.orc_lu_solve.restype = None
        lib.orc_matvec.restype = None
        _lib = lib
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# ---------------------------------------------------------------------------
# Network equation (Section II, Eq. (1)-(2))
# ---------------------------------------------------------------------------

def branch_conductance(net) -> np.ndarray:
    """g = 1 / (R + 2L/dt): trapezoidal companion of a series R-L branch."""
    return 1.0 / (net.R + 2.0 * net.L / net.dt)


def assemble_G(net, alive: Optional[np.ndarray] = None) -> np.ndarray:
    """Dense nodal conductance matrix G (n x n, FP64)."""
    n = net.n_bus
    G = np.empty((n, n), np.float64)
    fr, to = _c(net.frm, np.int32), _c(net.to, np.int32)
    R, L, C = _c(net.R, np.float64), _c(net.L, np.float64), _c(net.C, np.float64)
    al = None if alive is None else _c(alive, np.uint8)
    st = _load().orc_assemble(n, net.n_branch, _ip(fr), _ip(to), _dp(R), _dp(L), _dp(C), net.dt,
                              None if al is None else al.ctypes.data_as(ctypes.c_void_p), _dp(G))
    if st != 0:
        raise ValueError("branch with invalid bus index")
    return G


def solve(G: np.ndarray, b: np.ndarray) -> np.ndarray:
    """x with G x = b, by LU with partial pivoting (b: one vector or rows of vectors)."""
    G = _c(G, np.float64)
    n = G.shape[0]
    b = _c(b, np.float64)
    if b.ndim == 1:
        x = np.empty(n, np.float64)
        st = _load().orc_solve(n, _dp(G), _dp(b), _dp(x))
    else:
        x = np.empty_like(b)
        st = _load().orc_solve_many(n, _dp(G), b.shape[0], _dp(b), _dp(x))
    if st != 0:
        raise np.linalg.LinAlgError(f"singular matrix (status {st})")
    return x


def inverse(G: np.ndarray) -> np.ndarray:
    """Explicit G^{-1}: column j solves G x = e_j."""
    G = _c(G, np.float64)
    n = G.shape[0]
    X = np.empty((n, n), np.float64)
    st = _load().orc_inverse(n, _dp(G), _dp(X))
    if st != 0:
        raise np.linalg.LinAlgError(f"singular matrix (status {st})")
    return X


def matvec(M: np.ndarray, x: np.ndarray) -> np.ndarray:
    M = _c(M, np.float64)
    x = _c(x, np.float64)
    y = np.empty(M.shape[0], np.float64)
    _load().orc_matvec(M.shape[0], _dp(M), _dp(x), _dp(y))
    return y


class _LU:
    def __init__(self, G):
        self.n = G.shape[0]
        self.A = _c(G, np.float64).copy()
        self.piv = np.empty(self.n, np.int32)
        st = _load().orc_lu_factor(self.n, _dp(self.A), _ip(self.piv))
        if st != 0:
            raise np.linalg.LinAlgError(f"singular matrix (status {st})")

    def __call__(self, b):
        x = _c(b, np.float64).copy()
        _load().orc_lu_solve(self.n, _dp(self.A), _ip(self.piv), _dp(x))
        return x


def line_matrices3(net, mutual: float):
    """Per line e, the 3x3 series impedance of its trapezoidal companion and what follows from it.

    Line e is a three-phase series R-L: resistance R[e] per phase, self inductance L[e] and mutual
    inductance mutual * L[e] between any two phases, L_e = L[e] ((1 - mutual) I + mutual J), J the
    all-ones matrix.  The trapezoidal rule applied to R i + L_e di/dt = v over one step gives
    (R I + (2/dt) L_e) i^n = v^n + v^{n-1} + ((2/dt) L_e - R I) i^{n-1}, so with
    Y_e = (R I + (2/dt) L_e)^{-1} (a library 3x3 inverse) and A_e = Y_e ((2/dt) L_e - R I):
    i^n = Y_e v^n + h^n and h^{n+1} = Y_e v^n + A_e i^n.  Returns (Y, A), each (n_branch, 3, 3).
    """
    J = np.ones((3, 3))
    Y = np.empty((net.n_branch, 3, 3))
    A = np.empty((net.n_branch, 3, 3))
    for e in range(net.n_branch):
        Le = net.L[e] * ((1.0 - mutual) * np.eye(3) + mutual * J)
        Y[e] = inverse(net.R[e] * np.eye(3) + (2.0 / net.dt) * Le)
        A[e] = Y[e] @ ((2.0 / net.dt) * Le - net.R[e] * np.eye(3))
    return Y, A


def assemble_G3(net, mutual: float, alive: Optional[np.ndarray] = None) -> np.ndarray:
    """Dense three-phase nodal conductance matrix (rows 3a + p; Section III.A, each bus has three phases).

    Line e's companion admittance Y_e (``line_matrices3``) is entered as the single-phase conductance
    is: +Y_e on the two buses' diagonal blocks, -Y_e between them; a lost line (alive[e] false) enters
    nothing.  Shunt 2C/dt per phase.
    """
    n = net.n_bus
    G = np.zeros((3 * n, 3 * n))
    for a in range(n):
        G[3 * a:3 * a + 3, 3 * a:3 * a + 3] += 2.0 * net.C[a] / net.dt * np.eye(3)
    Ys, _ = line_matrices3(net, mutual)
    for e in range(net.n_branch):
        if alive is not None and not alive[e]:
            continue
        Y = Ys[e]
        a, b = int(net.frm[e]), int(net.to[e])
        G[3 * a:3 * a + 3, 3 * a:3 * a + 3] += Y
        G[3 * b:3 * b + 3, 3 * b:3 * b + 3] += Y
        G[3 * a:3 * a + 3, 3 * b:3 * b + 3] -= Y
        G[3 * b:3 * b + 3, 3 * a:3 * a + 3] -= Y
    return G


BALANCED = (0.0, -2.0 * np.pi / 3.0, 2.0 * np.pi / 3.0)


def source_current3(net, t: float, shift=BALANCED) -> np.ndarray:
    """Three-phase injections (n_bus, 3): source q drives phase p of its bus with
    amp*sin(2*pi*f*t + phase + shift[p]); the default shift is a balanced (positive-sequence) set."""
    out = np.zeros((net.n_bus, 3))
    for p in range(3):
        val = net.src_amp * np.sin(2.0 * np.pi * net.freq * t + net.src_phase + shift[p])
        out[:, p] = np.bincount(net.src_bus, weights=val, minlength=net.n_bus)
    return out


def emt_run3(net, n_steps: int, mutual: float, loss_steps: Sequence[int] = (), loss_branches: Sequence[int] = (),
             solver: str = "lu", shift=BALANCED, record_b: bool = False):
    """Node voltages of the three-phase trapezoidal EMT time loop (Eq. (1) with three rows per bus).

    Same loop as ``emt_run`` with every quantity a 3-vector per bus or line: the line companions are
    3x3 (``line_matrices3``), shunts are per phase, sources per ``source_current3``.  A line lost at
    step s loses all three phases: it is absent from G_s and its history is zero from step s on.
    Returns (V, B) with V[k] (3 n_bus,) the voltages at step k + 1 in row order 3a + p.
    solver: "lu" (dense LU each new G) or "inv" (explicit inverse times the current vector).
    """
    n, dt = net.n_bus, net.dt
    fr, to = net.frm.astype(np.int64), net.to.astype(np.int64)
    Y, A = line_matrices3(net, mutual)
    gC = (2.0 * net.C / dt)[:, None]
    dead_from = np.full(net.n_branch, np.iinfo(np.int64).max, np.int64)
    for s, e in zip(loss_steps, loss_branches):
        dead_from[int(e)] = min(dead_from[int(e)], int(s))
    V = np.zeros((n_steps, 3 * n))
    B = np.zeros((n_steps, 3 * n)) if record_b else None
    h = np.zeros((net.n_branch, 3))                   # line history currents, per phase
    hC = -source_current3(net, 0.0, shift)            # KCL-consistent start, per phase
    alive_prev, apply = None, None
    for step in range(1, n_steps + 1):
        alive = dead_from > step
        if alive_prev is None or not np.array_equal(alive, alive_prev):
            G = assemble_G3(net, mutual, alive)
            if solver == "inv":
                Ginv = inverse(G)
                apply = lambda x, M=Ginv: matvec(M, x)
            elif solver == "lu":
                apply = _LU(G)
            else:
                raise ValueError(solver)
            alive_prev = alive
        h = np.where(alive[:, None], h, 0.0)
        inj = np.zeros((n, 3))
        np.add.at(inj, fr, h)
        np.add.at(inj, to, -h)
        b = source_current3(net, step * dt, shift) - inj - hC
        v = apply(b.ravel()).reshape(n, 3)
        vft = v[fr] - v[to]
        yv = np.einsum("epq,eq->ep", Y, vft)
        i = yv + h                                     # line currents at step n
        h = np.where(alive[:, None], yv + np.einsum("epq,eq->ep", A, i), 0.0)
        iC = gC * v + hC
        hC = -gC * v - iC
        V[step - 1] = v.ravel()
        if B is not None:
            B[step - 1] = b.ravel()
    return V, B


def paper_inverse(G: np.ndarray, parent: Sequence[int], bus_leaf: Sequence[int]) -> np.ndarray:
    """The paper's approximate inverse G~^{-1} of G for a partition tree (Section III.A-B, Algorithm 1).

    parent[k]: parent of tree node k (-1 for the root); bus_leaf[a]: the leaf owning bus a.  A leaf's
    block is inverted directly; an internal node joins its children's approximate inverses as the
    diagonal blocks (Eq. (4)) and fills the block of children i, j with M_ij = -G~_i^{-1} H_ij G~_j^{-1}
    (Eq. (8)), H_ij being G's block between the two children's buses (Eq. (3)).  Returned in the
    caller's bus order.
    """
    G = _c(G, np.float64)
    n = G.shape[0]
    parent = np.asarray(parent, np.int64)
    bus_leaf = np.asarray(bus_leaf, np.int64)
    children = [[] for _ in range(len(parent))]
    root = -1
    for t, p in enumerate(parent):
        if p < 0:
            root = t
        else:
            children[p].append(t)

    def approx(t):
        if not children[t]:                                  # leaf: direct inversion
            b = np.nonzero(bus_leaf == t)[0]
            return b, inverse(G[np.ix_(b, b)])
        parts = [approx(c) for c in children[t]]
        sizes = [len(b) for b, _ in parts]
        off = np.concatenate([[0], np.cumsum(sizes)])
        buses = np.concatenate([b for b, _ in parts])
        Gt = np.zeros((len(buses), len(buses)))
        for i, (bi, Gi) in enumerate(parts):
            Gt[off[i]:off[i + 1], off[i]:off[i + 1]] = Gi                       # Eq. (4)
            for j, (bj, Gj) in enumerate(parts):
                if i != j:
                    H = G[np.ix_(bi, bj)]                                       # Eq. (3)
                    Gt[off[i]:off[i + 1], off[j]:off[j + 1]] = -(Gi @ H @ Gj)   # Eq. (8)
        return buses, Gt

    buses, Gt = approx(root)
    out = np.zeros((n, n))
    out[np.ix_(buses, buses)] = Gt
    return out


def sparse_G(net, alive: Optional[np.ndarray] = None):
    """G as a scipy CSC matrix (same definition as assemble_G)."""
    import scipy.sparse as sp
    n = net.n_bus
    g = branch_conductance(net)
    if alive is not None:
        g = np.where(alive.astype(bool), g, 0.0)
    a, b = net.frm.astype(np.int64), net.to.astype(np.int64)
    rows = np.concatenate([a, b, a, b, np.arange(n)])
    cols = np.concatenate([a, b, b, a, np.arange(n)])
    vals = np.concatenate([g, g, -g, -g, 2.0 * net.C / net.dt])
    return sp.csc_matrix((vals, (rows, cols)), shape=(n, n))


def sparse_solver(net, alive: Optional[np.ndarray] = None):
    """Library sparse direct solve (SuperLU) of G x = b, for networks too big for dense LU."""
    import scipy.sparse.linalg as spl
    return spl.splu(sparse_G(net, alive), permc_spec="MMD_AT_PLUS_A").solve


def source_current(net, t: float) -> np.ndarray:
    """i_in(t): sum of amp*sin(2*pi*f*t + phase) at each source bus."""
    val = net.src_amp * np.sin(2.0 * np.pi * net.freq * t + net.src_phase)
    return np.bincount(net.src_bus, weights=val, minlength=net.n_bus)


def emt_run(net, n_steps: int, loss_steps: Sequence[int] = (), loss_branches: Sequence[int] = (),
            solver: str = "inv", record_b: bool = False, record_steps: Optional[np.ndarray] = None,
            changes: Sequence = ()):
    """Node voltages v_1..v_N of the trapezoidal EMT time loop (Eq. (1)).

    solver: "inv" (explicit inverse times the current vector), "lu" (LU solve
    each step) or "sparse" (library sparse LU).  Returns (V, B): V[k] is the
    voltage at the k-th recorded step (steps 1..n_steps, or ``record_steps``),
    B the right-hand side i_in + i_his of the same steps (or None).

    changes: (step, a, b, dg) memoryless conductances (a fault of resistance
    1/dg between buses a and b, b = -1 for ground; a negative dg removes one)
    in force from that step on: G_on = G_pre + dg (e_a - e_b)(e_a - e_b)^T,
    the fault-on stage of Section IV.A.  A resistor has no history current, so
    the right-hand side is the same with or without it.
    """
    n, dt = net.n_bus, net.dt
    fr, to = net.frm.astype(np.int64), net.to.astype(np.int64)
    g = branch_conductance(net)
    alpha = g * (2.0 * net.L / dt - net.R)          # history weight of the branch current
    gC = 2.0 * net.C / dt
    dead_from = np.full(net.n_branch, np.iinfo(np.int64).max, np.int64)
    for s, e in zip(loss_steps, loss_branches):
        dead_from[int(e)] = min(dead_from[int(e)], int(s))
    rec = np.arange(1, n_steps + 1) if record_steps is None else np.asarray(record_steps)
    rec_pos = {int(s): k for k, s in enumerate(rec)}
    V = np.zeros((len(rec), n), np.float64)
    B = np.zeros((len(rec), n), np.float64) if record_b else None
    h = np.zeros(net.n_branch)                        # branch history currents
    hC = -source_current(net, 0.0)                    # shunt history, KCL-consistent start
    changes = [(int(s), int(a), int(b), float(d)) for s, a, b, d in changes]
    if changes and solver == "sparse":
        raise ValueError("changes need the dense solvers")
    alive_prev = None
    on_prev = None
    apply = None
    for step in range(1, n_steps + 1):
        alive = dead_from > step
        on = [k for k, c in enumerate(changes) if c[0] <= step]
        if alive_prev is None or not np.array_equal(alive, alive_prev) or on != on_prev:
            G = None if solver == "sparse" else assemble_G(net, alive)
            for k in on:
                _, a, b, dg = changes[k]
                G[a, a] += dg
                if b >= 0:
                    G[b, b] += dg
                    G[a, b] -= dg
                    G[b, a] -= dg
            if solver == "inv":
                Ginv = inverse(G)
                apply = lambda x, M=Ginv: matvec(M, x)
            elif solver == "lu":
                apply = _LU(G)
            elif solver == "sparse":
                apply = sparse_solver(net, alive)
            else:
                raise ValueError(solver)
            alive_prev, on_prev = alive, on
        h = np.where(alive, h, 0.0)
        b = source_current(net, step * dt) - (np.bincount(fr, h, n) - np.bincount(to, h, n)) - hC
        v = apply(b)
        vbr = v[fr] - v[to]
        ibr = g * vbr + h                              # branch current at step n
        h = np.where(alive, g * vbr + alpha * ibr, 0.0)
        iC = gC * v + hC                               # capacitor current at step n
        hC = -gC * v - iC
        k = rec_pos.get(step)
        if k is not None:
            V[k] = v
            if B is not None:
                B[k] = b
    return V, B
