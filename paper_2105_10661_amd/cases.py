"""Seeded synthetic EMT networks, partition trees and event schedules.

This module only draws inputs: topology, R/L/C values, sources, the partition
tree (which buses each sub-network owns) and line-loss / arrival schedules.  It
holds none of the solver's arithmetic (no conductances, no companion models,
no inverses), so both the FP64 oracle and the GPU library can be fed from it.

The paper's case studies use copies of a 179-bus system tiled into arrays
(Section V, "CPU time in terms of FLOPS").  That data set is not available,
so a geometric random graph with the same bus and branch counts stands in for
it: buses at uniform positions in the unit square, a Euclidean minimum
spanning tree, then the shortest non-tree links among each bus's six nearest
neighbours until the branch count is reached.  Copies share the topology and
draw their own R, L, C and sources; copies are joined by random tie lines on a
ring or a 2-D torus.

Random streams: one numpy PCG64 SeedSequence per purpose (topology, per-copy
parameters, sources, tie lines, events, arrivals), so that changing one part
of a configuration does not shift the draws of another.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

BASE_BUSES = 179
BASE_BRANCHES = 263
DT = 50e-6
FREQ = 60.0
TOPOLOGY_SEED = 2105_10661
R_RANGE = (0.001, 0.05)          # ohm
L_RANGE = (0.5e-3, 5e-3)         # henry
C_RANGE = (1e-9, 10e-9)          # farad, shunt to ground per bus
AMP_RANGE = (0.5, 2.0)           # ampere
SOURCES_PER_COPY = 10
TIES_PER_PAIR = 3


@dataclass
class Network:
    """One EMT network plus its partition tree.

    Branch e connects bus ``frm[e]`` to bus ``to[e]`` through a series R-L;
    every bus has a shunt capacitance ``C`` to ground; current sources
    ``amp*sin(2*pi*freq*t + phase)`` are injected at ``src_bus``.
    ``parent[k]`` is the parent of tree node k (-1 for the root); children are
    the nodes whose parent is k, in index order.  ``bus_leaf[a]`` is the leaf
    node that owns bus a.
    """
    name: str
    n_bus: int
    frm: np.ndarray
    to: np.ndarray
    R: np.ndarray
    L: np.ndarray
    C: np.ndarray
    src_bus: np.ndarray
    src_amp: np.ndarray
    src_phase: np.ndarray
    parent: np.ndarray
    bus_leaf: np.ndarray
    dt: float = DT
    freq: float = FREQ
    pos: Optional[np.ndarray] = None

    @property
    def n_branch(self) -> int:
        return int(self.frm.shape[0])

    @property
    def n_nodes(self) -> int:
        return int(self.parent.shape[0])

    def n_leaves(self) -> int:
        has_child = np.zeros(self.n_nodes, bool)
        has_child[self.parent[self.parent >= 0]] = True
        return int((~has_child).sum())


@dataclass
class Case:
    """A network, a step count and a line-loss schedule (branch lost from a step on)."""
    net: Network
    n_steps: int
    loss_steps: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    loss_branches: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))


def _streams(seed: int, n: int) -> List[np.random.Generator]:
    return [np.random.Generator(np.random.PCG64(s)) for s in np.random.SeedSequence(seed).spawn(n)]


def base_topology(seed: int = TOPOLOGY_SEED, n: int = BASE_BUSES, m: int = BASE_BRANCHES
                  ) -> Tuple[np.ndarray, np.ndarray]:
    """Positions (n,2) and branch list (m,2) of the geometric base graph."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = rng.random((n, 2))
    d = np.sqrt(((pos[:, None, :] - pos[None, :, :]) ** 2).sum(-1))
    # Prim's minimum spanning tree.
    in_tree = np.zeros(n, bool)
    in_tree[0] = True
    best = d[0].copy()
    best_from = np.zeros(n, np.int64)
    edges = []
    for _ in range(n - 1):
        cand = np.where(in_tree, np.inf, best)
        j = int(np.argmin(cand))
        edges.append((min(j, int(best_from[j])), max(j, int(best_from[j]))))
        in_tree[j] = True
        closer = d[j] < best
        best = np.where(closer, d[j], best)
        best_from = np.where(closer, j, best_from)
    have = set(edges)
    extra = set()
    order = np.argsort(d, axis=1, kind="stable")
    for i in range(n):
        for j in order[i, 1:7]:
            e = (min(i, int(j)), max(i, int(j)))
            if e not in have:
                extra.add(e)
    extra = sorted(extra, key=lambda e: (d[e[0], e[1]], e))
    edges += extra[: m - len(edges)]
    if len(edges) != m:
        raise ValueError("not enough candidate links for the requested branch count")
    return pos, np.asarray(edges, np.int32)


def _copy_split(pos: np.ndarray, levels: int) -> List[np.ndarray]:
    """Split one copy's buses by coordinate medians: x first, then y, alternating.

    Returns 2**levels groups of local bus indices, in tree order.
    """
    groups = [np.arange(pos.shape[0])]
    for lev in range(levels):
        axis = lev % 2
        nxt = []
        for g in groups:
            o = g[np.argsort(pos[g, axis], kind="stable")]
            h = (len(o) + 1) // 2
            nxt += [np.sort(o[:h]), np.sort(o[h:])]
        groups = nxt
    return groups


def _draw_rl(rng: np.random.Generator, k: int) -> Tuple[np.ndarray, np.ndarray]:
    R = rng.uniform(*R_RANGE, size=k)
    L = rng.uniform(*L_RANGE, size=k)
    return R, L


def tiled_network(name: str, rows: int, cols: int, seed: int, copy_levels: int = 1,
                  torus: bool = False) -> Network:
    """Copies of the base graph on a ring (rows == 1) or a rows x cols torus.

    The partition tree follows the tiling: each copy is split into
    2**copy_levels leaves by coordinate bisection; then copies; then (torus)
    rows of copies; then the root.  A single copy (rows == cols == 1) has the
    copy node as the root.
    """
    pos, edges = base_topology()
    n_copies = rows * cols
    s_par, s_src, s_tie = _streams(seed, 3)
    nb = BASE_BUSES
    frm, to, R, L, C = [], [], [], [], []
    sb, sa, sp = [], [], []
    for k in range(n_copies):
        Rk, Lk = _draw_rl(s_par, BASE_BRANCHES)
        Ck = s_par.uniform(*C_RANGE, size=nb)
        frm.append(edges[:, 0] + k * nb)
        to.append(edges[:, 1] + k * nb)
        R.append(Rk)
        L.append(Lk)
        C.append(Ck)
        buses = s_src.choice(nb, SOURCES_PER_COPY, replace=False)
        sb.append(np.sort(buses) + k * nb)
        sa.append(s_src.uniform(*AMP_RANGE, size=SOURCES_PER_COPY))
        sp.append(s_src.uniform(0.0, 2.0 * np.pi, size=SOURCES_PER_COPY))
    # tie lines between neighbouring copies
    pairs = []
    if n_copies > 1:
        if rows == 1:
            for j in range(cols):
                pairs.append((j, (j + 1) % cols))
        else:
            for i in range(rows):
                for j in range(cols):
                    pairs.append((i * cols + j, i * cols + (j + 1) % cols))
                    pairs.append((i * cols + j, ((i + 1) % rows) * cols + j))
        pairs = sorted(set(tuple(p) for p in pairs if p[0] != p[1]))
    used = set()
    tf, tt = [], []
    for (p, q) in pairs:
        for _ in range(TIES_PER_PAIR):
            while True:
                u = int(s_tie.integers(nb)) + p * nb
                w = int(s_tie.integers(nb)) + q * nb
                key = (min(u, w), max(u, w))
                if key not in used:
                    used.add(key)
                    break
            tf.append(u)
            tt.append(w)
    if tf:
        Rt, Lt = _draw_rl(s_tie, len(tf))
        frm.append(np.asarray(tf))
        to.append(np.asarray(tt))
        R.append(Rt)
        L.append(Lt)
    n_bus = n_copies * nb
    # partition tree
    parent: List[int] = []
    bus_leaf = np.full(n_bus, -1, np.int64)

    def add(par: int) -> int:
        parent.append(par)
        return len(parent) - 1

    groups = _copy_split(pos, copy_levels)
    root = add(-1)

    def add_copy(k: int, copy_node: int) -> None:
        # binary bisection levels under the copy node; group 2*g+h is child h of group g
        def rec(node: int, lev: int, g: int) -> None:
            if lev == copy_levels:
                bus_leaf[groups[g] + k * nb] = node
                return
            for h in range(2):
                rec(add(node), lev + 1, 2 * g + h)
        rec(copy_node, 0, 0)

    if n_copies == 1:
        add_copy(0, root)
    elif rows == 1:
        for k in range(n_copies):
            add_copy(k, add(root))
    else:
        row_nodes = [add(root) for _ in range(rows)]
        for i in range(rows):
            for j in range(cols):
                add_copy(i * cols + j, add(row_nodes[i]))
    net = Network(
        name=name, n_bus=n_bus,
        frm=np.concatenate(frm).astype(np.int32), to=np.concatenate(to).astype(np.int32),
        R=np.concatenate(R).astype(np.float64), L=np.concatenate(L).astype(np.float64),
        C=np.concatenate(C).astype(np.float64),
        src_bus=np.concatenate(sb).astype(np.int32), src_amp=np.concatenate(sa).astype(np.float64),
        src_phase=np.concatenate(sp).astype(np.float64),
        parent=np.asarray(parent, np.int32), bus_leaf=bus_leaf.astype(np.int32),
        pos=np.concatenate([pos] * n_copies),
    )
    assert (net.bus_leaf >= 0).all()
    return net


def threshold_tree(pos: np.ndarray, d_th: int) -> Tuple[np.ndarray, np.ndarray]:
    """Recursive coordinate bisection until a group has at most d_th buses.

    Returns (parent, bus_leaf).  Stands in for the unavailable partitioner of
    the paper's Section III.B; the node threshold d_th bounds the leaf size.
    """
    n = pos.shape[0]
    parent: List[int] = []
    bus_leaf = np.full(n, -1, np.int64)

    def rec(idx: np.ndarray, par: int, axis: int) -> None:
        node = len(parent)
        parent.append(par)
        if len(idx) <= d_th:
            bus_leaf[idx] = node
            return
        o = idx[np.argsort(pos[idx, axis], kind="stable")]
        h = (len(o) + 1) // 2
        rec(np.sort(o[:h]), node, 1 - axis)
        rec(np.sort(o[h:]), node, 1 - axis)

    rec(np.arange(n), -1, 0)
    return np.asarray(parent, np.int32), bus_leaf.astype(np.int32)


def small_network(n_bus: int, n_branch: int, seed: int, d_th: int = 0) -> Network:
    """A tiny connected random network (for brute-force checks), same value ranges."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = rng.random((n_bus, 2))
    edges = set()
    perm = rng.permutation(n_bus)
    for i in range(1, n_bus):       # random spanning tree
        j = int(perm[rng.integers(i)])
        a, b = int(perm[i]), j
        edges.add((min(a, b), max(a, b)))
    while len(edges) < n_branch:
        a, b = rng.integers(n_bus, size=2)
        if a != b:
            edges.add((int(min(a, b)), int(max(a, b))))
    e = np.asarray(sorted(edges), np.int32)
    R, L = _draw_rl(rng, len(e))
    C = rng.uniform(*C_RANGE, size=n_bus)
    ns = max(1, n_bus // 3)
    sb = np.sort(rng.choice(n_bus, ns, replace=False))
    if d_th <= 0:
        d_th = max(1, (n_bus + 1) // 2)
    parent, bus_leaf = threshold_tree(pos, d_th)
    return Network(name=f"small{n_bus}", n_bus=n_bus, frm=e[:, 0].copy(), to=e[:, 1].copy(),
                   R=R, L=L, C=C, src_bus=sb.astype(np.int32),
                   src_amp=rng.uniform(*AMP_RANGE, size=ns), src_phase=rng.uniform(0, 2 * np.pi, size=ns),
                   parent=parent, bus_leaf=bus_leaf, pos=pos)


# ---------------------------------------------------------------------------
# Benchmark configurations (bus counts, tilings, step counts, event schedules)
# ---------------------------------------------------------------------------

def net_179(seed: int = 1) -> Network:
    """Single 179-bus network, 4 sub-networks (two bisection levels)."""
    return tiled_network("179-bus", 1, 1, seed, copy_levels=2)


def net_ring(n_copies: int, seed: int, copy_levels: int = 1) -> Network:
    """n_copies on a ring, 3 tie lines per neighbouring pair; leaves = copy halves (2**copy_levels
    leaves per copy; the network itself does not depend on copy_levels)."""
    return tiled_network(f"{n_copies * BASE_BUSES}-bus ring", 1, n_copies, seed, copy_levels=copy_levels)


MUTUAL_RATIO = 0.3      # three-phase lines: mutual inductance between phases / self inductance


def net_ring_fine(n_copies: int, seed: int) -> Network:
    """n_copies on a ring (as net_ring) with each copy split into 8 leaves of about 22 buses, so that a
    three-phase tree (three rows per bus) stays within the leaf limit."""
    return tiled_network(f"{n_copies * BASE_BUSES}-bus ring, 8 leaves per copy", 1, n_copies, seed, copy_levels=3)


def phase_rows(bus_leaf: np.ndarray, phases: int = 3) -> np.ndarray:
    """Leaf of each row when bus a has rows phases*a .. phases*a + phases - 1."""
    return np.repeat(np.asarray(bus_leaf, np.int32), phases)


def net_torus(rows: int, cols: int, seed: int) -> Network:
    """rows x cols torus of copies; tree: halves -> copies -> rows -> root."""
    return tiled_network(f"{rows * cols * BASE_BUSES}-bus torus", rows, cols, seed, copy_levels=1, torus=True)


def case_c1(seed: int = 1, n_steps: int = 1000) -> Case:
    return Case(net_179(seed), n_steps)


def case_c2(seed: int = 2, n_steps: int = 10000, loss_step: int = 2000) -> Case:
    net = net_ring(8, seed)
    (s_ev,) = _streams(seed + 1000, 1)
    br = int(s_ev.integers(net.n_branch))
    return Case(net, n_steps, np.asarray([loss_step], np.int32), np.asarray([br], np.int32))


def case_c3(seed: int = 3, n_steps: int = 10000) -> Case:
    return Case(net_torus(8, 8, seed), n_steps)


def cases_c4(seed: int = 4, n_cases: int = 256, n_steps: int = 8000,
             step_range: Tuple[int, int] = (500, 5000)) -> Tuple[Network, List[Case]]:
    """One shared 1432-bus base network; each case loses a distinct branch at a random step."""
    net = net_ring(8, seed)
    (s_ev,) = _streams(seed + 1000, 1)
    br = s_ev.choice(net.n_branch, n_cases, replace=False)
    st = s_ev.integers(step_range[0], step_range[1] + 1, size=n_cases)
    return net, [Case(net, n_steps, np.asarray([s], np.int32), np.asarray([b], np.int32))
                 for s, b in zip(st, br)]


SERVE_SIZES = (179, 716, 1432, 5728)


def serve_network(size: int, seed: int) -> Network:
    if size == 179:
        return tiled_network("179-bus", 1, 1, seed, copy_levels=2)
    if size == 716:
        return net_ring(4, seed)
    if size == 1432:
        return net_ring(8, seed)
    if size == 5728:
        return net_torus(4, 8, seed)
    raise ValueError(size)


@dataclass
class Arrival:
    t: float          # arrival time, seconds
    case: Case
    seed: int


def serve_arrivals(seed: int = 5, n_cases: int = 64, rate: float = 200.0,
                   steps: Tuple[int, int] = (2000, 20000), sizes: Sequence[int] = SERVE_SIZES,
                   max_losses: int = 2) -> List[Arrival]:
    """Poisson arrivals of mixed-size cases, each its own seeded network instance."""
    (s_arr,) = _streams(seed, 1)
    t = 0.0
    out = []
    for k in range(n_cases):
        t += float(s_arr.exponential(1.0 / rate))
        size = int(sizes[int(s_arr.integers(len(sizes)))])
        n_steps = int(s_arr.integers(steps[0], steps[1] + 1))
        case_seed = int(s_arr.integers(1, 2 ** 31 - 1))
        net = serve_network(size, case_seed)
        n_loss = int(s_arr.integers(0, max_losses + 1))
        br = s_arr.choice(net.n_branch, n_loss, replace=False).astype(np.int32)
        st = np.sort(s_arr.integers(1, n_steps + 1, size=n_loss)).astype(np.int32)
        out.append(Arrival(t, Case(net, n_steps, st, br), case_seed))
    return out
