"""Bounds checks of the cooperative engines' tables, on the CPU.

Every index that a team, panel or level workgroup uses to address its LDS regions, its register
item ranges or a global table is checked on the host against the size the kernel and its LDS layout
assume, each time a plan is built (emt_workspace_size, emt_create, and the rebuilds after a line
loss or a change of G).  A violation is reported as HINV_E_DEVICE ("... tables: ...") instead of
reaching a kernel.  These plans are built by the host-only emt_workspace_size, so this file drives
them over many networks, trees, case counts, loss sets and precisions: each call is accepted or
refused by an engine limit (HINV_E_INVALID), and none may fail the check.
"""
import os

import numpy as np
import pytest

from paper_2105_10661_amd import cases


@pytest.fixture(scope="module")
def hv():
    from paper_2105_10661_amd import hinv
    if not os.path.exists(hinv.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    hinv.load()
    return hinv


def _networks():
    out = {"179 (4 leaves)": cases.net_179(), "716 ring": cases.net_ring(4, 7),
           "1432 ring": cases.net_ring(8, 4), "1432 ring, 4 leaves per copy": cases.net_ring(8, 5, copy_levels=2),
           "358 ring, 8 leaves per copy": cases.net_ring_fine(2, 6), "5728 torus": cases.net_torus(4, 8, 8)}
    base = cases.net_179(3)
    for d_th in (12, 30, 60, 90):
        parent, leaf = cases.threshold_tree(base.pos, d_th)
        net = cases.net_179(3)
        net.parent, net.bus_leaf = parent, leaf
        out[f"179, d_th {d_th}"] = net
    return out


def _losses(net, n_cases, rank, seed):
    """Per case up to `rank` losses at random steps; the first cases lose lines between leaves."""
    rng = np.random.default_rng(seed)
    cut = np.nonzero(net.bus_leaf[net.frm] != net.bus_leaf[net.to])[0]
    out = []
    for k in range(n_cases):
        m = int(rng.integers(0, rank + 1))
        pool = cut if k < 3 and len(cut) else np.arange(net.n_branch)
        br = rng.choice(pool, min(m, len(pool)), replace=False)
        out.append([(int(rng.integers(1, 500)), int(b)) for b in br])
    return out


def _size(hv, net, n_cases, losses, prec, warm, rank, mode):
    try:
        return hv.emt_workspace_bytes(net, n_cases, losses=losses, prec=prec, max_refine=2, max_mod_rank=rank,
                                      warm_start=warm, kernel_mode=mode)
    except hv.HinvError as e:
        assert e.name == "INVALID", (mode, str(e))      # an engine limit, never a failed table check
        return None


@pytest.mark.parametrize("name", list(_networks()))
def test_plans_pass_the_table_checks(hv, name):
    net = _networks()[name]
    ok = {}
    for seed, rank in ((1, 1), (2, 2)):
        for prec, warm in (("fp64", False), ("fp64", True), ("fp32", True)):
            for n_cases, modes in ((1, ("team", "level", "auto")), (17, ("panel", "auto")), (64, ("panel",))):
                losses = _losses(net, n_cases, rank, seed + n_cases)
                for mode in modes:
                    nb = _size(hv, net, n_cases, losses, prec, warm, rank, mode)
                    ok[mode] = ok.get(mode, 0) + (nb is not None)
    print(f"[tables] {name}: accepted {ok}")
    assert ok["auto"] > 0


def test_every_engine_is_checked_somewhere(hv):
    """The configurations above reach every cooperative engine's plan (so every checker ran)."""
    net = cases.net_ring(8, 4)
    for n_cases, mode in ((1, "team"), (1, "level"), (17, "panel")):
        assert _size(hv, net, n_cases, _losses(net, n_cases, 2, 9), "fp64", False, 2, mode) is not None, mode
