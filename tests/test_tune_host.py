"""Host logic of the autotuner: candidate enumeration, the selection rule, the feasibility check
(emt_workspace_size runs host code only) and the JSON cache.  No kernel runs here."""
import os

import numpy as np
import pytest

from paper_2105_10661_amd import cases


@pytest.fixture(scope="module")
def tn():
    from paper_2105_10661_amd import hinv, tune
    if not os.path.exists(hinv.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    hinv.load()
    return tune


def _row(tune, label, us, err, status="ok", feasible=True):
    t, e, p = label.split("/")
    c = tune.Candidate(t, e, p, 0 if p == "fp64" else 2, p != "fp64")
    return tune.Row(c, feasible, us_per_step=us, err=err, status=status)


def test_enumeration_covers_the_product(tn):
    c = tn.enumerate_candidates(["a", "b"], ["panel", "fused"], tn.DEFAULT_PATHS)
    assert len(c) == 2 * 2 * len(tn.DEFAULT_PATHS)
    assert len(set(c)) == len(c)
    assert {x.tree for x in c} == {"a", "b"} and {x.engine for x in c} == {"panel", "fused"}


def test_select_takes_the_fastest_candidate_within_the_gate(tn):
    rows = [_row(tn, "a/panel/fp64", 20.0, 1e-13),
            _row(tn, "a/panel/fp32", 10.0, 5e-10),                 # faster but misses the gate
            _row(tn, "a/fused/fp64", 15.0, 1e-13, feasible=False),  # refused by the library
            _row(tn, "b/panel/fp64", 18.0, 2e-13),
            _row(tn, "b/fused/fp64", 12.0, 1e-13, status="DEVICE"),  # device error
            _row(tn, "b/fused/fp32", 19.0, 3e-11, status="NO_CONVERGENCE")]
    ch = tn.select(rows, 1e-10)
    assert ch == rows[3].cand
    assert tn.select(rows, 1e-9) == rows[1].cand
    assert tn.select(rows[:1] + rows[2:3], 1e-20) is None
    # ties go to the earlier candidate
    tie = [_row(tn, "a/panel/fp64", 5.0, 0.0), _row(tn, "b/panel/fp64", 5.0, 0.0)]
    assert tn.select(tie, 1e-10) == tie[0].cand


def test_nan_error_is_never_selected(tn):
    rows = [_row(tn, "a/panel/fp32", 1.0, float("nan")), _row(tn, "a/panel/fp64", 9.0, 0.0)]
    assert tn.select(rows, 1e-10) == rows[1].cand


def test_feasibility_follows_the_engine_limits(tn):
    # whole 179-bus copies as leaves exceed every fused engine's leaf limit; halves fit the panel
    big = cases.tiled_network("ring", 1, 4, 9, copy_levels=0)
    half = cases.tiled_network("ring", 1, 4, 9, copy_levels=1)
    losses = [[(5, k)] for k in range(32)]
    c = tn.Candidate("t", "panel", "fp32", 2, True)
    r = tn.check_feasible(big, c, 32, losses, 1, 1e-9)
    assert not r.feasible and "179" in r.reason
    r = tn.check_feasible(half, c, 32, losses, 1, 1e-9)
    assert r.feasible and r.workspace_mb > 0


def test_tree_swap_keeps_the_network(tn):
    a = cases.tiled_network("ring", 1, 4, 9, copy_levels=1)
    b = cases.tiled_network("ring", 1, 4, 9, copy_levels=2)
    for k in ("frm", "to", "R", "L", "C", "src_bus", "src_amp", "src_phase"):
        assert np.array_equal(getattr(a, k), getattr(b, k))
    s = tn.with_tree(a, b.parent, b.bus_leaf)
    assert s.n_leaves() == b.n_leaves() == 2 * a.n_leaves()
    assert a.n_leaves() == 8          # the original is untouched


def test_cache_round_trip_and_key(tn, tmp_path):
    from paper_2105_10661_amd import hinv
    net = cases.tiled_network("ring", 1, 2, 9, copy_levels=1)
    trees = {"t": (net.parent, net.bus_leaf)}
    k1 = tn.cache_key(net, trees, [[(5, 1)]], 1, ["team"], tn.DEFAULT_PATHS, 1e-10, "dev", hinv.LIB_PATH)
    k2 = tn.cache_key(net, trees, [[(5, 2)]], 1, ["team"], tn.DEFAULT_PATHS, 1e-10, "dev", hinv.LIB_PATH)
    k3 = tn.cache_key(net, trees, [[(5, 1)]], 1, ["team"], tn.DEFAULT_PATHS, 1e-10, "dev2", hinv.LIB_PATH)
    assert len({k1, k2, k3}) == 3
    assert k1 == tn.cache_key(net, trees, [[(5, 1)]], 1, ["team"], tn.DEFAULT_PATHS, 1e-10, "dev", hinv.LIB_PATH)
    rows = [_row(tn, "t/team/fp64", 7.0, 1e-13), _row(tn, "t/level/fp64", 14.0, 1e-13),
            _row(tn, "t/panel/fp64", float("inf"), float("inf"), feasible=False)]
    res = tn.TuneResult(k1, tn.select(rows, 1e-10), rows)
    path = str(tmp_path / "sub" / "tune.json")
    tn.save_cache(path, k1, res)
    back = tn.from_cache(path, k1)
    assert back.cached and back.choice == rows[0].cand
    assert [r.cand for r in back.rows] == [r.cand for r in rows]
    assert back.rows[2].us_per_step == float("inf") and back.best().us_per_step == 7.0
    assert tn.from_cache(path, k2) is None
    tn.save_cache(path, k2, tn.TuneResult(k2, None, []))
    assert tn.from_cache(path, k1).choice == rows[0].cand and tn.from_cache(path, k2).choice is None


def test_cache_write_failure_is_not_fatal(tn, tmp_path):
    ro = tmp_path / "ro"
    ro.mkdir()
    blocker = ro / "file"
    blocker.write_text("x")
    # a path below a regular file cannot be created
    assert tn.save_cache(str(blocker / "sub" / "tune.json"), "k", tn.TuneResult("k", None, [])) is False
    assert tn.from_cache(str(blocker / "sub" / "tune.json"), "k") is None
