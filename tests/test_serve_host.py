"""Serving admission on the host (no GPU): the workspace size is queried before a case is built, a case
that waits for memory is never built while it waits, and a case larger than the whole budget is refused.

The pool is a stand-in that records what the serving loop asks of it; the sizes come from the library's
host-only query (emt_workspace_size), so the budget arithmetic is the real one.
"""
import os

import pytest

from paper_2105_10661_amd import cases, serve


@pytest.fixture(scope="module")
def hv():
    from paper_2105_10661_amd import hinv
    if not os.path.exists(hinv.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    hinv.load()
    return hinv


class _Handle:
    def __init__(self, pool, nbytes):
        self.pool, self.ws_bytes, self.closed = pool, nbytes, False

    def close(self):
        self.closed = True
        self.pool.live -= 1


class _Pool:
    """Records calls; a tick advances nothing on a device."""

    def __init__(self, hv):
        self.hv = hv
        self.created, self.queried, self.live, self.max_live = [], [], 0, 0
        self.next_id = 0

    def case_bytes(self, net, losses=None, max_mod_rank=2):
        self.queried.append(net.n_bus)
        return self.hv.emt_workspace_bytes(net, 1, [losses or []], prec="fp32", rel_tol=1e-9, max_refine=2,
                                           max_mod_rank=max_mod_rank, warm_start=True)

    def new_case(self, net, losses=None, max_mod_rank=2):
        nb = self.case_bytes(net, losses, max_mod_rank)
        self.queried.pop()
        self.created.append(net.n_bus)
        self.live += 1
        self.max_live = max(self.max_live, self.live)
        return _Handle(self, nb)

    def attach(self, emt, record_steps=0):
        self.next_id += 1
        return self.next_id, None

    def detach(self, sid):
        pass

    def step(self, k):
        pass

    def synchronize(self):
        pass

    def close(self):
        pass


def _arrivals(sizes, steps=200):
    out = []
    for k, s in enumerate(sizes):
        net = cases.serve_network(s, seed=100 + k)
        out.append(cases.Arrival(t=0.0, case=cases.Case(net, steps), seed=100 + k))
    return out


def test_held_case_is_not_built_while_it_waits(hv):
    arr = _arrivals([1432, 1432, 1432])
    pool = _Pool(hv)
    one = pool.case_bytes(arr[0].case.net, [])
    pool.queried.clear()
    # room for one case at a time: the second and third wait for the first to finish
    res = serve.run_serving(arr, budget_bytes=int(one * 1.5), tick_steps=100, time_scale=0, pool=pool)
    assert res.completed == 3 and res.refused == []
    assert res.created == 3 and len(pool.created) == 3      # one build per case, none while waiting
    assert pool.max_live == 1                              # never two cases in the budget at once
    assert res.max_active == 1
    assert len(pool.queried) == 3                          # one size query per case, cached while it waits


def test_case_larger_than_budget_is_refused(hv):
    arr = _arrivals([179, 5728, 179])
    pool = _Pool(hv)
    small = pool.case_bytes(arr[0].case.net, [])
    big = pool.case_bytes(arr[1].case.net, [])
    assert big > 4 * small
    res = serve.run_serving(arr, budget_bytes=2 * small + 1, tick_steps=100, time_scale=0, pool=pool)
    assert res.refused == [1]
    assert res.completed == 2 and pool.created == [179, 179]
    assert res.max_active == 2
