"""Serving: continuous batching of mixed-size EMT cases (serve_* ABI).

Each case's trajectory in the mix must equal the same case served alone,
bitwise (a case's arithmetic is independent of the other cases in a launch
and of where launches start and end); sampled cases must match the FP64 CPU
oracle within 1e-10 (peak-normalised).
"""
import numpy as np
import pytest

import oracle
from paper_2105_10661_amd import cases

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def served():
    import torch
    from paper_2105_10661_amd import serve
    torch.cuda.set_device(0)
    arr = cases.serve_arrivals(seed=5, n_cases=10, steps=(150, 400))
    print(f"[gpu] serving {len(arr)} cases, sizes {[a.case.net.n_bus for a in arr]}", flush=True)
    res = serve.run_serving(arr, budget_bytes=40 << 20, max_slots=3, tick_steps=64, record=True, time_scale=20.0)
    return arr, res


def test_all_cases_complete_with_queueing(served):
    arr, res = served
    assert res.completed == len(arr)
    assert res.max_active <= 3
    assert res.solves == sum(a.case.n_steps for a in arr)


def test_mix_equals_alone_bitwise(served):
    from paper_2105_10661_amd import serve
    arr, res = served
    for i in (0, 3, 7):
        alone = serve.run_serving([arr[i]], budget_bytes=1 << 40, max_slots=1, tick_steps=50, record=True,
                                  time_scale=0.0)
        assert np.array_equal(alone.records[0], res.records[i]), i


def test_served_cases_match_oracle(served):
    arr, res = served
    for i in range(len(arr)):
        case = arr[i].case
        solver = "sparse" if case.net.n_bus > 2000 else "inv"
        Vref, _ = oracle.emt_run(case.net, case.n_steps, loss_steps=case.loss_steps,
                                 loss_branches=case.loss_branches, solver=solver)
        err = np.abs(res.records[i] - Vref).max() / np.abs(Vref).max()
        assert err <= 1e-10, (i, case.net.n_bus, err)


def test_fp64_incremental_serving_floating_bus():
    """FP64 serving with warm_start runs the incremental form on both launch kinds: a 1432-bus case
    (one workgroup) losing a line that leaves a bus on its shunt capacitor (solved directly, such a loss
    drifts past 1e-10), and a 5728-bus torus case (level-engine team) with a loss, within 1e-10 of the
    oracle."""
    import torch
    from paper_2105_10661_amd import serve
    torch.cuda.set_device(0)
    ring, _ = cases.cases_c4(n_cases=1, n_steps=8000)
    deg = np.bincount(ring.frm, minlength=ring.n_bus) + np.bincount(ring.to, minlength=ring.n_bus)
    assert min(deg[ring.frm[145]], deg[ring.to[145]]) == 1
    torus = cases.serve_network(5728, 11)
    arr = [cases.Arrival(0.0, cases.Case(ring, 6000, np.array([2000], np.int32), np.array([145], np.int32)), 1),
           cases.Arrival(0.0, cases.Case(torus, 1500, np.array([300], np.int32), np.array([4321], np.int32)), 2)]
    print("[gpu] FP64 incremental serving: 1432-bus floating-bus loss, 5728-bus torus", flush=True)
    res = serve.run_serving(arr, budget_bytes=1 << 40, max_slots=2, tick_steps=500, prec="fp64", warm_start=True,
                            max_refine=0, record=True, time_scale=0.0)
    assert res.completed == 2
    for i, a in enumerate(arr):
        c = a.case
        Vref, _ = oracle.emt_run(c.net, c.n_steps, loss_steps=c.loss_steps, loss_branches=c.loss_branches,
                                 solver="sparse" if c.net.n_bus > 2000 else "inv")
        err = np.abs(res.records[i] - Vref).max() / np.abs(Vref).max()
        print(f"[gpu] served {c.net.n_bus} buses: {err:.2e}", flush=True)
        assert err <= 1e-10, (i, err)
