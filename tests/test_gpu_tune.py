"""GPU checks of the autotuner on a 32-case contingency batch of the 716-bus ring.

* Two partition trees (2 and 4 leaves per 179-bus copy) x two engines (16-case panels on the matrix
  cores, one workgroup per case) x four precision paths are timed; every candidate that ran has an
  error against the FP64 reference (the incremental form) over the horizon (every step of the first
  160, every 40th after; each case normalised by its own peak), the incremental FP64 candidates at
  the FP64 floor.
* The choice is the fastest candidate within the gate, and it is accurate against the FP64 oracle
  on sampled cases (1e-10 of the peak voltage).
* A second call with the same key comes from the JSON cache without running anything.
"""
import time

import numpy as np
import pytest

import oracle
from paper_2105_10661_amd import cases

pytestmark = pytest.mark.gpu

STEPS = 160
HORIZON = 400       # the gate samples every 40th step after the first 160


@pytest.fixture(scope="module")
def tuned(tmp_path_factory):
    import torch
    from paper_2105_10661_amd import hinv, tune
    torch.cuda.set_device(0)
    hinv.load()
    nets = {f"{2 ** cl} leaves per copy": cases.tiled_network("716-bus ring", 1, 4, 12, copy_levels=cl)
            for cl in (1, 2)}
    net = next(iter(nets.values()))
    rng = np.random.default_rng(3)
    br = rng.choice(net.n_branch, 32, replace=False)
    st = rng.integers(1, 100, size=32)
    losses = [[(int(s), int(b))] for s, b in zip(st, br)]
    trees = {k: (v.parent, v.bus_leaf) for k, v in nets.items()}
    path = str(tmp_path_factory.mktemp("tune") / "tune.json")
    res = tune.tune(net, trees, n_cases=32, losses=losses, max_mod_rank=1, gate_steps=STEPS, horizon=HORIZON,
                    stride=40, timed_steps=50, reps=2, cache=path)
    return tune, net, nets, losses, trees, path, res


def test_every_candidate_ran_or_was_refused(tuned):
    tune, net, nets, losses, trees, path, res = tuned
    assert not res.cached
    assert len(res.rows) == 2 * 2 * len(tune.DEFAULT_PATHS)
    for r in res.rows:
        if not r.feasible:
            assert r.reason
            continue
        assert r.status in ("ok", "NO_CONVERGENCE"), (r.cand, r.status)
        assert np.isfinite(r.us_per_step) and r.us_per_step > 0
        assert np.isfinite(r.err)
        assert r.err >= r.err_first          # the horizon includes the first gate_steps steps
        assert r.err_extrapolated == pytest.approx(r.err_first * HORIZON / STEPS)
        if r.cand.prec == "fp64" and r.cand.warm:
            assert r.err <= 1e-11, (r.cand, r.err)
        elif r.cand.prec == "fp64":
            # the direct form drifts along a bus that a loss leaves floating (its error grows with the
            # steps after the loss); each case is normalised by its own peak voltage
            assert r.err <= 1e-9, (r.cand, r.err)
    assert sum(r.feasible for r in res.rows) >= 8


def test_choice_is_the_fastest_within_the_gate(tuned):
    tune, net, nets, losses, trees, path, res = tuned
    assert res.choice is not None
    ok = [r for r in res.rows if r.feasible and r.status in ("ok", "NO_CONVERGENCE") and r.err <= res.gate]
    assert min(ok, key=lambda r: r.us_per_step).cand == res.choice
    assert res.best().err <= 1e-10


def test_choice_matches_the_oracle(tuned):
    import torch
    from paper_2105_10661_amd import hinv
    tune, net, nets, losses, trees, path, res = tuned
    c = res.choice
    tnet = tune.with_tree(net, *trees[c.tree])
    emt = hinv.EMT(tnet, 32, losses=losses, prec=c.prec, max_refine=c.max_refine, max_mod_rank=1,
                   warm_start=c.warm, kernel_mode=c.engine)
    V, _ = emt.step(STEPS)
    torch.cuda.synchronize()
    V = V.cpu().numpy()
    emt.close()
    for k in (0, 13, 31):
        (s, b), = losses[k]
        Vo, _ = oracle.emt_run(net, STEPS, loss_steps=[s], loss_branches=[b], solver="lu")
        err = np.abs(V[:, k, :] - Vo).max() / np.abs(Vo).max()
        assert err <= 1e-10, (c, k, err)


def test_second_call_comes_from_the_cache(tuned):
    tune, net, nets, losses, trees, path, res = tuned
    t = time.perf_counter()
    again = tune.tune(net, trees, n_cases=32, losses=losses, max_mod_rank=1, gate_steps=STEPS, horizon=HORIZON,
                      stride=40, timed_steps=50, reps=2, cache=path)
    assert again.cached and again.choice == res.choice and again.key == res.key
    assert [r.us_per_step for r in again.rows] == pytest.approx([r.us_per_step for r in res.rows])
    assert time.perf_counter() - t < 5.0
