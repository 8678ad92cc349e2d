"""GPU parity at the benchmark configurations' stated horizons.

* Contingency batch: 256 cases of the 1432-bus ring, each losing a distinct
  line at a random step in [500, 5000], 8000 steps, on the panel engine and on
  one workgroup per case: FP64 in the incremental form
  v = v_prev + P (b - G v_prev) and FP32 applies + FP64 refinement.
  - Full trajectories of 39 cases against the oracle (explicit FP64 inverse,
    re-inversion at the loss): every tie-line loss of the batch (its SMW
    endpoints sit in two workgroups' rows), every loss that leaves a bus on
    its shunt capacitor alone (26 cases: that bus keeps its voltage, a mode the
    step map does not damp, so rounding accumulates along it for the rest of
    the horizon), the earliest and the latest loss, and seeded picks.
    Peak-normalised, 1e-10.
  - Per solve at 64 seeded (case, step) points spread over all 256 cases and
    the whole horizon: the engine's own right-hand side at that step, solved by
    the oracle (library sparse LU of that step's G, pinned against the dense LU
    in the oracle tests), against the engine's voltage.  Per-vector infinity
    norm, 1e-10.
  The run is recorded in 500-step chunks (the whole record would be 23 GB).
  FP64 solved directly (v = P b) meets 1e-10 per solve and on the cases whose
  loss leaves no bus floating; on the floating ones its trajectory error grows
  after the loss (rounding of the SMW-corrected apply, amplified by the
  capacitance, adds up along the undamped mode: 1.5e-9 at worst, 8 of the 26
  above 1e-10), which is what the incremental form removes.
* 11456-bus torus: 10000 steps on the level engine, FP64 and FP32 + FP64
  refinement, one line lost at step 2000, against the oracle's sparse LU time
  loop (refactorised only at the loss step).  Peak-normalised, 1e-10.
* One 1432-bus case losing, at step 2000, a line that leaves a bus on its shunt
  capacitor alone, 10000 steps on the single-case engines (team, level): FP64
  in the incremental form and FP32 + FP64 refinement within 1e-10 of the
  oracle (solved directly, FP64 drifts along the undamped mode: 7.8e-10).
"""
import numpy as np
import pytest

import oracle
from paper_2105_10661_amd import cases

pytestmark = pytest.mark.gpu

C4_STEPS = 8000
CHUNK = 500
# The device flags a step whose last FP64-residual correction exceeds this fraction of max |v|, and the
# one-workgroup-per-case engine stops refining once a correction is below it.  The error left after the
# last correction is about the refinement's contraction factor (<= 1e-4 measured for FP32 storage, worst
# on cases whose lost line islands a bus) times that correction; over 8000 steps it adds up, so the
# engine that stops early needs 1e-9 (at 1e-7 one case drifted to 1.2e-10).  The panel's last
# correction stays below 1e-10 on this batch.  The per-solve and trajectory checks measure the error.
MIXED_CHECK = 1e-9


@pytest.fixture(scope="module")
def hv():
    import torch
    from paper_2105_10661_amd import hinv
    torch.cuda.set_device(0)
    hinv.load()
    return hinv


@pytest.fixture(scope="module")
def c4():
    base, bcases = cases.cases_c4(n_cases=256, n_steps=C4_STEPS)
    losses = [list(zip(c.loss_steps.tolist(), c.loss_branches.tolist())) for c in bcases]
    st = np.array([c[0][0] for c in losses])
    br = np.array([c[0][1] for c in losses])
    ties = [int(k) for k in np.nonzero(br >= 8 * cases.BASE_BRANCHES)[0]]
    assert len(ties) >= 1
    deg = np.bincount(base.frm, minlength=base.n_bus) + np.bincount(base.to, minlength=base.n_bus)
    floating = [k for k in range(256) if min(deg[base.frm[br[k]]], deg[base.to[br[k]]]) == 1]
    assert len(floating) == 26
    rng = np.random.default_rng(404)
    pick = set(ties) | set(floating) | {int(st.argmin()), int(st.argmax())}
    rest = [k for k in range(256) if k not in pick]
    pick |= set(int(k) for k in rng.choice(rest, 8, replace=False))
    sample = sorted(pick)
    print(f"[gpu] c4 oracle trajectories of cases {sample} (tie-line losses {ties}, floating buses {floating})",
          flush=True)
    refs = {}
    for k in sample:
        refs[k], _ = oracle.emt_run(base, C4_STEPS, loss_steps=[st[k]], loss_branches=[br[k]], solver="inv")
    points = sorted(zip(rng.integers(0, 256, 64).tolist(), rng.integers(1, C4_STEPS + 1, 64).tolist()),
                    key=lambda p: p[1])
    return base, losses, sample, refs, points, floating


def _batch_errors(hv, c4, prec, warm, refine, engine="panel"):
    """Run the batch over the horizon; per sampled case the peak-normalised trajectory error, the
    per-solve errors at the seeded points and the device status."""
    import torch
    base, losses, sample, refs, points, floating = c4
    form = "incremental" if prec == "fp64" and warm else "direct" if prec == "fp64" else f"refine {refine}"
    print(f"[gpu] c4 256 cases x {C4_STEPS} steps, {engine} engine, {prec} ({form})", flush=True)
    emt = hv.EMT(base, 256, losses=losses, prec=prec, max_refine=refine, rel_tol=MIXED_CHECK, warm_start=warm,
                 max_mod_rank=1, kernel_mode=engine)
    Vbuf = torch.empty((CHUNK, 256, base.n_bus), dtype=torch.float64, device="cuda")
    Bbuf = torch.empty_like(Vbuf)
    idx = torch.tensor(sample, device="cuda")
    dmax = {k: 0.0 for k in sample}
    solve_err = []
    pi = 0
    for c0 in range(0, C4_STEPS, CHUNK):
        emt.step(CHUNK, record_b=True, v_out=Vbuf, b_out=Bbuf)
        Vs = Vbuf.index_select(1, idx).cpu().numpy()
        for j, k in enumerate(sample):
            d = np.abs(Vs[:, j, :] - refs[k][c0:c0 + CHUNK]).max()
            dmax[k] = max(dmax[k], float(d))
        while pi < len(points) and points[pi][1] <= c0 + CHUNK:
            k, s = points[pi]
            lst, lbr = losses[k][0]
            alive = np.ones(base.n_branch, bool)
            if s >= lst:
                alive[lbr] = False
            b = Bbuf[s - 1 - c0, k].cpu().numpy()
            v = Vbuf[s - 1 - c0, k].cpu().numpy()
            x = oracle.sparse_solver(base, alive)(b)
            solve_err.append((np.abs(v - x).max() / np.abs(x).max(), k, s))
            pi += 1
    try:
        emt.sync_status()
        status = "ok"
    except hv.HinvError as e:
        status = e.name
    emt.close()
    assert pi == len(points)
    worst = max(solve_err)
    traj = {k: dmax[k] / np.abs(refs[k]).max() for k in sample}
    print(f"[gpu] c4 {prec} ({form}): per-solve max {worst[0]:.2e} at case {worst[1]} step {worst[2]}; "
          "trajectories " + ", ".join(f"{k}:{traj[k]:.1e}" for k in sample), flush=True)
    return traj, worst, status


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec,warm,refine", [("fp64", True, 0), ("fp32", True, 2)])
def test_contingency_batch_full_horizon(hv, c4, prec, warm, refine):
    traj, worst, status = _batch_errors(hv, c4, prec, warm, refine)
    assert worst[0] <= 1e-10, worst
    for k, e in traj.items():
        assert e <= 1e-10, (k, e)
    assert status == "ok", status


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec,warm,refine", [("fp64", True, 0), ("fp32", True, 2)])
def test_contingency_batch_full_horizon_one_workgroup_per_case(hv, c4, prec, warm, refine):
    """The same batch, horizon and checks with one workgroup per case.  Its line-loss coefficient is
    u^T x of the apply's input, as on the panel: taken from the apply's FP32 values at the loss's
    endpoints instead, the refined path drifted to 1.8e-10 on the batch (at rel_tol 1e-7)."""
    traj, worst, status = _batch_errors(hv, c4, prec, warm, refine, engine="fused")
    assert worst[0] <= 1e-10, worst
    for k, e in traj.items():
        assert e <= 1e-10, (k, e)
    assert status == "ok", status


@pytest.mark.timeout(900)
def test_contingency_batch_direct_fp64(hv, c4):
    """FP64 solved directly: 1e-10 per solve and on every sampled case whose loss leaves no bus
    floating; on the floating ones the drift along the undamped mode is bounded by 2e-9 (1.5e-9
    measured), recorded here as the reason the incremental form exists."""
    floating = set(c4[5])
    traj, worst, status = _batch_errors(hv, c4, "fp64", False, 0)
    assert worst[0] <= 1e-10, worst
    for k, e in traj.items():
        assert e <= (2e-9 if k in floating else 1e-10), (k, e)
    assert status == "ok", status


@pytest.fixture(scope="module")
def c3_ref():
    net = cases.case_c3(n_steps=10000).net
    print("[gpu] c3 oracle trajectory (sparse LU, 10000 steps, loss at 2000)", flush=True)
    Vref, _ = oracle.emt_run(net, 10000, loss_steps=[2000], loss_branches=[4321], solver="sparse")
    return net, Vref


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec,warm,refine", [("fp64", False, 0), ("fp32", True, 2)])
def test_torus_11456_full_horizon(hv, c3_ref, prec, warm, refine):
    import torch
    net, Vref = c3_ref
    print(f"[gpu] c3 11456 buses x 10000 steps, level engine, {prec} (refine {refine})", flush=True)
    emt = hv.EMT(net, 1, losses=[[(2000, 4321)]], prec=prec, max_refine=refine, rel_tol=MIXED_CHECK,
                 warm_start=warm, kernel_mode="level")
    V = torch.empty((10000, 1, net.n_bus), dtype=torch.float64, device="cuda")
    for c0 in range(0, 10000, CHUNK):
        emt.step(CHUNK, v_out=V[c0:c0 + CHUNK])
    emt.sync_status()
    emt.close()
    d = np.abs(V[:, 0, :].cpu().numpy() - Vref)
    err = d.max() / np.abs(Vref).max()
    print(f"[gpu] c3 {prec}: peak-normalised {err:.2e}, per-step-normalised "
          f"{(d.max(1) / np.abs(Vref).max(1)).max():.2e}", flush=True)
    assert err <= 1e-10


@pytest.fixture(scope="module")
def floating_single():
    base, _ = cases.cases_c4(n_cases=256, n_steps=C4_STEPS)
    deg = np.bincount(base.frm, minlength=base.n_bus) + np.bincount(base.to, minlength=base.n_bus)
    br = 145          # a line whose loss leaves a bus on its shunt capacitor (direct FP64 drifts most here)
    assert min(deg[base.frm[br]], deg[base.to[br]]) == 1
    print(f"[gpu] single-case oracle: branch {br} lost at step 2000, 10000 steps", flush=True)
    Vref, _ = oracle.emt_run(base, 10000, loss_steps=[2000], loss_branches=[br], solver="inv")
    return base, br, Vref


@pytest.mark.timeout(600)
@pytest.mark.parametrize("mode,prec,refine", [(m, p, r) for p, r in [("fp64", 0), ("fp32", 2)] for m in ("team", "level")]
                         + [("per_kernel", "fp64", 0)])
def test_single_case_floating_bus_full_horizon(hv, floating_single, mode, prec, refine):
    base, br, Vref = floating_single
    print(f"[gpu] single case, floating-bus loss, {mode} engine, {prec} warm", flush=True)
    emt = hv.EMT(base, 1, losses=[[(2000, br)]], prec=prec, max_refine=refine, rel_tol=MIXED_CHECK, warm_start=True,
                 kernel_mode=mode)
    err = 0.0
    for c0 in range(0, 10000, 2000):
        V, _ = emt.step(2000)
        err = max(err, float(np.abs(V[:, 0, :].cpu().numpy() - Vref[c0:c0 + 2000]).max()))
    emt.sync_status()
    emt.close()
    err /= float(np.abs(Vref).max())
    print(f"[gpu] {mode} {prec}: {err:.2e}", flush=True)
    assert err <= 1e-10


@pytest.mark.timeout(600)
def test_single_case_floating_bus_direct_fp64_drifts(hv, floating_single):
    """The same case solved directly in FP64 on the team engine drifts past 1e-10 along the undamped
    mode (7.8e-10 measured), which is why the single-case engines take the incremental form too."""
    base, br, Vref = floating_single
    emt = hv.EMT(base, 1, losses=[[(2000, br)]], prec="fp64", max_refine=0, rel_tol=MIXED_CHECK, warm_start=False,
                 kernel_mode="team")
    err = 0.0
    for c0 in range(0, 10000, 2000):
        V, _ = emt.step(2000)
        err = max(err, float(np.abs(V[:, 0, :].cpu().numpy() - Vref[c0:c0 + 2000]).max()))
    emt.sync_status()
    emt.close()
    err /= float(np.abs(Vref).max())
    print(f"[gpu] team fp64 direct: {err:.2e}", flush=True)
    assert 1e-10 < err <= 5e-9
