"""Autotuner of the EMT time loop's launch configuration.

For one network, case count and loss schedule it picks, by timing on the device:

- the partition tree among the caller's candidates.  The leaf blocks are the tiles of every leaf
  product: in the panel engine a leaf of m rows is an m x m by m x 16 product on the matrix cores
  (16x16x4 MFMA tiles), in the other engines an m x m GEMV per case.  Smaller leaves mean fewer leaf
  flops but more coupling columns and levels, the trade-off of the leaf-size threshold of the
  hierarchy (Section III.B);
- the engine (the schedule of a step): 16-case panels with one workgroup per leaf and per panel
  (``panel``), one workgroup per case (``fused``), one cooperative team per case (``team``, ``level``)
  or one launch per phase (``per_kernel``);
- the precision path: FP64 solved directly (v = P b), FP64 in the incremental form (v = v_prev +
  P (b - G v_prev), one apply per step; on the engines that have it), or FP32 applies with FP64
  residual refinement and a fixed number of corrections per step (warm start from the previous
  step's voltages).

A candidate is kept only if the library accepts it (``emt_workspace_size``, host only: leaf, column
and LDS limits of the engine) and if its voltages stay within ``gate`` of the FP64 path of the same
library on the same tree (the incremental form where the tree has a feasible one: the direct form
lets rounding accumulate along a bus that a line loss leaves on its shunt capacitor alone, up to
1.5e-9 over the contingency batch's horizon) over the run's whole ``horizon``: every case and bus at
every one of the first ``gate_steps`` steps and at every ``stride``-th step after them, each case
normalised by its own peak voltage.  The trajectories drift slowly (the trapezoidal step map has an eigenvalue of 1), so a
sampled step every few dozen misses nothing between samples.  The fastest kept candidate wins.  Each
row also carries the error over the first ``gate_steps`` steps and its linear extrapolation to the
horizon, the cheaper estimate this gate replaced: measured on the 256-case contingency batch it
overstated the full-horizon error of the mixed paths several times over.  Every measurement runs in the library's kernels; this module only times them
and compares their outputs.

Results persist as JSON, keyed by the network (branch endpoints, tree candidates), the cases, the
device name and the library binary, so a later call with the same key returns the stored choice
without timing anything.
"""
from __future__ import annotations

import hashlib
import json
import os
from dataclasses import asdict, dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import hinv

SINGLE_CASE_ENGINES = ("team", "level", "fused", "per_kernel")
BATCH_ENGINES = ("panel", "fused")
# (precision, corrections per step, warm start)
DEFAULT_PATHS = (("fp64", 0, False), ("fp64", 0, True), ("fp32", 1, True), ("fp32", 2, True))
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_2105_10661_amd", "tune.json")


@dataclass(frozen=True)
class Candidate:
    tree: str
    engine: str
    prec: str
    max_refine: int
    warm: bool

    def label(self) -> str:
        if self.prec == "fp64":
            p = "fp64inc" if self.warm else "fp64"
        else:
            p = f"{self.prec}+{self.max_refine}ir"
        return f"{self.tree}/{self.engine}/{p}"


@dataclass
class Row:
    cand: Candidate
    feasible: bool
    reason: str = ""
    workspace_mb: float = 0.0
    us_per_step: float = float("inf")
    solves_per_s: float = 0.0
    err: float = float("inf")              # over the whole horizon (the gate)
    err_first: float = float("inf")        # over the first gate_steps steps only
    err_extrapolated: float = float("inf")  # err_first x horizon / gate_steps
    applies_per_step: float = 0.0
    status: str = ""

    def to_json(self) -> dict:
        d = asdict(self)
        d["cand"] = asdict(self.cand)
        d["label"] = self.cand.label()
        for k in ("us_per_step", "err", "err_first", "err_extrapolated"):
            if not np.isfinite(d[k]):
                d[k] = None
        return d

    @staticmethod
    def from_json(d: dict) -> "Row":
        d = dict(d)
        d.pop("label", None)
        d["cand"] = Candidate(**d["cand"])
        for k in ("us_per_step", "err", "err_first", "err_extrapolated"):
            if d.get(k) is None:
                d[k] = float("inf")
        return Row(**d)


@dataclass
class TuneResult:
    key: str
    choice: Optional[Candidate]
    rows: List[Row] = field(default_factory=list)
    cached: bool = False
    gate: float = 1e-10

    def best(self) -> Optional[Row]:
        for r in self.rows:
            if self.choice is not None and r.cand == self.choice:
                return r
        return None

    def table(self) -> List[dict]:
        return [r.to_json() for r in self.rows]


def enumerate_candidates(trees: Sequence[str], engines: Sequence[str],
                         paths: Sequence[Tuple[str, int, bool]]) -> List[Candidate]:
    return [Candidate(t, e, p, int(mr), bool(w)) for t in trees for e in engines for (p, mr, w) in paths]


def select(rows: Sequence[Row], gate: float) -> Optional[Candidate]:
    """Fastest candidate that the library accepted, that ran without a device error and whose error
    against the FP64 reference is within the gate; ties go to the earlier candidate.  A device report
    that a step's last correction stayed above rel_tol (NO_CONVERGENCE) does not exclude a candidate:
    its measured error decides."""
    best = None
    for r in rows:
        if not r.feasible or r.status not in ("ok", "NO_CONVERGENCE") or not (r.err <= gate) \
                or not np.isfinite(r.us_per_step):
            continue
        if best is None or r.us_per_step < best.us_per_step:
            best = r
    return None if best is None else best.cand


def with_tree(net, parent, bus_leaf):
    """The same network with another partition tree."""
    import copy
    out = copy.copy(net)
    out.parent = np.ascontiguousarray(parent, np.int32)
    out.bus_leaf = np.ascontiguousarray(bus_leaf, np.int32)
    return out


def cache_key(net, trees: Dict[str, Tuple[np.ndarray, np.ndarray]], losses, max_mod_rank: int,
              engines: Sequence[str], paths, gate: float, device_name: str, lib_path: str) -> str:
    h = hashlib.sha1()
    for a in (net.frm, net.to, net.R, net.L, net.C, net.src_bus):
        h.update(np.ascontiguousarray(a).tobytes())
    for name in sorted(trees):
        h.update(name.encode())
        for a in trees[name]:
            h.update(np.ascontiguousarray(a, np.int32).tobytes())
    h.update(json.dumps([losses, max_mod_rank, list(engines), [list(p) for p in paths], gate,
                         device_name]).encode())
    with open(lib_path, "rb") as f:
        h.update(hashlib.sha1(f.read()).digest())
    return h.hexdigest()


def load_cache(path: str) -> dict:
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def save_cache(path: str, key: str, res: TuneResult) -> bool:
    """Add one result to the JSON cache; returns False (and keeps the result) if the file cannot be
    written, e.g. on a read-only home directory."""
    d = load_cache(path)
    d[key] = {"choice": None if res.choice is None else asdict(res.choice), "rows": res.table(), "gate": res.gate}
    try:
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1)
        os.replace(tmp, path)
    except OSError:
        return False
    return True


def from_cache(path: str, key: str) -> Optional[TuneResult]:
    e = load_cache(path).get(key)
    if not e:
        return None
    choice = None if e["choice"] is None else Candidate(**e["choice"])
    return TuneResult(key, choice, [Row.from_json(r) for r in e["rows"]], cached=True, gate=e.get("gate", 1e-10))


def check_feasible(net, cand: Candidate, n_cases: int, losses, max_mod_rank: int, rel_tol: float) -> Row:
    try:
        nb = hinv.emt_workspace_bytes(net, n_cases, losses, prec=cand.prec, rel_tol=rel_tol,
                                      max_refine=cand.max_refine, max_mod_rank=max_mod_rank, warm_start=cand.warm,
                                      kernel_mode=cand.engine)
    except hinv.HinvError as e:
        return Row(cand, False, reason=str(e))
    return Row(cand, True, workspace_mb=round(nb / 2**20, 2))


def _emt(net, cand: Candidate, n_cases, losses, max_mod_rank, rel_tol):
    return hinv.EMT(net, n_cases, losses=losses, prec=cand.prec, max_refine=cand.max_refine, rel_tol=rel_tol,
                    max_mod_rank=max_mod_rank, warm_start=cand.warm, kernel_mode=cand.engine)


def _status(emt) -> str:
    try:
        emt.sync_status()
        return "ok"
    except hinv.HinvError as e:
        return e.name


def _run(net, cand: Candidate, ref_net, ref_cand: Candidate, n_cases, losses, max_mod_rank, rel_tol, gate_steps,
         horizon, stride, chunk, timed_steps, reps):
    """One candidate.  Gate: the candidate and the FP64 reference in lockstep over the horizon; per
    case, max |v - v_ref| over every bus at every one of the first gate_steps steps (in chunks; also
    the warm-up) and at every stride-th step after them, divided by that case's max |v_ref| over the
    same steps; the gate error is the largest over the cases (a peak over all cases would understate
    the error of a case whose voltages are small next to another's).
    Then `reps` timed launches of timed_steps each (HIP events on the launch stream).  Returns
    (us per step, error over the horizon, error over the first gate_steps steps, applies per step,
    status of the candidate, status of the reference)."""
    import torch
    emt = _emt(net, cand, n_cases, losses, max_mod_rank, rel_tol)
    try:
        same = cand == ref_cand
        ref = None if same else _emt(ref_net, ref_cand, n_cases, losses, max_mod_rank, rel_tol)
        # per case: largest |v - v_ref| and largest |v_ref| over the compared steps and buses
        dmax, peak, done = torch.zeros(n_cases, dtype=torch.float64), torch.zeros(n_cases, dtype=torch.float64), 0
        first = (dmax.clone(), peak.clone())
        try:
            def compare(k):
                nonlocal dmax, peak
                V, _ = emt.step(k, record_v=True)
                if ref is not None:
                    Vr, _ = ref.step(k, record_v=True)
                    # recorded rows are in original bus order for every engine and tree
                    dmax = torch.maximum(dmax, (V - Vr).abs().amax(dim=(0, 2)).cpu())
                    peak = torch.maximum(peak, Vr.abs().amax(dim=(0, 2)).cpu())
                    del Vr
                del V

            while done < gate_steps:
                k = min(chunk, gate_steps - done)
                compare(k)
                done += k
            first = (dmax.clone(), peak.clone())
            while done < horizon:
                skip = min(stride - 1, horizon - done - 1)
                if skip > 0:
                    emt.step(skip, record_v=False)
                    if ref is not None:
                        ref.step(skip, record_v=False)
                    done += skip
                compare(1)
                done += 1
            ref_status = "ok" if ref is None else _status(ref)
        finally:
            if ref is not None:
                ref.close()
        def worst(d, p):    # the largest error of any case, each normalised by its own peak voltage
            return float("inf") if bool((p <= 0).any()) else float((d / p).max())
        err = 0.0 if same else worst(dmax, peak)
        err_first = 0.0 if same else worst(*first)
        s = torch.cuda.current_stream()
        ms = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            emt.step(timed_steps, record_v=False)
            e1.record(s)
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        applies, _ = emt.stats()
        status = _status(emt)
        aps = applies / (n_cases * (horizon + reps * timed_steps))
        us = float(np.median(ms)) * 1e3 / timed_steps
        return us, err, err_first, aps, status, ref_status
    finally:
        emt.close()


def tune(net, trees: Optional[Dict[str, Tuple[np.ndarray, np.ndarray]]] = None, n_cases: int = 1, losses=None,
         engines: Optional[Sequence[str]] = None, paths: Sequence[Tuple[str, int, bool]] = DEFAULT_PATHS,
         max_mod_rank: int = 2, rel_tol: float = 1e-9, gate: float = 1e-10, gate_steps: int = 1000,
         horizon: Optional[int] = None, stride: int = 50, chunk: int = 250, timed_steps: int = 200, reps: int = 3,
         cache: Optional[str] = DEFAULT_CACHE, refresh: bool = False, log=None) -> TuneResult:
    """Pick the fastest accurate configuration for n_cases cases of `net` (see the module docstring).

    trees: label -> (parent, bus_leaf); default: the network's own tree, labelled "given".
    losses: per case a list of (step, branch), as for hinv.EMT; losses inside the first gate_steps
    steps make the gate cover the rank-r corrections.
    horizon: steps the cases will run.  The trajectory error of a low-precision path grows with the
    step count (the trapezoidal step map has an eigenvalue of 1), so the gate runs every candidate
    over the whole horizon, comparing every step of the first gate_steps and every `stride`-th after.
    cache: JSON file of earlier results (None: no cache); refresh: time again even if cached.
    """
    import torch
    if trees is None:
        trees = {"given": (net.parent, net.bus_leaf)}
    if engines is None:
        engines = BATCH_ENGINES if n_cases > 1 else SINGLE_CASE_ENGINES
    if losses is None:
        losses = [[] for _ in range(n_cases)]
    losses = [[(int(s), int(b)) for (s, b) in lst] for lst in losses]
    horizon = max(int(horizon or gate_steps), gate_steps)
    scale = horizon / gate_steps
    stride = max(1, int(stride))
    key = cache_key(net, trees, losses, max_mod_rank, engines, paths, gate,
                    f"{torch.cuda.get_device_name()} gate {gate_steps} horizon {horizon} stride {stride}",
                    hinv.LIB_PATH)
    if cache and not refresh:
        hit = from_cache(cache, key)
        if hit is not None:
            return hit
    nets = {name: with_tree(net, *tr) for name, tr in trees.items()}
    rows = [check_feasible(nets[c.tree], c, n_cases, losses, max_mod_rank, rel_tol)
            for c in enumerate_candidates(list(trees), engines, paths)]
    # FP64 reference of the same library on the candidate's own tree (its first feasible FP64 candidate in
    # the incremental form, else its first feasible FP64 one, else auto): two exact FP64 trees drift apart
    # by rounding along the recursion's unit eigenvalue, which is not an error of either
    def reference(t):
        fp64 = [r.cand for r in rows if r.feasible and r.cand.tree == t and r.cand.prec == "fp64"]
        inc = [c for c in fp64 if c.warm and c.engine in ("panel", "fused")]
        return (inc or fp64 or [Candidate(t, "auto", "fp64", 0, False)])[0]
    ref_cands = {t: reference(t) for t in trees}
    for r in rows:
        if not r.feasible:
            continue
        ref_cand = ref_cands[r.cand.tree]
        us, err, err_first, aps, status, ref_status = _run(
            nets[r.cand.tree], r.cand, nets[r.cand.tree], ref_cand, n_cases, losses, max_mod_rank, rel_tol,
            gate_steps, horizon, stride, chunk, timed_steps, reps)
        if ref_status != "ok":
            raise hinv.HinvError(4, "tune", f"the FP64 reference run ({ref_cand.label()}) ended with {ref_status}")
        r.us_per_step, r.err, r.applies_per_step, r.status = us, err, round(aps, 3), status
        r.err_first, r.err_extrapolated = err_first, err_first * scale
        r.solves_per_s = round(n_cases / (us * 1e-6), 1)
        if log:
            log(f"tune {r.cand.label()}: {us:.2f} us/step, err {err:.2e} over {horizon} steps "
                f"({err_first:.2e} over {gate_steps}), {status}")
    res = TuneResult(key, select(rows, gate), rows, cached=False, gate=gate)
    if cache:
        save_cache(cache, key, res)
    return res
