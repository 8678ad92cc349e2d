"""ctypes binding of libhinv.so (argument marshalling only).

Device memory and streams come from PyTorch: workspaces and vectors are torch
tensors on a ROCm device, streams are ``torch.cuda.current_stream()``.  Every
step of the computation runs in the library's HIP kernels; if the library is
not built this module raises instead of computing anything itself.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhinv.so")

FP64, FP32, BF16, FP8 = 0, 1, 2, 3
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16": BF16, "fp8": FP8}

STATUS = {0: "OK", 1: "INVALID", 2: "NOT_SPD", 3: "NO_MEMORY", 4: "DEVICE", 5: "NO_SUCH_LINE",
          6: "NO_CONVERGENCE", 7: "RANK_LIMIT", 8: "SINGULAR"}

EXPORTS = ("hinv_workspace_size", "hinv_build", "hinv_modify_line", "hinv_update_line", "hinv_solve",
           "hinv_solve_noalloc", "hinv_sync_status",
           "hinv_get_info", "hinv_destroy", "emt_network_csr", "emt_network3_csr", "emt_workspace_size", "emt_create",
           "emt_step", "emt_lose_line", "emt_update_line", "emt_sync_status", "emt_get_step", "emt_get_stats",
           "emt_set_step_clock", "emt_destroy",
           "hinv_wall_clock_khz", "serve_workspace_size", "serve_create", "serve_attach", "serve_detach",
           "serve_step", "serve_active", "serve_destroy", "chol_workspace_size", "chol_create", "chol_solve",
           "chol_get_info", "chol_destroy", "hinv_last_error", "emt3_workspace_size", "emt3_create",
           "hinv_gmres_workspace_size", "hinv_solve_gmres", "emt_state_size", "emt_save_state", "emt_load_state")


class HinvError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class _CSR(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
                ("val", ctypes.c_void_p)]


class _Tree(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int32), ("parent", ctypes.c_void_p), ("bus_leaf", ctypes.c_void_p)]


class _Options(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int32), ("rel_tol", ctypes.c_double), ("max_refine", ctypes.c_int32),
                ("max_mod_rank", ctypes.c_int32), ("max_nrhs", ctypes.c_int32), ("warm_start", ctypes.c_int32),
                ("kernel_mode", ctypes.c_int32), ("coupling", ctypes.c_int32)]


COUPLINGS = {"exact": 0, "paper": 1}


class _Info(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("n", "n_leaves", "n_internal", "n_levels", "n_cols", "leaf_entries",
                                             "z_entries", "s_entries", "max_leaf", "max_cols")] + \
               [("apply_flops", ctypes.c_double), ("build_flops", ctypes.c_double)]


class _GmresInfo(ctypes.Structure):
    _fields_ = [("corrections", ctypes.c_int32), ("inner_iterations", ctypes.c_int32), ("last_update", ctypes.c_double)]


class _UpdateInfo(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int32) for k in ("lca_level", "leaves", "columns", "nodes")]


class _CholInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz_l", ctypes.c_int64), ("fwd_levels", ctypes.c_int64),
                ("bwd_levels", ctypes.c_int64), ("solve_flops", ctypes.c_double), ("factor_flops", ctypes.c_double)]


class _Network(ctypes.Structure):
    _fields_ = [("n_bus", ctypes.c_int32), ("n_branch", ctypes.c_int32), ("from_", ctypes.c_void_p),
                ("to", ctypes.c_void_p), ("R", ctypes.c_void_p), ("L", ctypes.c_void_p), ("C", ctypes.c_void_p),
                ("dt", ctypes.c_double), ("n_src", ctypes.c_int32), ("src_bus", ctypes.c_void_p),
                ("amp", ctypes.c_void_p), ("phase", ctypes.c_void_p), ("freq", ctypes.c_double)]


class _Cases(ctypes.Structure):
    _fields_ = [("n_cases", ctypes.c_int32), ("loss_ptr", ctypes.c_void_p), ("loss_step", ctypes.c_void_p),
                ("loss_branch", ctypes.c_void_p)]


_lib = None
_live = weakref.WeakSet()      # every open handle, closed explicitly at interpreter exit


def close_all() -> None:
    """Destroy every handle still open: serving pools first, then EMT batches, then hierarchies and
    factorisations.  Registered with atexit when the library is loaded (after torch, so it runs before
    torch's own exit handlers), so no handle is left to garbage collection during interpreter teardown."""
    order = {"Serve": 0, "EMT": 1, "Hierarchy": 2, "Chol": 2}
    for obj in sorted(list(_live), key=lambda o: order.get(type(o).__name__, 3)):
        obj.close()


def load() -> ctypes.CDLL:
    """Load libhinv.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "hinv_workspace_size": [P, P, P, P],
        "hinv_build": [P, P, P, P, ctypes.c_size_t, P, P],
        "hinv_modify_line": [P, i32, i32, d, P],
        "chol_workspace_size": [P, P],
        "chol_create": [P, P, ctypes.c_size_t, P, P],
        "chol_solve": [P, P, P, i32, i32, P],
        "chol_get_info": [P, P],
        "chol_destroy": [P],
        "hinv_update_line": [P, i32, i32, d, P, P],
        "hinv_solve": [P, P, P, i32, i32, P],
        "hinv_solve_noalloc": [P, P, P, i32, i32, P],
        "hinv_sync_status": [P],
        "hinv_get_info": [P, P],
        "hinv_destroy": [P],
        "emt_network_csr": [P, P, P, P, P],
        "emt_network3_csr": [P, d, P, P, P, P],
        "emt_workspace_size": [P, P, P, P, P],
        "emt_create": [P, P, P, P, P, ctypes.c_size_t, P, P],
        "emt3_workspace_size": [P, d, P, P, P, P, P],
        "hinv_gmres_workspace_size": [P, i32, i32, P],
        "hinv_solve_gmres": [P, P, P, i32, i32, i32, i32, i32, d, d, P, ctypes.c_size_t, P, P],
        "emt3_create": [P, d, P, P, P, P, P, ctypes.c_size_t, P, P],
        "emt_step": [P, i32, P, P, P],
        "emt_lose_line": [P, i32, i32, P],
        "emt_update_line": [P, i32, i32, d, P, P],
        "emt_sync_status": [P],
        "emt_get_step": [P, P],
        "emt_state_size": [P, P],
        "emt_save_state": [P, P, ctypes.c_size_t, P],
        "emt_load_state": [P, P, ctypes.c_size_t, P],
        "emt_get_stats": [P, P, P],
        "emt_set_step_clock": [P, P, i64],
        "hinv_wall_clock_khz": [i32, P],
        "serve_workspace_size": [i32, P],
        "serve_create": [P, i32, P, ctypes.c_size_t, P],
        "serve_attach": [P, P, P, i64, P, P],
        "serve_detach": [P, i32, P],
        "serve_step": [P, i32, P],
        "serve_active": [P, P],
        "serve_destroy": [P],
        "emt_destroy": [P],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.hinv_last_error.restype = ctypes.c_char_p
    lib.hinv_last_error.argtypes = []
    _lib = lib
    atexit.register(close_all)
    return lib


def _check(st: int, where: str) -> None:
    if st != 0:
        raise HinvError(st, where, load().hinv_last_error().decode())


def _ptr(a) -> int:
    if a is None:
        return 0
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


def _stream(torch_stream=None) -> int:
    import torch
    s = torch_stream if torch_stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


KERNEL_MODES = {"auto": 0, "per_kernel": 1, "fused": 2, "team": 3, "panel": 4, "level": 5}


def _options(prec, rel_tol, max_refine, max_mod_rank, max_nrhs, warm_start=False, kernel_mode="auto",
             coupling="exact") -> _Options:
    if isinstance(prec, str):
        prec = PRECISIONS[prec]
    if isinstance(kernel_mode, str):
        kernel_mode = KERNEL_MODES[kernel_mode]
    if isinstance(coupling, str):
        coupling = COUPLINGS[coupling]
    return _Options(int(prec), float(rel_tol), int(max_refine), int(max_mod_rank), int(max_nrhs),
                    int(bool(warm_start)), int(kernel_mode), int(coupling))


class _NetArrays:
    """Keeps the contiguous host arrays of a network alive while the library reads them."""

    def __init__(self, net):
        c = np.ascontiguousarray
        self.frm = c(net.frm, np.int32)
        self.to = c(net.to, np.int32)
        self.R = c(net.R, np.float64)
        self.L = c(net.L, np.float64)
        self.C = c(net.C, np.float64)
        self.sb = c(net.src_bus, np.int32)
        self.sa = c(net.src_amp, np.float64)
        self.sp = c(net.src_phase, np.float64)
        self.parent = c(net.parent, np.int32)
        self.bus_leaf = c(net.bus_leaf, np.int32)
        self.s = _Network(int(net.n_bus), int(len(self.frm)), _ptr(self.frm), _ptr(self.to), _ptr(self.R),
                          _ptr(self.L), _ptr(self.C), float(net.dt), int(len(self.sb)), _ptr(self.sb),
                          _ptr(self.sa), _ptr(self.sp), float(net.freq))
        self.tree = _Tree(int(len(self.parent)), _ptr(self.parent), _ptr(self.bus_leaf))


def wall_clock_khz(device: int = 0) -> int:
    v = ctypes.c_int32(0)
    _check(load().hinv_wall_clock_khz(int(device), ctypes.byref(v)), "hinv_wall_clock_khz")
    return v.value


def network_csr(net) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """G of the network as assembled by the library (row_ptr, col_idx, val)."""
    lib = load()
    na = _NetArrays(net)
    nnz = ctypes.c_int64(0)
    _check(lib.emt_network_csr(ctypes.byref(na.s), None, None, None, ctypes.byref(nnz)), "emt_network_csr")
    rp = np.zeros(net.n_bus + 1, np.int32)
    ci = np.zeros(nnz.value, np.int32)
    cv = np.zeros(nnz.value, np.float64)
    _check(lib.emt_network_csr(ctypes.byref(na.s), _ptr(rp), _ptr(ci), _ptr(cv), ctypes.byref(nnz)),
           "emt_network_csr")
    return rp, ci, cv


def network3_csr(net, mutual: float) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Three-phase G of the network (rows 3a + p) as assembled by the library (row_ptr, col_idx, val)."""
    lib = load()
    na = _NetArrays(net)
    nnz = ctypes.c_int64(0)
    _check(lib.emt_network3_csr(ctypes.byref(na.s), float(mutual), None, None, None, ctypes.byref(nnz)),
           "emt_network3_csr")
    rp = np.zeros(3 * net.n_bus + 1, np.int32)
    ci = np.zeros(nnz.value, np.int32)
    cv = np.zeros(nnz.value, np.float64)
    _check(lib.emt_network3_csr(ctypes.byref(na.s), float(mutual), _ptr(rp), _ptr(ci), _ptr(cv), ctypes.byref(nnz)),
           "emt_network3_csr")
    return rp, ci, cv


class Hierarchy:
    """Exact hierarchical inverse of a symmetric G (hinv_build / hinv_solve / hinv_modify_line)."""

    def __init__(self, row_ptr, col_idx, val, parent, bus_leaf, prec="fp64", rel_tol=1e-9, max_refine=2,
                 max_mod_rank=4, max_nrhs=1, device="cuda", coupling="exact"):
        import torch
        self._lib = load()
        self.device = torch.device(device)
        c = np.ascontiguousarray
        self._rp, self._ci, self._cv = c(row_ptr, np.int32), c(col_idx, np.int32), c(val, np.float64)
        self._parent, self._leaf = c(parent, np.int32), c(bus_leaf, np.int32)
        self.n = len(self._rp) - 1
        self._csr = _CSR(self.n, _ptr(self._rp), _ptr(self._ci), _ptr(self._cv))
        self._tree = _Tree(len(self._parent), _ptr(self._parent), _ptr(self._leaf))
        self._opt = _options(prec, rel_tol, max_refine, max_mod_rank, max_nrhs, coupling=coupling)
        nb = ctypes.c_size_t(0)
        _check(self._lib.hinv_workspace_size(ctypes.byref(self._csr), ctypes.byref(self._tree),
                                             ctypes.byref(self._opt), ctypes.byref(nb)), "hinv_workspace_size")
        self.ws_bytes = nb.value
        self._ws = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p(0)
        with torch.cuda.device(self.device):
            _check(self._lib.hinv_build(ctypes.byref(self._csr), ctypes.byref(self._tree), ctypes.byref(self._opt),
                                        _ptr(self._ws), nb.value, _stream(), ctypes.byref(h)), "hinv_build")
        self._h = h
        _live.add(self)

    @classmethod
    def from_network(cls, net, **kw):
        rp, ci, cv = network_csr(net)
        return cls(rp, ci, cv, net.parent, net.bus_leaf, **kw)

    def solve(self, i, out=None):
        """v = G^{-1} i; i: (n,) or (nrhs, n) float64 tensor on the device."""
        import torch
        x = i.contiguous()
        squeeze = x.dim() == 1
        if squeeze:
            x = x.unsqueeze(0)
        if x.dtype != torch.float64 or x.device.type != "cuda":
            raise ValueError("i must be a float64 device tensor")
        if out is None:
            out = torch.empty_like(x)
        _check(self._lib.hinv_solve(self._h, _ptr(x), _ptr(out), x.shape[0], self.n, _stream()), "hinv_solve")
        return out[0] if squeeze else out

    def solve_gmres(self, i, m=30, max_outer=6, smooth=0, inner_tol=1e-6, rel_tol=1e-12, raise_on_fail=True):
        """hinv_solve_gmres: v = G^{-1} i by GMRES-based refinement with the stored inverse (in its
        storage precision, then `smooth` damped-Jacobi sweeps) as preconditioner.  i: (nrhs, n) float64
        device tensor.  Returns (v, info); info: corrections, inner_iterations, last_update, status."""
        import torch
        x = i.contiguous()
        if x.dim() != 2 or x.dtype != torch.float64 or x.device.type != "cuda":
            raise ValueError("i must be a (nrhs, n) float64 device tensor")
        nb = ctypes.c_size_t(0)
        _check(self._lib.hinv_gmres_workspace_size(self._h, x.shape[0], int(m), ctypes.byref(nb)),
               "hinv_gmres_workspace_size")
        ws = torch.empty(nb.value, dtype=torch.uint8, device=x.device)
        out = torch.empty_like(x)
        inf = _GmresInfo()
        st = self._lib.hinv_solve_gmres(self._h, _ptr(x), _ptr(out), x.shape[0], self.n, int(m), int(max_outer),
                                        int(smooth), float(inner_tol), float(rel_tol), _ptr(ws), nb.value, _stream(),
                                        ctypes.byref(inf))
        info = {k: getattr(inf, k) for k, _ in _GmresInfo._fields_}
        info["status"] = STATUS.get(st, st)
        if raise_on_fail:
            _check(st, "hinv_solve_gmres")
        return out, info

    def solve_noalloc(self, i, out):
        """hinv_solve_noalloc: v = G^{-1} i with the library's static scratch (no allocation in the
        library; `out` must be given).  i, out: (nrhs, n) float64 device tensors."""
        import torch
        if i.dim() != 2 or out.shape != i.shape or i.dtype != torch.float64 or out.dtype != torch.float64 \
                or not i.is_contiguous() or not out.is_contiguous():
            raise ValueError("i and out must be contiguous (nrhs, n) float64 device tensors")
        _check(self._lib.hinv_solve_noalloc(self._h, _ptr(i), _ptr(out), i.shape[0], self.n, _stream()),
               "hinv_solve_noalloc")
        return out

    def modify_line(self, a: int, b: int, delta_g: float) -> None:
        _check(self._lib.hinv_modify_line(self._h, int(a), int(b), float(delta_g), _stream()), "hinv_modify_line")

    def update_line(self, a: int, b: int, delta_g: float) -> dict:
        """G <- G + delta_g (e_a - e_b)(e_a - e_b)^T in the base matrix, with a local FP64 rebuild
        of the stored inverse; returns what was rebuilt."""
        inf = _UpdateInfo()
        _check(self._lib.hinv_update_line(self._h, int(a), int(b), float(delta_g), _stream(), ctypes.byref(inf)),
               "hinv_update_line")
        return {k: getattr(inf, k) for k, _ in _UpdateInfo._fields_}

    def sync_status(self) -> None:
        import torch
        torch.cuda.current_stream().synchronize()
        _check(self._lib.hinv_sync_status(self._h), "hinv_sync_status")

    def info(self) -> dict:
        inf = _Info()
        _check(self._lib.hinv_get_info(self._h, ctypes.byref(inf)), "hinv_get_info")
        return {k: getattr(inf, k) for k, _ in _Info._fields_}

    def close(self) -> None:
        if getattr(self, "_h", None):
            self._lib.hinv_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _case_arrays(n_cases: int, losses: Optional[Sequence[Sequence[Tuple[int, int]]]]):
    ptr = np.zeros(n_cases + 1, np.int32)
    st, br = [], []
    if losses is not None:
        if len(losses) != n_cases:
            raise ValueError("one loss list per case")
        for k, lst in enumerate(losses):
            for (s, b) in lst:
                st.append(int(s))
                br.append(int(b))
            ptr[k + 1] = len(st)
    return ptr, np.asarray(st, np.int32), np.asarray(br, np.int32)


class Chol:
    """Comparison baseline: sparse Cholesky of G, triangular solves on the GPU (chol_* ABI)."""

    def __init__(self, row_ptr, col_idx, val, device="cuda"):
        import torch
        self._lib = load()
        self.device = torch.device(device)
        c = np.ascontiguousarray
        self._rp, self._ci, self._cv = c(row_ptr, np.int32), c(col_idx, np.int32), c(val, np.float64)
        self.n = len(self._rp) - 1
        self._csr = _CSR(self.n, _ptr(self._rp), _ptr(self._ci), _ptr(self._cv))
        nb = ctypes.c_size_t(0)
        _check(self._lib.chol_workspace_size(ctypes.byref(self._csr), ctypes.byref(nb)), "chol_workspace_size")
        self._ws = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p(0)
        with torch.cuda.device(self.device):
            _check(self._lib.chol_create(ctypes.byref(self._csr), _ptr(self._ws), nb.value, _stream(),
                                         ctypes.byref(h)), "chol_create")
        self._h = h
        _live.add(self)

    @classmethod
    def from_network(cls, net, **kw):
        rp, ci, cv = network_csr(net)
        return cls(rp, ci, cv, **kw)

    def solve(self, i, out=None):
        """x = G^{-1} i; i: (n,) or (nrhs, n) float64 device tensor."""
        import torch
        x = i.contiguous()
        squeeze = x.dim() == 1
        if squeeze:
            x = x.unsqueeze(0)
        if x.dtype != torch.float64 or x.device.type != "cuda":
            raise ValueError("i must be a float64 device tensor")
        if out is None:
            out = torch.empty_like(x)
        _check(self._lib.chol_solve(self._h, _ptr(x), _ptr(out), x.shape[0], self.n, _stream()), "chol_solve")
        return out[0] if squeeze else out

    def info(self) -> dict:
        inf = _CholInfo()
        _check(self._lib.chol_get_info(self._h, ctypes.byref(inf)), "chol_get_info")
        return {k: getattr(inf, k) for k, _ in _CholInfo._fields_}

    def close(self) -> None:
        if getattr(self, "_h", None):
            self._lib.chol_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def emt_workspace_bytes(net, n_cases: int = 1, losses=None, prec="fp64", rel_tol=1e-9, max_refine=2,
                        max_mod_rank=2, warm_start=False, kernel_mode="auto") -> int:
    """Device workspace an EMT context of these arguments needs (emt_workspace_size, host only).

    Raises HinvError when the arguments are refused, e.g. a kernel_mode whose engine cannot take the
    network (leaf or LDS limits)."""
    lib = load()
    na = _NetArrays(net)
    ptr, st, br = _case_arrays(int(n_cases), losses)
    cs = _Cases(int(n_cases), _ptr(ptr), _ptr(st), _ptr(br))
    opt = _options(prec, rel_tol, max_refine, max_mod_rank, 1, warm_start, kernel_mode)
    nb = ctypes.c_size_t(0)
    _check(lib.emt_workspace_size(ctypes.byref(na.s), ctypes.byref(na.tree), ctypes.byref(opt), ctypes.byref(cs),
                                  ctypes.byref(nb)), "emt_workspace_size")
    return nb.value


class EMT:
    """EMT time stepping of n_cases cases sharing one network (emt_create / emt_step).

    losses: per case a list of (step, branch) line losses (branch lost from that step on).
    mutual: None for the single-phase network; a float makes it the three-phase network with that
    ratio of mutual to self inductance between a line's phases (emt3_create): vectors then have
    3 n_bus rows (3a + p), losses name lines (all three phases lost), each taking 3 of max_mod_rank.
    shift: three-phase source phase shifts (None: balanced 0, -120, +120 degrees).
    """

    def __init__(self, net, n_cases: int = 1, losses=None, prec="fp64", rel_tol=1e-9, max_refine=2,
                 max_mod_rank=2, warm_start=False, kernel_mode="auto", device="cuda", mutual=None, shift=None):
        import torch
        self._lib = load()
        self.device = torch.device(device)
        self.net = net
        self.phases = 1 if mutual is None else 3
        self.n = self.phases * int(net.n_bus)
        self.n_cases = int(n_cases)
        self._na = _NetArrays(net)
        self._ptr, self._st, self._br = _case_arrays(self.n_cases, losses)
        self._cases = _Cases(self.n_cases, _ptr(self._ptr), _ptr(self._st), _ptr(self._br))
        self._opt = _options(prec, rel_tol, max_refine, max_mod_rank, 1, warm_start, kernel_mode)
        self._shift = None if shift is None else np.ascontiguousarray(shift, np.float64)
        nb = ctypes.c_size_t(0)
        if mutual is None:
            _check(self._lib.emt_workspace_size(ctypes.byref(self._na.s), ctypes.byref(self._na.tree),
                                                ctypes.byref(self._opt), ctypes.byref(self._cases), ctypes.byref(nb)),
                   "emt_workspace_size")
        else:
            _check(self._lib.emt3_workspace_size(ctypes.byref(self._na.s), float(mutual), _ptr(self._shift),
                                                 ctypes.byref(self._na.tree), ctypes.byref(self._opt),
                                                 ctypes.byref(self._cases), ctypes.byref(nb)), "emt3_workspace_size")
        self.ws_bytes = nb.value
        self._ws = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p(0)
        with torch.cuda.device(self.device):
            if mutual is None:
                _check(self._lib.emt_create(ctypes.byref(self._na.s), ctypes.byref(self._na.tree),
                                            ctypes.byref(self._opt), ctypes.byref(self._cases), _ptr(self._ws),
                                            nb.value, _stream(), ctypes.byref(h)), "emt_create")
            else:
                _check(self._lib.emt3_create(ctypes.byref(self._na.s), float(mutual), _ptr(self._shift),
                                             ctypes.byref(self._na.tree), ctypes.byref(self._opt),
                                             ctypes.byref(self._cases), _ptr(self._ws), nb.value, _stream(),
                                             ctypes.byref(h)), "emt3_create")
        self._h = h
        _live.add(self)

    def step(self, n_steps: int, record_v: bool = True, record_b: bool = False, v_out=None, b_out=None):
        """Advance all cases; returns (V, B) of shape (n_steps, n_cases, n_bus) or None."""
        import torch
        V = B = None
        if record_v:
            V = v_out if v_out is not None else torch.empty((n_steps, self.n_cases, self.n), dtype=torch.float64,
                                                            device=self.device)
        if record_b:
            B = b_out if b_out is not None else torch.empty((n_steps, self.n_cases, self.n), dtype=torch.float64,
                                                            device=self.device)
        _check(self._lib.emt_step(self._h, int(n_steps), _ptr(V), _ptr(B), _stream()), "emt_step")
        return V, B

    def lose_line(self, case_idx: int, branch: int) -> None:
        _check(self._lib.emt_lose_line(self._h, int(case_idx), int(branch), _stream()), "emt_lose_line")

    def update_line(self, a: int, b: int, delta_g: float) -> dict:
        """From the next step on, every case's G <- G + delta_g (e_a - e_b)(e_a - e_b)^T (b = -1:
        a to ground): a memoryless fault conductance switched on, or off with its negative.
        Returns what the local rebuild of the stored inverse touched."""
        inf = _UpdateInfo()
        _check(self._lib.emt_update_line(self._h, int(a), int(b), float(delta_g), _stream(), ctypes.byref(inf)),
               "emt_update_line")
        return {k: getattr(inf, k) for k, _ in _UpdateInfo._fields_}

    def sync_status(self) -> None:
        """Raise HinvError if a device-side failure (barrier time-out, unmapped change
        endpoint, non-finite value, refinement above rel_tol) happened since the last call."""
        import torch
        torch.cuda.current_stream().synchronize()
        _check(self._lib.emt_sync_status(self._h), "emt_sync_status")

    @property
    def next_step(self) -> int:
        s = ctypes.c_int64(0)
        _check(self._lib.emt_get_step(self._h, ctypes.byref(s)), "emt_get_step")
        return s.value

    def save_state(self) -> np.ndarray:
        """Checkpoint of the time loop (emt_save_state): a uint8 array that load_state takes."""
        nb = ctypes.c_size_t(0)
        _check(self._lib.emt_state_size(self._h, ctypes.byref(nb)), "emt_state_size")
        buf = np.zeros(nb.value, np.uint8)
        _check(self._lib.emt_save_state(self._h, _ptr(buf), nb.value, _stream()), "emt_save_state")
        return buf

    def load_state(self, buf) -> None:
        """Resume from a checkpoint of a handle on the same network (emt_load_state)."""
        buf = np.ascontiguousarray(buf, np.uint8)
        _check(self._lib.emt_load_state(self._h, _ptr(buf), buf.nbytes, _stream()), "emt_load_state")

    def stats(self) -> Tuple[int, float]:
        import torch
        torch.cuda.current_stream().synchronize()
        a, r = ctypes.c_int64(0), ctypes.c_double(0)
        _check(self._lib.emt_get_stats(self._h, ctypes.byref(a), ctypes.byref(r)), "emt_get_stats")
        return a.value, r.value

    def set_step_clock(self, clock=None) -> None:
        """clock: int64 device tensor receiving the GPU wall clock after each step (or None)."""
        cap = 0 if clock is None else clock.numel()
        _check(self._lib.emt_set_step_clock(self._h, _ptr(clock), cap), "emt_set_step_clock")
        self._clock = clock

    def close(self) -> None:
        if getattr(self, "_h", None):
            self._lib.emt_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Serve:
    """Pool of single-case EMT handles advanced by one launch per step call (serve_*)."""

    def __init__(self, max_slots: int, prec="fp32", warm_start=True, max_refine=2, rel_tol=1e-9, device="cuda"):
        import torch
        self._lib = load()
        self.device = torch.device(device)
        self.prec, self.warm_start, self.max_refine, self.rel_tol = prec, warm_start, max_refine, rel_tol
        self._opt = _options(prec, rel_tol, max_refine, 0, 1, warm_start, "auto")
        nb = ctypes.c_size_t(0)
        _check(self._lib.serve_workspace_size(int(max_slots), ctypes.byref(nb)), "serve_workspace_size")
        self._ws = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p(0)
        _check(self._lib.serve_create(ctypes.byref(self._opt), int(max_slots), _ptr(self._ws), nb.value,
                                      ctypes.byref(h)), "serve_create")
        self._h = h
        _live.add(self)
        self._cases = {}

    def case_bytes(self, net, losses=None, max_mod_rank=2) -> int:
        """Device workspace new_case would take for this case (host-only size query, builds nothing)."""
        return emt_workspace_bytes(net, 1, [losses or []], prec=self.prec, rel_tol=self.rel_tol,
                                   max_refine=self.max_refine, max_mod_rank=max_mod_rank,
                                   warm_start=self.warm_start)

    def new_case(self, net, losses=None, max_mod_rank=2) -> "EMT":
        """An EMT handle with the pool's precision settings (one case)."""
        return EMT(net, 1, losses=[losses or []], prec=self.prec, rel_tol=self.rel_tol, max_refine=self.max_refine,
                   max_mod_rank=max_mod_rank, warm_start=self.warm_start, device=self.device)

    def attach(self, emt: "EMT", record_steps: int = 0):
        """Attach a case; returns (slot id, record tensor or None)."""
        import torch
        rec = None
        if record_steps:
            rec = torch.empty((record_steps, emt.n), dtype=torch.float64, device=self.device)
        sid = ctypes.c_int32(0)
        _check(self._lib.serve_attach(self._h, emt._h, _ptr(rec), int(record_steps), _stream(), ctypes.byref(sid)),
               "serve_attach")
        self._cases[sid.value] = (emt, rec)
        return sid.value, rec

    def detach(self, slot_id: int) -> None:
        _check(self._lib.serve_detach(self._h, int(slot_id), _stream()), "serve_detach")
        self._cases.pop(slot_id, None)

    def step(self, n_steps: int) -> None:
        _check(self._lib.serve_step(self._h, int(n_steps), _stream()), "serve_step")

    def synchronize(self) -> None:
        import torch
        torch.cuda.current_stream().synchronize()

    @property
    def active(self) -> int:
        v = ctypes.c_int32(0)
        _check(self._lib.serve_active(self._h, ctypes.byref(v)), "serve_active")
        return v.value

    def close(self) -> None:
        if getattr(self, "_h", None):
            self._lib.serve_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
