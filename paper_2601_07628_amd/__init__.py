"""Python binding of libdpdlp (the single-GPU restarted Halpern PDHG solver).

Argument marshalling only: every step of the method runs in the library's
HIP kernels on the GPU.  The functions keep the C names of ``include/dpdlp.h``;
``Problem`` is a small convenience wrapper over them.  PyTorch is used only
for device memory and streams, and only when the caller passes tensors.

Loading fails loudly (ImportError) when ``libdpdlp.so`` has not been built;
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdpdlp.so")

OK = 0
E_INVALID_ARG, E_BAD_CSR, E_BAD_BOUNDS, E_HIP, E_OOM, E_NOT_SUPPORTED = -1, -2, -3, -4, -5, -6
RUNNING, CONVERGED, ITER_LIMIT, TIME_LIMIT, NUMERICAL = 0, 1, 2, 3, 4
MEM_HOST, MEM_DEVICE = 0, 1
FP64, FP32_MIXED = 0, 1
KERNEL_CLASSES = ("primal", "dual", "check_csr", "check_csc", "control")


class DpdlpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"dpdlp error {code}: {msg}")
        self.code = code


class CsrLP(C.Structure):
    _fields_ = [("m", C.c_int32), ("n", C.c_int32), ("row_ptr", C.c_void_p),
                ("col_idx", C.c_void_p), ("val", C.c_void_p), ("c", C.c_void_p),
                ("con_lo", C.c_void_p), ("con_hi", C.c_void_p),
                ("var_lo", C.c_void_p), ("var_hi", C.c_void_p),
                ("mem_kind", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("eps", C.c_double), ("max_iters", C.c_int64),
                ("time_limit", C.c_double), ("check_period", C.c_int32),
                ("ruiz_iters", C.c_int32), ("gamma", C.c_double),
                ("beta_suf", C.c_double), ("beta_nec", C.c_double),
                ("beta_art", C.c_double), ("kp", C.c_double), ("ki", C.c_double),
                ("kd", C.c_double), ("eta", C.c_double), ("omega0", C.c_double),
                ("eta_safety", C.c_double), ("power_max_iters", C.c_int32),
                ("use_pc", C.c_int32), ("power_tol", C.c_double),
                ("pc_alpha", C.c_double), ("perm_block", C.c_int32),
                ("tile_nnz", C.c_int32), ("perm_seed", C.c_uint64),
                ("precision", C.c_int32), ("xcd_remap", C.c_int32),
                ("fp32_switch_tol", C.c_double), ("fp32_stall_checks", C.c_int32),
                ("gather_slices", C.c_int32), ("use_graphs", C.c_int32),
                ("perm_order", C.c_int32), ("gather_sort", C.c_int32), ("fp32_diverge", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("restarts", C.c_int32),
                ("iters", C.c_int64), ("fp32_iters", C.c_int64),
                ("r_primal", C.c_double), ("r_dual", C.c_double),
                ("r_gap", C.c_double), ("obj_primal", C.c_double),
                ("obj_dual", C.c_double), ("omega", C.c_double),
                ("eta", C.c_double), ("sigma_max", C.c_double),
                ("setup_seconds", C.c_double), ("solve_seconds", C.c_double),
                ("power_iters", C.c_int32), ("n_checks", C.c_int32),
                ("slices_primal", C.c_int32), ("slices_dual", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class State(C.Structure):
    _fields_ = [("omega", C.c_double), ("r0", C.c_double), ("r_prev", C.c_double),
                ("pid_int", C.c_double), ("pid_prev", C.c_double),
                ("k", C.c_int64), ("t", C.c_int64), ("pid_started", C.c_int32),
                ("restarts", C.c_int32), ("status", C.c_int32),
                ("n_checks", C.c_int32), ("r_primal", C.c_double),
                ("r_dual", C.c_double), ("r_gap", C.c_double),
                ("obj_primal", C.c_double), ("obj_dual", C.c_double),
                ("r_fixed_point", C.c_double)]


class LogRec(C.Structure):
    _fields_ = [("t", C.c_int64), ("k", C.c_int64), ("r", C.c_double),
                ("r0", C.c_double), ("r_primal", C.c_double),
                ("r_dual", C.c_double), ("r_gap", C.c_double),
                ("omega", C.c_double), ("restart", C.c_int32), ("pad", C.c_int32)]


class CostParams(C.Structure):
    _fields_ = [("b_mem", C.c_double), ("b_net", C.c_double), ("beta_sync", C.c_double),
                ("n_hop", C.c_double), ("c_spmv", C.c_double), ("c_vec", C.c_double),
                ("c_net", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# Every symbol include/dpdlp.h declares (checked by the CPU test suite).
EXPORTS = (
    "dpdlp_params_default", "dpdlp_problem_create", "dpdlp_problem_destroy",
    "dpdlp_problem_update_data", "dpdlp_set_params",
    "dpdlp_init", "dpdlp_iterate", "dpdlp_solve", "dpdlp_get_result",
    "dpdlp_state_export", "dpdlp_state_import", "dpdlp_get_log", "dpdlp_spmv",
    "dpdlp_kkt", "dpdlp_kkt_noalloc", "dpdlp_get_scaling", "dpdlp_time_kernel",
    "dpdlp_profile_enable", "dpdlp_get_profile", "dpdlp_validate",
    "dpdlp_block_permutation", "dpdlp_build_tiles", "dpdlp_row_bounds", "dpdlp_status_string",
    "dpdlp_last_error", "dpdlp_gnn_create", "dpdlp_gnn_destroy", "dpdlp_gnn_num_params",
    "dpdlp_gnn_set_params", "dpdlp_gnn_get_params", "dpdlp_gnn_set_reference",
    "dpdlp_gnn_set_instance", "dpdlp_gnn_forward", "dpdlp_gnn_backward",
    "dpdlp_gnn_adam_step", "dpdlp_gnn_gemm_test", "dpdlp_cost_params_default",
    "dpdlp_cost_step", "dpdlp_grid_select", "dpdlp_auto_devices", "dpdlp_set_objective_diag",
    "dpdlp_time_gather",
)


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with "
            "`python paper_2601_07628_amd/build.py` (there is no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, u64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
    sig = {
        "dpdlp_params_default": ([C.POINTER(Params)], None),
        "dpdlp_problem_create": ([C.POINTER(CsrLP), C.POINTER(Params), vp, C.POINTER(vp)], C.c_int),
        "dpdlp_problem_destroy": ([vp], C.c_int),
        "dpdlp_problem_update_data": ([vp, vp, vp, vp, vp, vp, i32, vp], C.c_int),
        "dpdlp_init": ([vp, vp, vp, i32, vp], C.c_int),
        "dpdlp_set_params": ([vp, C.POINTER(Params)], C.c_int),
        "dpdlp_iterate": ([vp, i64, vp], C.c_int),
        "dpdlp_solve": ([vp, vp, vp, vp, vp, i32, C.POINTER(Result), vp], C.c_int),
        "dpdlp_get_result": ([vp, vp, vp, i32, C.POINTER(Result), vp], C.c_int),
        "dpdlp_state_export": ([vp, C.POINTER(State), vp, vp, vp, vp, vp, vp, i32, vp], C.c_int),
        "dpdlp_state_import": ([vp, C.POINTER(State), vp, vp, vp, vp, vp, vp, i32, vp], C.c_int),
        "dpdlp_get_log": ([vp, vp, i32, C.POINTER(i32)], C.c_int),
        "dpdlp_spmv": ([vp, i32, vp, vp, vp], C.c_int),
        "dpdlp_kkt": ([vp, vp, vp, dbl, i32, vp, vp], C.c_int),
        "dpdlp_kkt_noalloc": ([C.POINTER(CsrLP), vp, vp, vp, vp, vp, vp, vp, dbl, vp, vp],
                              C.c_int),
        "dpdlp_get_scaling": ([vp, vp, vp, vp, vp, vp, vp], C.c_int),
        "dpdlp_time_kernel": ([vp, i32, i32, vp, vp, vp], C.c_int),
        "dpdlp_time_gather": ([i64, i32, i64, i32, i32, u64, vp, vp, vp], C.c_int),
        "dpdlp_profile_enable": ([vp, i32], C.c_int),
        "dpdlp_get_profile": ([vp, vp, vp, vp], C.c_int),
        "dpdlp_validate": ([C.POINTER(CsrLP)], C.c_int),
        "dpdlp_block_permutation": ([i32, i32, u64, vp], C.c_int),
        "dpdlp_row_bounds": ([i32, vp, vp, vp, vp], C.c_int),
        "dpdlp_build_tiles": ([vp, i32, i32, vp, C.POINTER(i32)], C.c_int),
        "dpdlp_status_string": ([i32], C.c_char_p),
        "dpdlp_gnn_create": ([vp, i32, vp, C.POINTER(vp)], C.c_int),
        "dpdlp_gnn_destroy": ([vp], C.c_int),
        "dpdlp_gnn_num_params": ([vp], i64),
        "dpdlp_gnn_set_params": ([vp, vp, i64, vp], C.c_int),
        "dpdlp_gnn_get_params": ([vp, vp, vp, i64, vp], C.c_int),
        "dpdlp_gnn_set_reference": ([vp, vp, vp, vp, vp, i32, vp], C.c_int),
        "dpdlp_gnn_set_instance": ([vp, vp, vp, vp, i32, vp], C.c_int),
        "dpdlp_gnn_forward": ([vp, vp, vp, i32, vp], C.c_int),
        "dpdlp_gnn_backward": ([vp, vp, vp, i32, vp, vp], C.c_int),
        "dpdlp_gnn_adam_step": ([vp, dbl, dbl, dbl, dbl, vp], C.c_int),
        "dpdlp_gnn_gemm_test": ([vp, C.c_long, C.c_long, vp, C.c_long, C.c_long, vp, C.c_long,
                                 i32, i32, i32, vp], C.c_int),
        "dpdlp_last_error": ([], C.c_char_p),
        "dpdlp_set_objective_diag": ([vp, vp, i32, vp], C.c_int),
        "dpdlp_cost_params_default": ([C.POINTER(CostParams)], None),
        "dpdlp_cost_step": ([i64, i64, i64, i32, i32, C.POINTER(CostParams), vp], C.c_int),
        "dpdlp_grid_select": ([i64, i64, i32, C.POINTER(i32), C.POINTER(i32)], C.c_int),
        "dpdlp_auto_devices": ([i64, i64, i64, vp, i32, C.POINTER(CostParams), C.POINTER(i32),
                                C.POINTER(i32), C.POINTER(i32), C.POINTER(dbl)], C.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    return L


_lib = _load()


def lib():
    return _lib


def _check(rc):
    if rc != OK:
        raise DpdlpError(rc, _lib.dpdlp_last_error().decode())
    return rc


def _ptr(a):
    """Plain address of a numpy array or torch tensor (None -> NULL)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()                  # torch.Tensor


def _stream(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream            # torch.cuda.Stream


# ---- same-name functions (marshalling only) --------------------------------
def dpdlp_params_default() -> Params:
    p = Params()
    _lib.dpdlp_params_default(C.byref(p))
    return p


def dpdlp_status_string(status: int) -> str:
    return _lib.dpdlp_status_string(status).decode()


def dpdlp_last_error() -> str:
    return _lib.dpdlp_last_error().decode()


def _csr_struct(arrays, m, n, mem_kind):
    return CsrLP(m, n, *[_ptr(arrays[k]) for k in (
        "row_ptr", "col_idx", "val", "c", "con_lo", "con_hi", "var_lo", "var_hi")],
        mem_kind)


def host_arrays(lp) -> dict:
    """Contiguous host arrays (int32 / float64) of an LP-like object."""
    return dict(
        row_ptr=np.ascontiguousarray(lp.row_ptr, np.int32),
        col_idx=np.ascontiguousarray(lp.col_idx, np.int32),
        val=np.ascontiguousarray(lp.val, np.float64),
        c=np.ascontiguousarray(lp.c, np.float64),
        con_lo=np.ascontiguousarray(lp.con_lo, np.float64),
        con_hi=np.ascontiguousarray(lp.con_hi, np.float64),
        var_lo=np.ascontiguousarray(lp.var_lo, np.float64),
        var_hi=np.ascontiguousarray(lp.var_hi, np.float64))


def dpdlp_validate(lp) -> int:
    """Host-side validation (no GPU needed); returns the C return code."""
    a = host_arrays(lp)
    s = _csr_struct(a, int(lp.m), int(lp.n), MEM_HOST)
    return int(_lib.dpdlp_validate(C.byref(s)))


def dpdlp_block_permutation(count: int, block: int, seed: int) -> np.ndarray:
    perm = np.zeros(max(count, 1), np.int32)
    _check(_lib.dpdlp_block_permutation(count, block, seed, _ptr(perm)))
    return perm[:count]


def dpdlp_row_bounds(b, row_type):
    """(con_lo, con_hi) for rows given as b and types 0 '=', 1 '>=', 2 '<='."""
    b = np.ascontiguousarray(b, np.float64)
    t = np.ascontiguousarray(row_type, np.int32)
    if b.shape != t.shape:
        raise ValueError("b and row_type differ in length")
    lo, hi = np.empty_like(b), np.empty_like(b)
    _check(_lib.dpdlp_row_bounds(b.size, _ptr(b), _ptr(t), _ptr(lo), _ptr(hi)))
    return lo, hi


def dpdlp_build_tiles(seg_ptr, tile_nnz: int = 0) -> np.ndarray:
    """Nonzero-aware tiles; rows of {seg_begin, seg_end, nnz_begin, nnz_end,
    width_log2, piece, npieces, 0}."""
    sp_ = np.ascontiguousarray(seg_ptr, np.int32)
    cnt = C.c_int32(0)
    _check(_lib.dpdlp_build_tiles(_ptr(sp_), sp_.size - 1, tile_nnz, None, C.byref(cnt)))
    out = np.zeros((max(cnt.value, 1), 8), np.int32)
    cnt2 = C.c_int32(cnt.value)
    _check(_lib.dpdlp_build_tiles(_ptr(sp_), sp_.size - 1, tile_nnz, _ptr(out), C.byref(cnt2)))
    return out[: cnt.value]


def dpdlp_cost_params_default(**kw) -> CostParams:
    p = CostParams()
    _lib.dpdlp_cost_params_default(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def dpdlp_cost_step(m: int, n: int, nnz: int, R: int, C_: int,
                    params: Optional[CostParams] = None) -> dict:
    """Modelled seconds per iteration on an R x C grid, by term."""
    p = params if params is not None else dpdlp_cost_params_default()
    out = np.zeros(5)
    _check(_lib.dpdlp_cost_step(m, n, nnz, R, C_, C.byref(p), _ptr(out)))
    return dict(spmv=float(out[0]), vec=float(out[1]), net=float(out[2]),
                sync=float(out[3]), total=float(out[4]))


def dpdlp_grid_select(m: int, n: int, ndev: int):
    r, c = C.c_int32(0), C.c_int32(0)
    _check(_lib.dpdlp_grid_select(m, n, ndev, C.byref(r), C.byref(c)))
    return r.value, c.value


def dpdlp_auto_devices(m: int, n: int, nnz: int, counts=(1, 2, 4, 8),
                       params: Optional[CostParams] = None) -> dict:
    p = params if params is not None else dpdlp_cost_params_default()
    cnt = np.ascontiguousarray(counts, np.int32)
    nd, r, c, t = C.c_int32(0), C.c_int32(0), C.c_int32(0), C.c_double(0.0)
    _check(_lib.dpdlp_auto_devices(m, n, nnz, _ptr(cnt), cnt.size, C.byref(p), C.byref(nd),
                                   C.byref(r), C.byref(c), C.byref(t)))
    return dict(ndev=nd.value, R=r.value, C=c.value, t_step=t.value)


def dpdlp_time_gather(n_vec: int, slices: int, n_gathers: int, precision: int = 0,
                      reps: int = 20, seed: int = 1, stream=None) -> dict:
    """Random-gather rate probe (the sliced steps' gather pattern): mean ms
    per pass of n_gathers gathers and the gathers per second."""
    ms, rate = C.c_double(), C.c_double()
    _check(_lib.dpdlp_time_gather(n_vec, slices, n_gathers, precision, reps, seed,
                                  _stream(stream), C.byref(ms), C.byref(rate)))
    return dict(avg_ms=ms.value, gathers_per_s=rate.value)


def dpdlp_problem_create(lp, params: Optional[Params] = None, stream=None,
                         device_arrays: Optional[dict] = None):
    """Create a problem handle from an LP-like object (host arrays) or from a
    dict of device tensors (``device_arrays``, same keys as host_arrays)."""
    if device_arrays is not None:
        keep = device_arrays
        s = _csr_struct(keep, int(lp.m), int(lp.n), MEM_DEVICE)
    else:
        keep = host_arrays(lp)
        s = _csr_struct(keep, int(lp.m), int(lp.n), MEM_HOST)
    h = C.c_void_p()
    prm = params if params is not None else dpdlp_params_default()
    _check(_lib.dpdlp_problem_create(C.byref(s), C.byref(prm), _stream(stream), C.byref(h)))
    return h


def dpdlp_kkt_noalloc(m: int, n: int, csr: dict, csc: dict, x, y, tau: float, out5,
                      col_scale=None, q=None, stream=None):
    """KKT at (x, y) of an LP given as device tensors, without allocation:
    ``csr`` has the host_arrays keys, ``csc`` the keys col_ptr, row_idx, val;
    x, y, col_scale, q and out5 (5 doubles) are device tensors."""
    s = _csr_struct(csr, int(m), int(n), MEM_DEVICE)
    _check(_lib.dpdlp_kkt_noalloc(C.byref(s), _ptr(csc["col_ptr"]), _ptr(csc["row_idx"]),
                                  _ptr(csc["val"]), _ptr(col_scale), _ptr(q), _ptr(x), _ptr(y),
                                  float(tau), _ptr(out5), _stream(stream)))


def dpdlp_problem_destroy(h):
    return _check(_lib.dpdlp_problem_destroy(h))


# ---- convenience wrapper ------------------------------------------------------
class Problem:
    """A prepared problem on the current GPU (owns the library handle).

    An instance that carries ``lp.q`` (diag(Q), Sec. 6) is set up as a
    diagonal QP, unless ``q`` is given (an array, or False for the LP)."""

    def __init__(self, lp, params: Optional[Params] = None, stream=None, q=None, **kw):
        prm = params if params is not None else dpdlp_params_default()
        for k, v in kw.items():
            if not hasattr(prm, k):
                raise AttributeError(f"no parameter {k}")
            setattr(prm, k, v)
        self.params = prm
        self.m, self.n = int(lp.m), int(lp.n)
        self.stream = stream
        self.h = dpdlp_problem_create(lp, prm, stream)
        if q is None:
            q = getattr(lp, "q", None)
        if q is not None and q is not False:
            self.set_objective_diag(q)

    def set_objective_diag(self, q):
        """diag(Q) of a QP objective x^T Q x / 2 (host array), or None for the LP."""
        if q is None:
            _check(_lib.dpdlp_set_objective_diag(self.h, None, MEM_HOST, self._s))
            return
        qa = np.ascontiguousarray(q, np.float64)
        if qa.shape != (self.n,):
            raise ValueError("q must have length n")
        _check(_lib.dpdlp_set_objective_diag(self.h, _ptr(qa), MEM_HOST, self._s))

    def close(self):
        if getattr(self, "h", None) is not None:
            _lib.dpdlp_problem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def _s(self):
        return _stream(self.stream)

    def set_params(self, **kw):
        """Change run-time parameters (eps, max_iters, time_limit, ...)."""
        for k, v in kw.items():
            if not hasattr(self.params, k):
                raise AttributeError(f"no parameter {k}")
            setattr(self.params, k, v)
        _check(_lib.dpdlp_set_params(self.h, C.byref(self.params)))

    def update_data(self, c=None, con_lo=None, con_hi=None, var_lo=None, var_hi=None):
        """Another member of the same family: new objective / bounds, same A."""
        a = [None if v is None else np.ascontiguousarray(v, np.float64)
             for v in (c, con_lo, con_hi, var_lo, var_hi)]
        _check(_lib.dpdlp_problem_update_data(self.h, *[_ptr(v) for v in a], MEM_HOST, self._s))

    def init(self, x0=None, y0=None):
        x0 = None if x0 is None else np.ascontiguousarray(x0, np.float64)
        y0 = None if y0 is None else np.ascontiguousarray(y0, np.float64)
        _check(_lib.dpdlp_init(self.h, _ptr(x0), _ptr(y0), MEM_HOST, self._s))

    def iterate(self, n_iters: int):
        _check(_lib.dpdlp_iterate(self.h, int(n_iters), self._s))

    def result(self, want_xy: bool = True) -> dict:
        r = Result()
        x = np.zeros(self.n) if want_xy else None
        y = np.zeros(self.m) if want_xy else None
        _check(_lib.dpdlp_get_result(self.h, _ptr(x), _ptr(y), MEM_HOST, C.byref(r), self._s))
        d = r.as_dict()
        d["x"], d["y"] = x, y
        return d

    def solve(self, x0=None, y0=None) -> dict:
        r = Result()
        x, y = np.zeros(self.n), np.zeros(self.m)
        x0 = None if x0 is None else np.ascontiguousarray(x0, np.float64)
        y0 = None if y0 is None else np.ascontiguousarray(y0, np.float64)
        _check(_lib.dpdlp_solve(self.h, _ptr(x0), _ptr(y0), _ptr(x), _ptr(y), MEM_HOST,
                                C.byref(r), self._s))
        d = r.as_dict()
        d["x"], d["y"] = x, y
        return d

    def state(self) -> dict:
        st = State()
        arrs = {k: np.zeros(self.n if k.startswith("x") else self.m)
                for k in ("x", "y", "xa", "ya", "xh", "yh")}
        _check(_lib.dpdlp_state_export(self.h, C.byref(st), *[_ptr(arrs[k]) for k in (
            "x", "y", "xa", "ya", "xh", "yh")], MEM_HOST, self._s))
        arrs["scalars"] = {k: getattr(st, k) for k, _ in st._fields_}
        arrs["_state"] = st
        return arrs

    def load_state(self, s: dict):
        st = s["_state"]
        _check(_lib.dpdlp_state_import(self.h, C.byref(st), *[
            _ptr(np.ascontiguousarray(s[k], np.float64)) for k in (
                "x", "y", "xa", "ya", "xh", "yh")], MEM_HOST, self._s))

    def log(self) -> list:
        cnt = C.c_int32(0)
        _check(_lib.dpdlp_get_log(self.h, None, 0, C.byref(cnt)))
        recs = (LogRec * max(cnt.value, 1))()
        _check(_lib.dpdlp_get_log(self.h, C.cast(recs, C.c_void_p), cnt.value, C.byref(cnt)))
        return [dict(t=r.t, k=r.k, r=r.r, r0=r.r0, r_primal=r.r_primal, r_dual=r.r_dual,
                     r_gap=r.r_gap, omega=r.omega, restart=r.restart)
                for r in (recs[i] for i in range(cnt.value))]

    def spmv(self, vec, transpose=False):
        """A~ v or A~^T v on device tensors (torch), original order."""
        import torch
        out = torch.empty(self.n if transpose else self.m, dtype=torch.float64,
                          device=vec.device)
        _check(_lib.dpdlp_spmv(self.h, int(transpose), _ptr(vec), _ptr(out), self._s))
        return out

    def kkt(self, x=None, y=None, tau: float = 0.0):
        """KKT triple + objectives at (x, y), or at the current start point."""
        out = np.zeros(5)
        xp = None if x is None else np.ascontiguousarray(x, np.float64)
        yp = None if y is None else np.ascontiguousarray(y, np.float64)
        _check(_lib.dpdlp_kkt(self.h, _ptr(xp), _ptr(yp), float(tau), MEM_HOST, _ptr(out),
                              self._s))
        return out

    def scaling(self):
        dr, dc = np.zeros(self.m), np.zeros(self.n)
        eta, smax, w0 = C.c_double(), C.c_double(), C.c_double()
        _check(_lib.dpdlp_get_scaling(self.h, _ptr(dr), _ptr(dc), C.byref(eta),
                                      C.byref(smax), C.byref(w0), self._s))
        return dict(dr=dr, dc=dc, eta=eta.value, sigma_max=smax.value, omega0=w0.value)

    def time_kernel(self, which: int, reps: int = 20):
        ms, by = C.c_double(), C.c_double()
        _check(_lib.dpdlp_time_kernel(self.h, which, reps, self._s, C.byref(ms), C.byref(by)))
        return ms.value, by.value

    def profile_enable(self, on: bool = True):
        _check(_lib.dpdlp_profile_enable(self.h, int(on)))

    def profile(self) -> dict:
        ms = np.zeros(8)
        n = np.zeros(8, np.int64)
        b = np.zeros(8)
        _check(_lib.dpdlp_get_profile(self.h, _ptr(ms), _ptr(n), _ptr(b)))
        return {name: dict(total_ms=float(ms[i]), launches=int(n[i]),
                           bytes_per_launch=float(b[i]))
                for i, name in enumerate(KERNEL_CLASSES)}


# ---- learned warm start -------------------------------------------------------
def row_b(con_lo, con_hi):
    """Per-row right-hand side used by the network's row features: the finite
    lower bound, else the finite upper bound, else 0."""
    lo = np.asarray(con_lo, np.float64)
    hi = np.asarray(con_hi, np.float64)
    return np.where(np.isfinite(lo), lo, np.where(np.isfinite(hi), hi, 0.0))


class WarmStartNet:
    """The warm-start network on a prepared problem's graph (C ABI wrapper)."""

    def __init__(self, problem: Problem, layers: int = 3, stream=None):
        self.problem = problem
        self.stream = stream
        h = C.c_void_p()
        _check(_lib.dpdlp_gnn_create(problem.h, layers, _stream(stream), C.byref(h)))
        self.h = h
        self.layers = layers
        self.n_params = int(_lib.dpdlp_gnn_num_params(h))

    def close(self):
        if getattr(self, "h", None) is not None:
            _lib.dpdlp_gnn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def _s(self):
        return _stream(self.stream)

    def set_params(self, p):
        p = np.ascontiguousarray(p, np.float32)
        _check(_lib.dpdlp_gnn_set_params(self.h, _ptr(p), p.size, self._s))

    def params(self, grads=False):
        p = np.zeros(self.n_params, np.float32)
        g = np.zeros(self.n_params, np.float32) if grads else None
        _check(_lib.dpdlp_gnn_get_params(self.h, _ptr(p), _ptr(g), self.n_params, self._s))
        return (p, g) if grads else p

    def set_reference(self, c_ref, b_ref, x_ref, y_ref):
        a = [np.ascontiguousarray(v, np.float64) for v in (c_ref, b_ref, x_ref, y_ref)]
        _check(_lib.dpdlp_gnn_set_reference(self.h, *[_ptr(v) for v in a], MEM_HOST, self._s))

    def set_instance(self, c, con_lo, con_hi):
        a = [np.ascontiguousarray(v, np.float64) for v in (c, con_lo, con_hi)]
        _check(_lib.dpdlp_gnn_set_instance(self.h, *[_ptr(v) for v in a], MEM_HOST, self._s))

    def forward(self):
        x = np.zeros(self.problem.n)
        y = np.zeros(self.problem.m)
        _check(_lib.dpdlp_gnn_forward(self.h, _ptr(x), _ptr(y), MEM_HOST, self._s))
        return x, y

    def backward(self, x_target, y_target):
        loss = np.zeros(2)
        xt = np.ascontiguousarray(x_target, np.float64)
        yt = np.ascontiguousarray(y_target, np.float64)
        _check(_lib.dpdlp_gnn_backward(self.h, _ptr(xt), _ptr(yt), MEM_HOST, _ptr(loss), self._s))
        return loss

    def adam_step(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        _check(_lib.dpdlp_gnn_adam_step(self.h, lr, beta1, beta2, eps, self._s))


def dpdlp_gnn_gemm_test(A, a_rs, a_cs, B, b_rs, b_cs, M, Nc, K, stream=None):
    """Run the MFMA GEMM kernel on device tensors (BF16 bit patterns as int16)."""
    import torch
    Cout = torch.zeros((M, Nc), dtype=torch.float32, device=A.device)
    _check(_lib.dpdlp_gnn_gemm_test(_ptr(A), a_rs, a_cs, _ptr(B), b_rs, b_cs, _ptr(Cout), Nc,
                                    M, Nc, K, _stream(stream)))
    return Cout
