"""ctypes shim over the plain-C FP64 PDHG oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: the correctness oracle for the GPU library.  Only the
tests, the smoke check and the benchmark's CPU-baseline leg use it; the GPU
library never imports or calls it.

Each function names the passage of the D-PDLP paper (arXiv 2601.07628) it
follows; ``oracle.c`` holds the arithmetic.  Parity status of each part is
listed in the test suite (every part is pinned by a test that does not reuse
the oracle's own formulas).
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (plain FP64, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-shared", "-fPIC", "-std=c11", "-Wall", "-o", _LIB + ".tmp",
               _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _LP(C.Structure):
    _fields_ = [("m", C.c_int32), ("n", C.c_int32),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p),
                ("val", C.c_void_p), ("c", C.c_void_p), ("con_lo", C.c_void_p),
                ("con_hi", C.c_void_p), ("var_lo", C.c_void_p),
                ("var_hi", C.c_void_p)]


class _Params(C.Structure):
    _fields_ = [("eps", C.c_double), ("max_iters", C.c_int64),
                ("check_period", C.c_int32), ("ruiz_iters", C.c_int32),
                ("gamma", C.c_double), ("beta_suf", C.c_double),
                ("beta_nec", C.c_double), ("beta_art", C.c_double),
                ("kp", C.c_double), ("ki", C.c_double), ("kd", C.c_double),
                ("eta", C.c_double), ("omega0", C.c_double),
                ("eta_safety", C.c_double), ("power_max_iters", C.c_int32),
                ("use_pc", C.c_int32), ("power_tol", C.c_double),
                ("pc_alpha", C.c_double)]


class State(C.Structure):
    _fields_ = [("omega", C.c_double), ("r0", C.c_double), ("r_prev", C.c_double),
                ("pid_int", C.c_double), ("pid_prev", C.c_double),
                ("k", C.c_int64), ("t", C.c_int64),
                ("pid_started", C.c_int32), ("restarts", C.c_int32),
                ("status", C.c_int32), ("n_checks", C.c_int32),
                ("r_primal", C.c_double), ("r_dual", C.c_double),
                ("r_gap", C.c_double), ("obj_p", C.c_double),
                ("obj_d", C.c_double), ("kkt_r", C.c_double)]


class LogRec(C.Structure):
    _fields_ = [("t", C.c_int64), ("k", C.c_int64), ("r", C.c_double),
                ("r0", C.c_double), ("r_primal", C.c_double),
                ("r_dual", C.c_double), ("r_gap", C.c_double),
                ("omega", C.c_double), ("restart", C.c_int32),
                ("pad", C.c_int32)]


@dataclasses.dataclass
class Params:
    """Solver parameters (names follow the paper where it names them)."""
    eps: float = 1e-8
    max_iters: int = 100_000
    check_period: int = 64          # K, "every K iterations" (App. D)
    ruiz_iters: int = 10
    gamma: float = 1.0              # reflection (App. A / B.1)
    beta_suf: float = 0.2           # App. B.2
    beta_nec: float = 0.8
    beta_art: float = 0.36
    kp: float = 0.99                # App. B.3 PID gains
    ki: float = 0.01
    kd: float = 0.0
    eta: float = 0.0                # 0: 0.998 / sigma_max(A~) by power iteration
    omega0: float = 0.0             # 0: ||c~|| / ||b~||
    eta_safety: float = 0.998
    power_max_iters: int = 5000
    use_pc: int = 1
    power_tol: float = 1e-6
    pc_alpha: float = 1.0

    def _c(self) -> _Params:
        return _Params(**dataclasses.asdict(self))


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.ora_prepare.argtypes = [C.POINTER(_LP), C.POINTER(_Params), C.POINTER(vp)]
        L.ora_prepare.restype = C.c_int
        L.ora_free.argtypes = [vp]
        L.ora_info.argtypes = [vp, vp, vp]
        L.ora_get_scaled.argtypes = [vp] * 10
        L.ora_spmv.argtypes = [vp, i32, vp, vp]
        L.ora_sigma_max.argtypes = [vp, i32, dbl, vp]
        L.ora_sigma_max.restype = dbl
        L.ora_step.argtypes = [vp, vp, vp, vp, vp, i64, dbl, dbl, dbl, vp, vp, vp, vp, vp]
        L.ora_kkt.argtypes = [vp, vp, vp, dbl, vp]
        L.ora_kkt_scaled.argtypes = [vp, vp, vp, dbl, vp]
        L.ora_pid.argtypes = [vp, vp, vp, vp, dbl, dbl, dbl, dbl, dbl]
        L.ora_init_state.argtypes = [vp, vp, vp, vp, vp, vp, vp, C.POINTER(State)]
        L.ora_run.argtypes = [vp, C.POINTER(_Params), i64, vp, vp, vp, vp, vp, vp,
                              C.POINTER(State), vp, i32]
        L.ora_run.restype = i64
        L.ora_unscale.argtypes = [vp, vp, vp, vp, vp]
        L.ora_csr_to_csc.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp]
        L.ora_set_qdiag.argtypes = [vp, vp]
        L.ora_set_qdiag.restype = C.c_int
        L.ora_num_threads.restype = i32
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return int(lib().ora_num_threads())


def csr_to_csc(m, n, row_ptr, col_idx, val):
    """A0: CSR -> CSC (stable: row order kept inside each column)."""
    nnz = int(row_ptr[-1])
    cp = np.zeros(n + 1, np.int32)
    ri = np.zeros(max(nnz, 1), np.int32)
    vt = np.zeros(max(nnz, 1), np.float64)
    rp = np.ascontiguousarray(row_ptr, np.int32)
    ci = np.ascontiguousarray(col_idx, np.int32)
    v = _f64(val)
    lib().ora_csr_to_csc(m, n, _p(rp), _p(ci), _p(v), _p(cp), _p(ri), _p(vt))
    return cp, ri[:nnz], vt[:nnz]


class Problem:
    """A prepared problem: CSC built, rescaled, eta and omega0 chosen.

    A diagonal quadratic objective x^T Q x / 2 (Sec. 6) comes from ``q``
    (length n, >= 0), else from ``lp.q`` when the instance carries one."""

    def __init__(self, lp, params: Params | None = None, q=None):
        self.params = params or Params()
        self.m, self.n = int(lp.m), int(lp.n)
        self._keep = [np.ascontiguousarray(lp.row_ptr, np.int32),
                      np.ascontiguousarray(lp.col_idx, np.int32),
                      _f64(lp.val), _f64(lp.c), _f64(lp.con_lo), _f64(lp.con_hi),
                      _f64(lp.var_lo), _f64(lp.var_hi)]
        self.nnz = int(self._keep[0][-1])
        k = self._keep
        clp = _LP(self.m, self.n, *[a.ctypes.data for a in k])
        h = C.c_void_p()
        lib().ora_prepare(C.byref(clp), C.byref(self.params._c()), C.byref(h))
        self._h = h
        out6 = np.zeros(6)
        iout = np.zeros(2, np.int32)
        lib().ora_info(self._h, _p(out6), _p(iout))
        self.eta, self.omega0, self.sigma_max = out6[0], out6[1], out6[2]
        self.c_norm, self.b_norm = out6[3], out6[4]
        self.power_iters = int(iout[0])
        if q is None:
            q = getattr(lp, "q", None)
        self.q = None if q is None else _f64(q)
        if self.q is not None:
            assert self.q.shape == (self.n,) and np.all(self.q >= 0)
            lib().ora_set_qdiag(self._h, _p(self.q))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.ora_free(h)
            self._h = None

    def scaled(self) -> dict:
        """Scaled data: D_r, D_c, A~ (CSR/CSC values) and the scaled vectors."""
        m, n, nnz = self.m, self.n, self.nnz
        out = dict(v=np.zeros(max(nnz, 1)), vt=np.zeros(max(nnz, 1)),
                   dr=np.zeros(m), dc=np.zeros(n), c=np.zeros(n),
                   clo=np.zeros(m), chi=np.zeros(m), vlo=np.zeros(n),
                   vhi=np.zeros(n))
        lib().ora_get_scaled(self._h, *[_p(out[k]) for k in (
            "v", "vt", "dr", "dc", "c", "clo", "chi", "vlo", "vhi")])
        out["v"], out["vt"] = out["v"][:nnz], out["vt"][:nnz]
        return out

    def spmv(self, v, transpose=False):
        v = _f64(v)
        out = np.zeros(self.n if transpose else self.m)
        lib().ora_spmv(self._h, int(transpose), _p(v), _p(out))
        return out

    def sigma_max_power(self, max_iters=5000, tol=1e-6):
        it = np.zeros(1, np.int32)
        s = lib().ora_sigma_max(self._h, max_iters, tol, _p(it))
        return float(s), int(it[0])

    def step(self, x, y, xa, ya, k, tau, sigma, gamma=None):
        """One PDHG + Halpern step in the scaled space (Sec. 2.2, App. B.1)."""
        gamma = self.params.gamma if gamma is None else gamma
        x, y, xa, ya = map(_f64, (x, y, xa, ya))
        xh, xb, xn = (np.zeros(self.n) for _ in range(3))
        yh, yn = np.zeros(self.m), np.zeros(self.m)
        lib().ora_step(self._h, _p(x), _p(y), _p(xa), _p(ya), int(k), tau, sigma,
                       gamma, _p(xh), _p(xb), _p(yh), _p(xn), _p(yn))
        return dict(xh=xh, xb=xb, yh=yh, xn=xn, yn=yn)

    def kkt(self, x, y, tau=None, scaled=False):
        """(r_primal, r_dual, r_gap, obj_primal, obj_dual) (App. B.4)."""
        tau = self.eta / self.omega0 if tau is None else tau
        out = np.zeros(5)
        f = lib().ora_kkt_scaled if scaled else lib().ora_kkt
        f(self._h, _p(_f64(x)), _p(_f64(y)), tau, _p(out))
        return out

    def init_state(self, x0=None, y0=None):
        st = State()
        x, xa = np.zeros(self.n), np.zeros(self.n)
        y, ya = np.zeros(self.m), np.zeros(self.m)
        x0 = None if x0 is None else _f64(x0)
        y0 = None if y0 is None else _f64(y0)
        lib().ora_init_state(self._h, _p(x0), _p(y0), _p(x), _p(y), _p(xa), _p(ya),
                             C.byref(st))
        return dict(x=x, y=y, xa=xa, ya=ya, xh=np.zeros(self.n),
                    yh=np.zeros(self.m), state=st)

    def run(self, st: dict, n_iters: int, params: Params | None = None,
            log_cap: int = 4096):
        """Continue the restarted Halpern PDHG loop for up to n_iters."""
        prm = (params or self.params)._c()
        log = (LogRec * max(log_cap, 1))()
        S = st["state"]
        before = S.n_checks
        done = lib().ora_run(self._h, C.byref(prm), int(n_iters), _p(st["x"]),
                             _p(st["y"]), _p(st["xa"]), _p(st["ya"]), _p(st["xh"]),
                             _p(st["yh"]), C.byref(S),
                             C.cast(log, C.c_void_p), log_cap)
        nrec = min(S.n_checks - before, log_cap)
        st.setdefault("log", []).extend(
            dict(t=r.t, k=r.k, r=r.r, r0=r.r0, r_primal=r.r_primal,
                 r_dual=r.r_dual, r_gap=r.r_gap, omega=r.omega, restart=r.restart)
            for r in (log[i] for i in range(nrec)))
        return int(done)

    def unscale(self, xh, yh):
        x, y = np.zeros(self.n), np.zeros(self.m)
        lib().ora_unscale(self._h, _p(_f64(xh)), _p(_f64(yh)), _p(x), _p(y))
        return x, y

    def solve(self, x0=None, y0=None, max_iters=None):
        """Full solve from (x0, y0) (or zeros): returns a result dict."""
        st = self.init_state(x0, y0)
        n_it = self.params.max_iters if max_iters is None else max_iters
        self.run(st, n_it)
        S = st["state"]
        x, y = self.unscale(st["xh"], st["yh"])
        return dict(x=x, y=y, status=int(S.status), iters=int(S.t),
                    restarts=int(S.restarts), r_primal=S.r_primal,
                    r_dual=S.r_dual, r_gap=S.r_gap, obj_p=S.obj_p,
                    obj_d=S.obj_d, omega=S.omega, state=st)


def pid_update(omega, pid_int, pid_prev, started, dx, dy, kp, ki, kd):
    """App. B.3 PID step on log(omega); returns the new (omega, int, prev, started)."""
    w = C.c_double(omega)
    i_ = C.c_double(pid_int)
    p_ = C.c_double(pid_prev)
    s_ = C.c_int32(started)
    lib().ora_pid(C.byref(w), C.byref(i_), C.byref(p_), C.byref(s_), dx, dy, kp, ki, kd)
    return w.value, i_.value, p_.value, s_.value
