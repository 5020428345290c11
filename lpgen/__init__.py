"""Seeded synthetic LP instances shaped like the D-PDLP paper's workloads.

This module only builds problem data (a CSR matrix plus bound and cost
vectors).  It holds none of the solver's arithmetic: no scaling, no PDHG step,
no KKT evaluation.  Both the CPU oracle tests and the GPU path draw their inputs
from here, so the two sides see exactly the same numbers.

Every problem is returned as an ``LP`` with the paper's general form
(Sec. 2.1, problem (1)):  min c^T x  s.t.  con_lo <= A x <= con_hi,
var_lo <= x <= var_hi, where infinite entries are IEEE +-inf.

Instance recipes (the paper's own data sets are not available, so these stand
in for them):

* ``config0``    m=1000 (500 '=', 500 '>='), n=2000, 5 nonzeros per column,
                 0 <= x <= 10, constructed optimum.
* ``config1``    one GPU's share of a huge LP: m=2M, n=4M, ~40M nonzeros,
                 Zipf column degrees (exponent chosen so the mean is 10),
                 10% of rows hold half the nonzeros, per-row log-uniform value
                 scale in [1e-3, 1e3], constructed optimum.
* ``transport``  3000 x 3000 transportation LP, n=9M arcs, m=6000 rows.
* ``config4``    m=50k, n=100k, 10 nonzeros per column (the warm-start base),
                 and ``config4_family(i)`` its perturbed family members.
* ``tiny_lp``    dense tiny LPs (n<=6) with finite boxes and mixed row types,
                 for brute-force vertex enumeration.
* ``staircase_lp`` the multi-period (staircase) variant of config 1.
* ``constructed_qp`` / ``lasso_qp``  diagonal QPs (Sec. 6): a constructed
                 optimum with c shifted by -Q x*, and the LASSO of App. J on a
                 synthetic sparse feature matrix; ``LP.q`` holds diag(Q).

The constructed-optimum recipe: x* has 60% of its entries in (0, 10) and the
rest at 0; y* is N(0,1) on equality rows, |N(0,1)| on active '>=' rows and 0 on
slack '>=' rows; b = A x* minus a U(0.1, 1) slack on the slack rows; and
c = A^T y* + r with r_j = 0 where x*_j is interior and r_j ~ U(0,1) where
x*_j = 0.  (x*, y*) then satisfies every KKT condition exactly (in exact
arithmetic), so c^T x* = b^T y* is the optimal value.
"""
from __future__ import annotations

import dataclasses
import os
from typing import Optional

import numpy as np
import scipy.sparse as sp

INF = np.inf


@dataclasses.dataclass
class LP:
    m: int
    n: int
    row_ptr: np.ndarray   # int32[m+1]
    col_idx: np.ndarray   # int32[nnz], sorted inside each row
    val: np.ndarray       # float64[nnz]
    c: np.ndarray         # float64[n]
    con_lo: np.ndarray    # float64[m]
    con_hi: np.ndarray    # float64[m]
    var_lo: np.ndarray    # float64[n]
    var_hi: np.ndarray    # float64[n]
    name: str = ""
    x_star: Optional[np.ndarray] = None   # constructed primal optimum, if any
    y_star: Optional[np.ndarray] = None   # constructed dual optimum, if any
    obj_star: Optional[float] = None      # objective at the constructed optimum
    q: Optional[np.ndarray] = None        # diagonal of Q for a QP (x^T Q x / 2), else None
    lasso: Optional[dict] = None          # LASSO data (A, b, lam) of a lasso_qp instance

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def scipy_csr(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.col_idx, self.row_ptr),
                             shape=(self.m, self.n))

    def describe(self) -> dict:
        return {"name": self.name, "m": self.m, "n": self.n, "nnz": self.nnz}


def _csr_from_coo(m: int, n: int, rows: np.ndarray, cols: np.ndarray,
                  vals: np.ndarray):
    """CSR arrays (int32 pointers/indices) with column indices sorted per row."""
    order = np.lexsort((cols, rows))
    rows = rows[order]
    cols = cols[order].astype(np.int32)
    vals = vals[order].astype(np.float64)
    counts = np.bincount(rows, minlength=m)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("nnz does not fit in int32")
    return row_ptr.astype(np.int32), cols, vals


def _distinct_rows_per_column(rng, col_of: np.ndarray, draw_rows, m: int,
                              n: int):
    """Draw one row per entry so that rows are distinct inside each column.

    ``col_of`` holds the column of every entry (sorted).  ``draw_rows(k)``
    draws k candidate rows.  Duplicates are redrawn until none remain.
    Returns the row array aligned with the (col, row)-sorted entry order.
    """
    rows = draw_rows(col_of.size)
    cols = col_of
    for _ in range(64):
        key = cols.astype(np.int64) * m + rows
        order = np.argsort(key, kind="stable")
        key = key[order]
        rows = rows[order]
        cols = cols[order]
        dup = np.zeros(key.size, dtype=bool)
        dup[1:] = key[1:] == key[:-1]
        nd = int(dup.sum())
        if nd == 0:
            return cols, rows
        rows[dup] = draw_rows(nd)
    raise RuntimeError("could not make rows distinct inside columns")


def _construct_optimum(rng, A: sp.csr_matrix, m_eq: int, x_hi: float):
    """Constructed primal-dual optimum for rows [0,m_eq) '=' and the rest '>='.

    Returns x*, y*, con_lo, con_hi, c.
    """
    m, n = A.shape
    x_star = np.zeros(n)
    interior = rng.permutation(n)[: int(round(0.6 * n))]
    x_star[interior] = rng.uniform(0.0, x_hi, size=interior.size)
    # U(0, x_hi) is interior with probability one; guard the measure-zero ends.
    x_star[interior] = np.clip(x_star[interior], 1e-9 * x_hi, x_hi * (1 - 1e-9))
    m_ge = m - m_eq
    ge_rows = np.arange(m_eq, m)
    perm = rng.permutation(m_ge)
    active = ge_rows[perm[: m_ge // 2]]
    slack = ge_rows[perm[m_ge // 2:]]
    y_star = np.zeros(m)
    y_star[:m_eq] = rng.standard_normal(m_eq)
    y_star[active] = np.abs(rng.standard_normal(active.size))
    ax = A @ x_star
    b = ax.copy()
    b[slack] -= rng.uniform(0.1, 1.0, size=slack.size)
    r = np.zeros(n)
    at_zero = np.ones(n, dtype=bool)
    at_zero[interior] = False
    r[at_zero] = rng.uniform(0.0, 1.0, size=int(at_zero.sum()))
    c = A.T @ y_star + r
    con_lo = b.copy()
    con_hi = np.full(m, INF)
    con_hi[:m_eq] = b[:m_eq]
    return x_star, y_star, con_lo, con_hi, c


def constructed_lp(m: int, n: int, m_eq: int, per_col: int, seed: int,
                   name: str = "constructed", x_hi: float = 10.0) -> LP:
    """Random feasible LP with a constructed optimum (the config-0 recipe).

    Every column has exactly ``per_col`` distinct rows drawn uniformly; values
    are N(0,1).
    """
    rng = np.random.default_rng(seed)
    col_of = np.repeat(np.arange(n, dtype=np.int64), per_col)
    cols, rows = _distinct_rows_per_column(
        rng, col_of, lambda k: rng.integers(0, m, size=k), m, n)
    vals = rng.standard_normal(rows.size)
    row_ptr, col_idx, val = _csr_from_coo(m, n, rows, cols, vals)
    A = sp.csr_matrix((val, col_idx, row_ptr), shape=(m, n))
    x_star, y_star, con_lo, con_hi, c = _construct_optimum(rng, A, m_eq, x_hi)
    return LP(m, n, row_ptr, col_idx, val, c, con_lo, con_hi,
              np.zeros(n), np.full(n, x_hi), name=name, x_star=x_star,
              y_star=y_star, obj_star=float(c @ x_star))


def constructed_qp(m: int, n: int, m_eq: int, per_col: int, seed: int,
                   q_frac: float = 0.5, name: str = "constructed-qp") -> LP:
    """Diagonal QP with a constructed optimum (Sec. 6): the config-0 recipe's
    LP optimum (x*, y*) with Q_jj ~ U(0.1, 2) on a random q_frac of the
    columns, and c shifted by -Q x*, so that c + Q x* - A^T y* is the LP's
    reduced cost and (x*, y*) stays optimal."""
    base = constructed_lp(m, n, m_eq, per_col, seed, name=name)
    rng = np.random.default_rng(seed + 7919)
    q = np.zeros(n)
    on = rng.random(n) < q_frac
    q[on] = rng.uniform(0.1, 2.0, size=int(on.sum()))
    c = base.c - q * base.x_star
    obj = float(c @ base.x_star + 0.5 * base.x_star @ (q * base.x_star))
    return LP(base.m, base.n, base.row_ptr, base.col_idx, base.val, c, base.con_lo,
              base.con_hi, base.var_lo, base.var_hi, name=name, x_star=base.x_star,
              y_star=base.y_star, obj_star=obj, q=q)


def lasso_qp(samples: int, features: int, per_row: int, seed: int,
             lam_frac: float = 0.01, name: str = "lasso") -> LP:
    """LASSO as a diagonal QP (App. J): min ||A x - b||^2 / 2 + lam ||x||_1
    becomes min r^T r / 2 + lam 1^T t  s.t.  A x - r = b,  x - t <= 0,
    x + t >= 0, over (x, r, t).  A synthetic sparse feature matrix stands in
    for the LIBSVM data: each sample holds per_row features drawn with
    Zipf-like popularity, values U(0, 1).  As in App. J the target b is the
    last column of the matrix (the remaining columns are the features) and
    lam = lam_frac ||A^T b||_inf.  Variables: x and r free, t >= 0.

    Rows: samples '=' rows, then features '<=' rows (x - t), then features
    '>=' rows (x + t); columns: x (features), r (samples), t (features)."""
    rng = np.random.default_rng(seed)
    nf = features + 1
    w = 1.0 / np.arange(1, nf + 1) ** 0.8
    w /= w.sum()
    rows = np.repeat(np.arange(samples), per_row)
    cols = rng.choice(nf, size=rows.size, p=w)
    # the target column is present in about half of the samples
    tgt = rng.random(samples) < 0.5
    rows = np.concatenate([rows, np.flatnonzero(tgt)])
    cols = np.concatenate([cols, np.full(int(tgt.sum()), nf - 1)])
    key = np.unique(rows.astype(np.int64) * nf + cols)
    rows, cols = key // nf, key % nf
    vals = rng.uniform(0.0, 1.0, size=rows.size)
    F = sp.csr_matrix((vals, (rows, cols)), shape=(samples, nf))
    b = F[:, nf - 1].toarray().ravel()
    A = F[:, : nf - 1].tocsr()
    lam = lam_frac * float(np.max(np.abs(A.T @ b)))
    n_x, n_r = features, samples
    I_f = sp.identity(features, format="csr")
    I_s = sp.identity(samples, format="csr")
    Z_sf = sp.csr_matrix((samples, features))
    top = sp.hstack([A, -I_s, Z_sf])
    mid = sp.hstack([I_f, sp.csr_matrix((features, samples)), -I_f])
    bot = sp.hstack([I_f, sp.csr_matrix((features, samples)), I_f])
    M = sp.vstack([top, mid, bot]).tocsr()
    M.sort_indices()
    m_rows, n_cols = M.shape
    con_lo = np.concatenate([b, np.full(features, -INF), np.zeros(features)])
    con_hi = np.concatenate([b, np.zeros(features), np.full(features, INF)])
    c = np.concatenate([np.zeros(n_x + n_r), np.full(features, lam)])
    q = np.concatenate([np.zeros(n_x), np.ones(n_r), np.zeros(features)])
    var_lo = np.concatenate([np.full(n_x + n_r, -INF), np.zeros(features)])
    var_hi = np.full(n_cols, INF)
    return LP(m_rows, n_cols, M.indptr.astype(np.int32), M.indices.astype(np.int32),
              M.data.astype(np.float64), c, con_lo, con_hi, var_lo, var_hi, name=name, q=q,
              lasso=dict(A=A, b=b, lam=lam))


def config0() -> LP:
    """m=1000 (500 '=', 500 '>='), n=2000, 5 per column, seed 0."""
    return constructed_lp(1000, 2000, 500, 5, seed=0, name="c0")


def zipf_exponent_for_mean(mean: float, dmax: int) -> float:
    """Exponent s with E[d] = mean for P(d) ~ d^-s on d in [1, dmax]."""
    d = np.arange(1, dmax + 1, dtype=np.float64)

    def e(s):
        w = d ** (-s)
        return float((w * d).sum() / w.sum())

    lo, hi = 1.0001, 4.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if e(mid) > mean:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def huge_share_lp(m: int = 2_000_000, n: int = 4_000_000, mean_deg: float = 10.0,
                  dmax: int = 5000, heavy_frac: float = 0.1,
                  heavy_share: float = 0.5, seed: int = 1,
                  name: str = "c1") -> LP:
    """One GPU's share of a huge LP (config 1 recipe, any size).

    Column degrees follow a Zipf law clipped to [1, dmax] whose exponent is
    chosen so that the mean degree is ``mean_deg`` (the literal exponent 1.5
    would give ~54 nonzeros per column and ~217M in total, not ~40M).  The
    first ``heavy_frac`` of the rows are "heavy": every nonzero lands in the
    heavy set with probability ``heavy_share``.  Values are N(0,1) times a
    per-row factor 10^U(-3,3).  Half the rows are '=', half '>='.
    """
    rng = np.random.default_rng(seed)
    s = zipf_exponent_for_mean(mean_deg, dmax)
    d = np.arange(1, dmax + 1, dtype=np.float64)
    cdf = np.cumsum(d ** (-s))
    cdf /= cdf[-1]
    deg = np.searchsorted(cdf, rng.random(n), side="right").astype(np.int64) + 1
    deg = np.minimum(deg, dmax)
    m_heavy = max(1, int(round(heavy_frac * m)))
    # A column cannot hold more distinct rows than its row sets offer (only
    # binds for small test instances; at m=2M the clip [1, 5000] rules).
    deg = np.minimum(deg, max(1, min(m_heavy, m - m_heavy)))
    col_of = np.repeat(np.arange(n, dtype=np.int64), deg)

    def draw(k):
        heavy = rng.random(k) < heavy_share
        r = rng.integers(m_heavy, m, size=k)
        r[heavy] = rng.integers(0, m_heavy, size=int(heavy.sum()))
        return r

    cols, rows = _distinct_rows_per_column(rng, col_of, draw, m, n)
    # Every row gets at least one entry: an empty row receives one extra
    # nonzero in a random column.
    counts = np.bincount(rows, minlength=m)
    empty = np.flatnonzero(counts == 0)
    if empty.size:
        rows = np.concatenate([rows, empty])
        cols = np.concatenate([cols, rng.integers(0, n, size=empty.size)])
    row_scale = 10.0 ** rng.uniform(-3.0, 3.0, size=m)
    vals = rng.standard_normal(rows.size) * row_scale[rows]
    row_ptr, col_idx, val = _csr_from_coo(m, n, rows, cols, vals)
    del rows, cols, vals
    A = sp.csr_matrix((val, col_idx, row_ptr), shape=(m, n))
    x_star, y_star, con_lo, con_hi, c = _construct_optimum(rng, A, m // 2, 10.0)
    return LP(m, n, row_ptr, col_idx, val, c, con_lo, con_hi,
              np.zeros(n), np.full(n, 10.0), name=name, x_star=x_star,
              y_star=y_star, obj_star=float(c @ x_star))


def config1() -> LP:
    return _cached("c1", lambda: huge_share_lp(seed=1, name="c1"))


def staircase_lp(m: int = 2_000_000, n: int = 4_000_000, stages: int = 2000,
                 per_col: int = 10, link: float = 0.3, seed: int = 5,
                 name: str = "staircase") -> LP:
    """Multi-period (staircase) LP of config-1 size with a constructed optimum.

    Rows and columns are cut into ``stages`` contiguous stages.  Each column
    holds ``per_col`` distinct rows; each row is drawn uniformly from its own
    stage, or with probability ``link`` from the next stage (the linking
    constraints of a multi-period model; the last stage links to itself).
    In the natural order every column's rows lie in two consecutive stages,
    so the gathers of both products are local.  Values are N(0,1); half the
    rows are '=', half '>='.
    """
    rng = np.random.default_rng(seed)
    if per_col > m // stages:
        raise ValueError("per_col exceeds the rows of a stage")
    r_lo = (np.arange(stages + 1, dtype=np.int64) * m) // stages
    c_stage = (np.arange(n, dtype=np.int64) * stages) // n
    col_of = np.repeat(np.arange(n, dtype=np.int64), per_col)

    def draw(cols):
        s = c_stage[cols]
        nxt = rng.random(cols.size) < link
        s = np.where(nxt, np.minimum(s + 1, stages - 1), s)
        return r_lo[s] + (rng.random(cols.size) * (r_lo[s + 1] - r_lo[s])).astype(np.int64)

    cols, rows = col_of, draw(col_of)
    for _ in range(64):
        key = cols * m + rows
        order = np.argsort(key, kind="stable")
        key, rows, cols = key[order], rows[order], cols[order]
        dup = np.zeros(key.size, dtype=bool)
        dup[1:] = key[1:] == key[:-1]
        if not dup.any():
            break
        rows[dup] = draw(cols[dup])
    else:
        raise RuntimeError("could not make rows distinct inside columns")
    counts = np.bincount(rows, minlength=m)
    empty = np.flatnonzero(counts == 0)
    if empty.size:
        # an empty row takes one entry in a random column of its stage
        st = np.searchsorted(r_lo, empty, side="right") - 1
        c_lo = (st * n + stages - 1) // stages
        c_hi = ((st + 1) * n + stages - 1) // stages
        extra = c_lo + (rng.random(empty.size) * (c_hi - c_lo)).astype(np.int64)
        rows = np.concatenate([rows, empty])
        cols = np.concatenate([cols, extra])
    vals = rng.standard_normal(rows.size)
    row_ptr, col_idx, val = _csr_from_coo(m, n, rows, cols, vals)
    del rows, cols, vals
    A = sp.csr_matrix((val, col_idx, row_ptr), shape=(m, n))
    x_star, y_star, con_lo, con_hi, c = _construct_optimum(rng, A, m // 2, 10.0)
    return LP(m, n, row_ptr, col_idx, val, c, con_lo, con_hi,
              np.zeros(n), np.full(n, 10.0), name=name, x_star=x_star,
              y_star=y_star, obj_star=float(c @ x_star))


def config1_staircase() -> LP:
    """The staircase variant of config 1 (same m, n and nonzeros per column)."""
    return _cached("staircase", lambda: staircase_lp(seed=5))


def transport_lp(n_src: int = 3000, n_dst: int = 3000, seed: int = 2,
                 name: str = "c2") -> LP:
    """Transportation LP: supply rows '<=' then demand rows '>='.

    Arc (i, j) is column i*n_dst + j.  Supplies ~ U(50,150); demands ~
    U(50,150) rescaled to total 95% of the supply; costs are integers
    U{1..100}; 0 <= x < inf.
    """
    rng = np.random.default_rng(seed)
    n = n_src * n_dst
    m = n_src + n_dst
    supply = rng.uniform(50.0, 150.0, size=n_src)
    demand = rng.uniform(50.0, 150.0, size=n_dst)
    demand *= 0.95 * supply.sum() / demand.sum()
    cost = rng.integers(1, 101, size=n).astype(np.float64)
    nnz = 2 * n
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    row_ptr[1:n_src + 1] = np.arange(1, n_src + 1, dtype=np.int64) * n_dst
    row_ptr[n_src + 1:] = n + np.arange(1, n_dst + 1, dtype=np.int64) * n_src
    col_idx = np.empty(nnz, dtype=np.int32)
    col_idx[:n] = np.arange(n, dtype=np.int32)
    # demand row j holds columns j, n_dst + j, 2 n_dst + j, ...
    col_idx[n:] = (np.arange(n_src, dtype=np.int64)[None, :] * n_dst
                   + np.arange(n_dst, dtype=np.int64)[:, None]).ravel()
    val = np.ones(nnz)
    con_lo = np.concatenate([np.full(n_src, -INF), demand])
    con_hi = np.concatenate([supply, np.full(n_dst, INF)])
    return LP(m, n, row_ptr.astype(np.int32), col_idx, val, cost, con_lo,
              con_hi, np.zeros(n), np.full(n, INF), name=name)


def config2() -> LP:
    return _cached("c2", lambda: transport_lp(seed=2, name="c2"))


def config4() -> LP:
    """Warm-start family base: as config 0 at m=50k (25k/25k), n=100k."""
    return constructed_lp(50_000, 100_000, 25_000, 10, seed=4, name="c4")


def perturbed(base: LP, seed: int, sigma: float = 0.1, name: str = "") -> LP:
    """Family member: b and c scaled entrywise by lognormal(sigma) noise.

    Finite row bounds are multiplied by the same factor per row (so '=' rows
    stay equalities); every c_j gets its own factor.
    """
    rng = np.random.default_rng(seed)
    fb = np.exp(sigma * rng.standard_normal(base.m))
    fc = np.exp(sigma * rng.standard_normal(base.n))
    lo = np.where(np.isfinite(base.con_lo), base.con_lo * fb, base.con_lo)
    hi = np.where(np.isfinite(base.con_hi), base.con_hi * fb, base.con_hi)
    return LP(base.m, base.n, base.row_ptr, base.col_idx, base.val,
              base.c * fc, lo, hi, base.var_lo, base.var_hi,
              name=name or f"{base.name}-p{seed}")


def config4_family(i: int, base: Optional[LP] = None) -> LP:
    """Member i of the 512-instance family (0..383 train, 384..511 held out)."""
    base = base if base is not None else config4()
    return perturbed(base, 4_000_000 + i, name=f"c4-{i}")


def tiny_lp(seed: int, n: Optional[int] = None) -> LP:
    """Dense tiny LP (n <= 6) with a finite box and mixed '=', '>=', '<=' rows.

    The right-hand sides come from a random feasible point, so the LP is
    feasible and (the box being finite) bounded.
    """
    rng = np.random.default_rng(seed)
    n = int(n if n is not None else rng.integers(2, 7))
    n_rows = int(rng.integers(1, min(2 * n, 16 - 2 * n) + 1))
    A = rng.standard_normal((n_rows, n))
    A[rng.random(A.shape) < 0.25] = 0.0
    lo_v = -rng.uniform(0.5, 3.0, size=n)
    hi_v = rng.uniform(0.5, 3.0, size=n)
    xf = rng.uniform(lo_v, hi_v)
    ax = A @ xf
    kind = rng.integers(0, 3, size=n_rows)         # 0 '=', 1 '>=', 2 '<='
    n_eq_max = max(0, n - 1)
    eq = np.flatnonzero(kind == 0)
    kind[eq[n_eq_max:]] = 1
    con_lo = np.full(n_rows, -INF)
    con_hi = np.full(n_rows, INF)
    for i in range(n_rows):
        if kind[i] == 0:
            con_lo[i] = con_hi[i] = ax[i]
        elif kind[i] == 1:
            con_lo[i] = ax[i] - rng.uniform(0.0, 1.0)
        else:
            con_hi[i] = ax[i] + rng.uniform(0.0, 1.0)
    c = rng.standard_normal(n)
    rows, cols = np.nonzero(A)
    row_ptr, col_idx, val = _csr_from_coo(n_rows, n, rows, cols, A[rows, cols])
    return LP(n_rows, n, row_ptr, col_idx, val, c, con_lo, con_hi, lo_v, hi_v,
              name=f"tiny{seed}")


def from_dense(A, c, con_lo, con_hi, var_lo, var_hi, name="dense") -> LP:
    """LP from dense arrays (small hand-made test problems)."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    rows, cols = np.nonzero(A)
    row_ptr, col_idx, val = _csr_from_coo(m, n, rows, cols, A[rows, cols])
    f = lambda v, k: np.asarray(v, dtype=np.float64).reshape(k)
    return LP(m, n, row_ptr, col_idx, val, f(c, n), f(con_lo, m), f(con_hi, m),
              f(var_lo, n), f(var_hi, n), name=name)


def permute_lp(lp: LP, perm_row: np.ndarray, perm_col: np.ndarray) -> LP:
    """The same LP with rows/columns relabelled: new row i is old perm_row[i]."""
    A = lp.scipy_csr()[perm_row][:, perm_col].tocsr()
    A.sort_indices()
    return LP(lp.m, lp.n, A.indptr.astype(np.int32), A.indices.astype(np.int32),
              A.data.copy(), lp.c[perm_col], lp.con_lo[perm_row],
              lp.con_hi[perm_row], lp.var_lo[perm_col], lp.var_hi[perm_col],
              name=lp.name + "-perm")


# ---------------------------------------------------------------------------
# Disk cache for the big instances (generation takes tens of seconds).
_CACHE_VERSION = "v1"


def _cache_dir() -> Optional[str]:
    d = os.environ.get("DPDLP_CACHE", "/tmp/dpdlp_lpgen_cache")
    return d or None


def _cached(key: str, make) -> LP:
    d = _cache_dir()
    path = os.path.join(d, f"{key}-{_CACHE_VERSION}.npz") if d else None
    if path and os.path.exists(path):
        z = np.load(path, allow_pickle=False)
        kw = {k: z[k] for k in z.files if k not in ("m", "n", "name", "obj_star")}
        lp = LP(int(z["m"]), int(z["n"]), name=str(z["name"]), **{
            k: v for k, v in kw.items() if k in (
                "row_ptr", "col_idx", "val", "c", "con_lo", "con_hi", "var_lo",
                "var_hi")})
        if "x_star" in z.files:
            lp.x_star, lp.y_star = z["x_star"], z["y_star"]
            lp.obj_star = float(z["obj_star"])
        return lp
    lp = make()
    if path:
        try:
            os.makedirs(d, exist_ok=True)
            arrs = dict(row_ptr=lp.row_ptr, col_idx=lp.col_idx, val=lp.val,
                        c=lp.c, con_lo=lp.con_lo, con_hi=lp.con_hi,
                        var_lo=lp.var_lo, var_hi=lp.var_hi, m=lp.m, n=lp.n,
                        name=lp.name)
            if lp.x_star is not None:
                arrs.update(x_star=lp.x_star, y_star=lp.y_star,
                            obj_star=lp.obj_star)
            tmp = path + f".tmp{os.getpid()}.npz"
            np.savez(tmp, **arrs)
            os.replace(tmp, path)
        except OSError:
            pass
    return lp
