"""Independent LP references used to pin the oracle: brute-force vertex
enumeration for tiny LPs and scipy's HiGHS for moderate ones.  Neither shares
any arithmetic with the oracle or the GPU library."""
from __future__ import annotations

import itertools

import numpy as np
import scipy.optimize as so
import scipy.sparse as sp


def vertex_enumeration(lp, tol=1e-9):
    """Minimum of c^T x over all feasible vertices of a tiny LP (n <= 6).

    Every candidate vertex is the solution of n linearly independent active
    constraints taken from {a_i x = lo_i, a_i x = hi_i, x_j = l_j, x_j = u_j}.
    """
    A = lp.scipy_csr().toarray()
    m, n = A.shape
    planes = []
    for i in range(m):
        for b in (lp.con_lo[i], lp.con_hi[i]):
            if np.isfinite(b):
                planes.append((A[i], b))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        for b in (lp.var_lo[j], lp.var_hi[j]):
            if np.isfinite(b):
                planes.append((e, b))
    best, best_x = np.inf, None
    for idx in itertools.combinations(range(len(planes)), n):
        M = np.array([planes[q][0] for q in idx])
        if abs(np.linalg.det(M)) < 1e-10:
            continue
        x = np.linalg.solve(M, np.array([planes[q][1] for q in idx]))
        ax = A @ x
        scale = 1.0 + np.abs(x).max()
        if np.any(x < lp.var_lo - tol * scale) or np.any(x > lp.var_hi + tol * scale):
            continue
        if np.any(ax < lp.con_lo - tol * scale) or np.any(ax > lp.con_hi + tol * scale):
            continue
        v = float(lp.c @ x)
        if v < best:
            best, best_x = v, x
    return best, best_x


def highs(lp):
    """HiGHS optimum: (objective, x, y) with y in this project's sign
    convention (y >= 0 on rows with only a lower bound, y <= 0 on rows with
    only an upper bound)."""
    A = lp.scipy_csr()
    lo, hi = lp.con_lo, lp.con_hi
    eq = np.flatnonzero(np.isfinite(lo) & np.isfinite(hi) & (lo == hi))
    up = np.flatnonzero(np.isfinite(hi) & ~(np.isfinite(lo) & (lo == hi)))
    dn = np.flatnonzero(np.isfinite(lo) & ~(np.isfinite(hi) & (lo == hi)))
    A_ub = sp.vstack([A[up], -A[dn]]).tocsr() if (up.size + dn.size) else None
    b_ub = np.concatenate([hi[up], -lo[dn]]) if A_ub is not None else None
    A_eq = A[eq] if eq.size else None
    b_eq = lo[eq] if eq.size else None
    bounds = list(zip(np.where(np.isfinite(lp.var_lo), lp.var_lo, None),
                      np.where(np.isfinite(lp.var_hi), lp.var_hi, None)))
    res = so.linprog(lp.c, A_ub=A_ub, b_ub=b_ub, A_eq=A_eq, b_eq=b_eq,
                     bounds=bounds, method="highs")
    assert res.status == 0, res.message
    y = np.zeros(lp.m)
    if eq.size:
        y[eq] = res.eqlin.marginals
    if A_ub is not None:
        mu = res.ineqlin.marginals            # <= 0 for a minimisation
        y[up] += mu[: up.size]                # a x <= u : y <= 0
        y[dn] += -mu[up.size:]                # a x >= l : y >= 0
    return float(res.fun), res.x, y
