"""Pins of the CPU oracle to facts that do not come from the oracle itself.

Each test names what it pins (the paper passage and the independent fact):
constructed optima (closed form), LP duality, brute-force vertex enumeration,
scipy's HiGHS, textbook special cases, library routines (scipy transpose,
numpy 2-norm).  A plausible slip anywhere in the oracle (a dropped term, a
sign, an index, a transposed operand) fails at least one of them.
"""
import dataclasses

import numpy as np
import pytest
import scipy.sparse as sp

import lpgen
from tests import lputil


def _prm(oracle, **kw):
    return oracle.Params(**kw)


def _scaled_opt(P, lp):
    d = P.scaled()
    return lp.x_star / d["dc"], lp.y_star / d["dr"], d


# -- A0: CSR -> CSC equals scipy's transpose (library routine) ------------------
def test_csc_matches_scipy(oracle_mod):
    lp = lpgen.config0()
    cp, ri, vt = oracle_mod.csr_to_csc(lp.m, lp.n, lp.row_ptr, lp.col_idx, lp.val)
    ref = lp.scipy_csr().tocsc()
    ref.sort_indices()
    assert np.array_equal(cp, ref.indptr)
    assert np.array_equal(ri, ref.indices)
    assert np.array_equal(vt, ref.data)


# -- A3: scaled matrix is D_r A D_c, and Ruiz equilibrates -----------------------
def test_scaling_bookkeeping(oracle_mod):
    lp = lpgen.constructed_lp(300, 500, 150, 4, seed=11)
    P = oracle_mod.Problem(lp, _prm(oracle_mod, eta=1.0, omega0=1.0))
    d = P.scaled()
    A = lp.scipy_csr()
    At = (sp.diags(d["dr"]) @ A @ sp.diags(d["dc"])).tocsr()
    assert np.allclose(At.data, d["v"], rtol=1e-13, atol=0)
    # CSC copy holds the same numbers, bit for bit
    csc = sp.csr_matrix((d["v"], lp.col_idx, lp.row_ptr), shape=A.shape).tocsc()
    csc.sort_indices()
    assert np.array_equal(csc.data, d["vt"])
    # scaled vectors
    assert np.allclose(d["c"], d["dc"] * lp.c, rtol=1e-15)
    assert np.allclose(d["vhi"], lp.var_hi / d["dc"], rtol=1e-15)
    fin = np.isfinite(lp.con_lo)
    assert np.allclose(d["clo"][fin], d["dr"][fin] * lp.con_lo[fin], rtol=1e-15)


@pytest.mark.parametrize("passes,tol", [(10, 2e-2), (40, 1e-6)])
def test_ruiz_equilibrates(oracle_mod, passes, tol):
    """Ruiz infinity-norm passes drive every nonempty row and column max-norm
    to one (each pass roughly halves the log-deviation)."""
    lp = lpgen.huge_share_lp(m=2000, n=4000, seed=5)   # values span 1e-3..1e3
    P = oracle_mod.Problem(lp, _prm(oracle_mod, eta=1.0, omega0=1.0, use_pc=0,
                                    ruiz_iters=passes))
    d = P.scaled()
    At = sp.csr_matrix((np.abs(d["v"]), lp.col_idx, lp.row_ptr), shape=(lp.m, lp.n))
    rmax = At.max(axis=1).toarray().ravel()
    cmax = At.max(axis=0).toarray().ravel()
    nz_r = np.diff(lp.row_ptr) > 0
    nz_c = np.bincount(lp.col_idx, minlength=lp.n) > 0
    assert np.all(np.abs(rmax[nz_r] - 1) < tol)
    assert np.all(np.abs(cmax[nz_c] - 1) < tol)


def test_pock_chambolle_alpha1(oracle_mod):
    """After Ruiz=0 and one Pock-Chambolle(alpha=1) pass, the scale factors
    equal 1/sqrt of the absolute row / column sums of A (closed form)."""
    lp = lpgen.constructed_lp(200, 300, 100, 3, seed=12)
    P = oracle_mod.Problem(lp, _prm(oracle_mod, eta=1.0, omega0=1.0, ruiz_iters=0))
    d = P.scaled()
    A = abs(lp.scipy_csr())
    rs = np.asarray(A.sum(axis=1)).ravel()
    cs = np.asarray(A.sum(axis=0)).ravel()
    assert np.allclose(d["dr"], np.where(rs > 0, 1 / np.sqrt(np.where(rs > 0, rs, 1)), 1))
    assert np.allclose(d["dc"], np.where(cs > 0, 1 / np.sqrt(np.where(cs > 0, cs, 1)), 1))


# -- A4: power iteration vs numpy's spectral norm ----------------------------
def test_power_iteration_sigma_max(oracle_mod):
    lp = lpgen.config0()
    P = oracle_mod.Problem(lp)
    d = P.scaled()
    Ad = sp.csr_matrix((d["v"], lp.col_idx, lp.row_ptr), shape=(lp.m, lp.n)).toarray()
    ref = np.linalg.norm(Ad, 2)
    s_tight, _ = P.sigma_max_power(max_iters=20000, tol=1e-12)
    assert abs(s_tight - ref) <= 1e-6 * ref
    assert abs(P.sigma_max - ref) <= 2e-3 * ref         # default tolerance 1e-6
    assert np.isclose(P.eta, 0.998 / P.sigma_max, rtol=1e-15)


# -- P1: one PDHG step fixes a constructed optimum ----------------------------
@pytest.mark.parametrize("k", [0, 7])
def test_constructed_optimum_is_fixed_point(oracle_mod, k):
    lp = lpgen.config0()
    P = oracle_mod.Problem(lp)
    xs, ys, _ = _scaled_opt(P, lp)
    for tau, sig in [(P.eta / P.omega0, P.eta * P.omega0), (0.3, 0.5)]:
        o = P.step(xs, ys, xs, ys, k, tau, sig)
        assert np.allclose(o["xh"], xs, rtol=0, atol=1e-12 * np.abs(xs).max())
        assert np.allclose(o["yh"], ys, rtol=0, atol=1e-12 * np.abs(ys).max())
        assert np.allclose(o["xn"], xs, rtol=0, atol=1e-12 * np.abs(xs).max())
        assert np.allclose(o["yn"], ys, rtol=0, atol=1e-12 * np.abs(ys).max())


def test_halpern_anchor_weight(oracle_mod):
    """At z = z* with a different anchor z0: z_{k+1} = (k+1)/(k+2) z* + z0/(k+2)
    (App. B.1 read affinely: the coefficients sum to one)."""
    lp = lpgen.config0()
    P = oracle_mod.Problem(lp)
    xs, ys, d = _scaled_opt(P, lp)
    rng = np.random.default_rng(3)
    xa = np.clip(xs + rng.standard_normal(lp.n), d["vlo"], d["vhi"])
    ya = ys + rng.standard_normal(lp.m)
    for k in (0, 5, 100):
        o = P.step(xs, ys, xa, ya, k, 0.2, 0.3)
        a, b = (k + 1) / (k + 2), 1 / (k + 2)
        assert np.allclose(o["xn"], a * xs + b * xa, rtol=1e-12, atol=1e-12)
        assert np.allclose(o["yn"], a * ys + b * ya, rtol=1e-12, atol=1e-12)


def test_reflection_is_linear_in_gamma(oracle_mod):
    lp = lpgen.config0()
    P = oracle_mod.Problem(lp)
    rng = np.random.default_rng(4)
    d = P.scaled()
    x = np.clip(rng.uniform(0, 5, lp.n) / d["dc"], d["vlo"], d["vhi"])
    y = rng.standard_normal(lp.m)
    o0 = P.step(x, y, x, y, 3, 0.1, 0.2, gamma=0.0)
    o1 = P.step(x, y, x, y, 3, 0.1, 0.2, gamma=1.0)
    a = 4 / 5
    assert np.allclose(o1["xn"] - o0["xn"], a * (o0["xh"] - x), rtol=1e-10, atol=1e-12)
    assert np.allclose(o1["yn"] - o0["yn"], a * (o0["yh"] - y), rtol=1e-10, atol=1e-12)


def test_dual_step_matches_textbook_projected_gradient(oracle_mod):
    """For '=' rows y+ = y + sigma (b - A xbar); for '>=' rows
    y+ = max(0, y + sigma (l - A xbar)); for '<=' rows y+ = min(0, y + sigma
    (u - A xbar)).  Pins the sign reading of the Lagrangian."""
    lp = lpgen.from_dense(
        np.random.default_rng(0).standard_normal((7, 4)), np.ones(4),
        [1, -np.inf, 0.5, -2, -np.inf, -1, -0.5], [1, 2.0, np.inf, -2, 3, np.inf, 0.7],
        -np.ones(4), np.ones(4))
    P = oracle_mod.Problem(lp, _prm(oracle_mod, ruiz_iters=0, use_pc=0, eta=0.4, omega0=1.0))
    rng = np.random.default_rng(1)
    x = rng.uniform(-1, 1, 4)
    y = rng.standard_normal(7)
    tau, sig = 0.4, 0.4
    o = P.step(x, y, x, y, 0, tau, sig)
    A = lp.scipy_csr().toarray()
    g = y + sig * (-(A @ o["xb"]))
    ref = np.empty(7)
    for i in range(7):
        lo, hi = lp.con_lo[i], lp.con_hi[i]
        if lo == hi:
            ref[i] = g[i] + sig * lo
        elif np.isfinite(lo) and np.isfinite(hi):   # ranged row: soft threshold
            v = g[i]
            ref[i] = v + sig * hi if v < -sig * hi else (v + sig * lo if v > -sig * lo else 0.0)
        elif np.isfinite(lo):
            ref[i] = max(0.0, g[i] + sig * lo)
        else:
            ref[i] = min(0.0, g[i] + sig * hi)
    assert np.allclose(o["yh"], ref, rtol=1e-13, atol=1e-14)
    # primal: textbook clip(x - tau (c - A^T y))
    assert np.allclose(o["xh"], np.clip(x - tau * (lp.c - A.T @ y), -1, 1), rtol=1e-13, atol=1e-14)


# -- P2 / duality: KKT at known optima ----------------------------------------
@pytest.mark.parametrize("tau", [1e-3, 0.5, 10.0])
def test_kkt_zero_at_constructed_optimum(oracle_mod, tau):
    lp = lpgen.config0()
    P = oracle_mod.Problem(lp)
    k = P.kkt(lp.x_star, lp.y_star, tau=tau)
    assert k[0] < 1e-14 and k[1] < 1e-14 and k[2] < 1e-14
    assert np.isclose(k[3], lp.obj_star, rtol=1e-14)
    bty = lp.con_lo @ lp.y_star
    assert np.isclose(k[4], bty, rtol=1e-12)


def test_staircase_generator_structure_and_optimum(oracle_mod):
    """The staircase variant of config 1 (at 1/100 scale): every column's
    rows lie in its own stage or the next one, no row is empty, and the
    constructed optimum has zero KKT residuals with c^T x* = b^T y*."""
    lp = lpgen.staircase_lp(20000, 40000, stages=40, per_col=10, seed=3)
    A = lp.scipy_csr().tocoo()
    d = (A.row * 40) // lp.m - (A.col * 40) // lp.n
    assert set(np.unique(d).tolist()) <= {0, 1}
    assert np.all(np.diff(lp.row_ptr) > 0)
    assert np.all(np.bincount(lp.col_idx, minlength=lp.n) >= 10)
    k = oracle_mod.Problem(lp).kkt(lp.x_star, lp.y_star, tau=1.0)
    assert max(k[0], k[1], k[2]) < 1e-13
    assert np.isclose(k[4], lp.con_lo @ lp.y_star, rtol=1e-12)
    assert np.isclose(k[3], k[4], rtol=1e-10)


def test_kkt_at_highs_optimum_and_objective(oracle_mod):
    """HiGHS's primal/dual pair (converted to this sign convention) has tiny
    KKT residuals in the oracle's measure, and the oracle solve reaches the
    HiGHS objective."""
    lp = lpgen.transport_lp(40, 30, seed=7)
    obj, xh, yh = lputil.highs(lp)
    P = oracle_mod.Problem(lp)
    k = P.kkt(xh, yh, tau=1e-6)
    assert max(k[:3]) < 1e-7, k
    r = P.solve(max_iters=400_000)
    assert r["status"] == 1
    assert abs(r["obj_p"] - obj) <= 1e-6 * (1 + abs(obj))


def test_kkt_detects_infeasibility_and_sign_errors(oracle_mod):
    lp = lpgen.config0()
    P = oracle_mod.Problem(lp)
    # flipping the dual's sign breaks dual feasibility and the gap
    k = P.kkt(lp.x_star, -lp.y_star, tau=1e-3)
    assert k[1] > 1e-3 or k[2] > 1e-3
    # moving x off the optimum gives the exact primal residual
    x = lp.x_star.copy()
    x[0] += 1.0
    k = P.kkt(x, lp.y_star, tau=1e-3)
    A = lp.scipy_csr()
    ax = A @ x
    viol = ax - np.clip(ax, lp.con_lo, lp.con_hi)
    bn = np.sqrt(np.sum(lp.con_lo[np.isfinite(lp.con_lo)] ** 2)
                 + np.sum(lp.con_hi[np.isfinite(lp.con_hi)] ** 2))
    assert np.isclose(k[0], np.linalg.norm(viol) / (1 + bn), rtol=1e-10)


# -- P3 / P5: whole solver -----------------------------------------------------
def test_solve_config0_to_1e8(oracle_mod):
    lp = lpgen.config0()
    P = oracle_mod.Problem(lp)
    r = P.solve()
    assert r["status"] == 1
    assert max(r["r_primal"], r["r_dual"], r["r_gap"]) <= 1e-8
    assert abs(r["obj_p"] - lp.obj_star) <= 1e-7 * (1 + abs(lp.obj_star))
    obj_h, _, _ = lputil.highs(lp)
    assert abs(r["obj_p"] - obj_h) <= 1e-7 * (1 + abs(obj_h))


def test_solve_1e4_tolerance(oracle_mod):
    lp = lpgen.config0()
    P = oracle_mod.Problem(lp, _prm(oracle_mod, eps=1e-4))
    r = P.solve()
    assert r["status"] == 1
    assert max(r["r_primal"], r["r_dual"], r["r_gap"]) <= 1e-4
    assert abs(r["obj_p"] - lp.obj_star) <= 1e-3 * (1 + abs(lp.obj_star))


@pytest.mark.parametrize("seed", range(12))
def test_tiny_lp_vertex_enumeration(oracle_mod, seed):
    lp = lpgen.tiny_lp(seed)
    best, _ = lputil.vertex_enumeration(lp)
    P = oracle_mod.Problem(lp, _prm(oracle_mod, eps=1e-10, max_iters=2_000_000))
    r = P.solve()
    assert r["status"] == 1, (seed, r["iters"])
    assert abs(r["obj_p"] - best) <= 1e-7 * (1 + abs(best)), (r["obj_p"], best)


def test_moderate_constructed_lp_reaches_constructed_optimum(oracle_mod):
    """At 2500 x 5000 the constructed optimum's value c^T x* = b^T y* is the
    exact reference (HiGHS needs minutes here; it is used on config 0)."""
    lp = lpgen.constructed_lp(2500, 5000, 1250, 10, seed=44)
    P = oracle_mod.Problem(lp)
    r = P.solve(max_iters=300_000)
    assert r["status"] == 1
    assert abs(r["obj_p"] - lp.obj_star) <= 1e-7 * (1 + abs(lp.obj_star))


# -- P6: special cases with closed forms ---------------------------------------
def test_box_only_lp(oracle_mod):
    """No binding rows (one free row): x_j = l_j if c_j > 0 else u_j."""
    rng = np.random.default_rng(9)
    n = 50
    c = rng.standard_normal(n)
    lo, hi = -rng.uniform(0, 2, n), rng.uniform(0, 2, n)
    A = np.zeros((1, n))
    A[0, :3] = 1.0
    lp = lpgen.from_dense(A, c, [-np.inf], [np.inf], lo, hi)
    r = oracle_mod.Problem(lp).solve()
    assert r["status"] == 1
    assert np.allclose(r["x"], np.where(c > 0, lo, hi), atol=1e-7)
    assert abs(r["obj_p"] - np.sum(np.where(c > 0, c * lo, c * hi))) < 1e-7


def test_fractional_knapsack(oracle_mod):
    """One '<=' row: max v^T x, w^T x <= W, 0 <= x <= 1 has the greedy optimum."""
    rng = np.random.default_rng(10)
    n = 30
    v, w = rng.uniform(1, 10, n), rng.uniform(1, 10, n)
    W = 0.4 * w.sum()
    lp = lpgen.from_dense(w[None, :], -v, [-np.inf], [W], np.zeros(n), np.ones(n))
    order = np.argsort(-v / w)
    x = np.zeros(n)
    cap = W
    for j in order:
        take = min(1.0, cap / w[j])
        x[j] = take
        cap -= take * w[j]
        if cap <= 0:
            break
    r = oracle_mod.Problem(lp, _prm(oracle_mod, eps=1e-10)).solve()
    assert r["status"] == 1
    assert abs(r["obj_p"] - (-v @ x)) <= 1e-8 * (1 + v @ x)
    assert r["y"][0] <= 0                      # a '<=' row has y <= 0


def test_empty_rows_and_columns(oracle_mod):
    A = np.array([[1.0, 0, 1, 0], [0, 0, 0, 0], [1, 0, -1, 0]])
    lp = lpgen.from_dense(A, [1.0, 2.0, -1.0, -3.0], [1.0, -np.inf, -1.0],
                          [1.0, np.inf, np.inf], [0, 0, 0, 0], [5, 5, 5, 5])
    best, _ = lputil.vertex_enumeration(lp)
    r = oracle_mod.Problem(lp, _prm(oracle_mod, eps=1e-10)).solve()
    assert r["status"] == 1
    assert abs(r["obj_p"] - best) < 1e-8
    assert r["x"][1] < 1e-8 and abs(r["x"][3] - 5) < 1e-8      # empty columns
    assert r["y"][1] == 0.0                                     # free empty row


# -- A9: PID arithmetic, closed forms ------------------------------------------
def test_pid_pure_proportional_is_distance_ratio(oracle_mod):
    w, _, _, _ = oracle_mod.pid_update(3.0, 0.0, 0.0, 0, 2.0, 5.0, 1.0, 0.0, 0.0)
    assert np.isclose(w, 5.0 / 2.0, rtol=1e-15)


def test_pid_two_restarts_closed_form(oracle_mod):
    kp, ki, kd = 0.7, 0.2, 0.1
    w0, dx1, dy1, dx2, dy2 = 1.5, 0.3, 0.9, 0.8, 0.1
    w1, i1, p1, s1 = oracle_mod.pid_update(w0, 0.0, 0.0, 0, dx1, dy1, kp, ki, kd)
    e1 = np.log(w0 * dx1 / dy1)
    assert np.isclose(w1, w0 * np.exp(-(kp * e1 + ki * e1)), rtol=1e-14)
    w2, _, _, _ = oracle_mod.pid_update(w1, i1, p1, s1, dx2, dy2, kp, ki, kd)
    e2 = np.log(w1 * dx2 / dy2)
    assert np.isclose(w2, w1 * np.exp(-(kp * e2 + ki * (e1 + e2) + kd * (e2 - e1))),
                      rtol=1e-13)
    # degenerate distances leave omega alone
    assert oracle_mod.pid_update(2.0, 0, 0, 0, 0.0, 1.0, kp, ki, kd)[0] == 2.0


# -- restart log: consistent with the stated rule ------------------------------
def test_restart_log_consistency(oracle_mod):
    lp = lpgen.config0()
    P = oracle_mod.Problem(lp)
    r = P.solve()
    log = r["state"]["log"]
    assert r["restarts"] == sum(1 for e in log if e["restart"])
    prev = None
    for e in log:
        if e["k"] == 0:
            assert e["restart"] == 0 and e["r0"] == e["r"]
        if e["restart"] == 1:
            assert e["r"] <= 0.2 * e["r0"]
        if e["restart"] == 2:
            assert e["r"] <= 0.8 * e["r0"] and prev is not None and e["r"] > prev["r"]
        if e["restart"] == 3:
            assert e["k"] >= 0.36 * e["t"]
        if prev is not None and prev["restart"]:
            assert e["k"] == 0 and e["t"] == prev["t"] + 1
        prev = e


def test_thread_count_does_not_change_results(oracle_mod):
    import subprocess, sys, json, os
    code = ("import sys, json; sys.path.insert(0, %r); import oracle, lpgen;"
            "lp = lpgen.config0(); r = oracle.Problem(lp).solve(max_iters=500);"
            "print(json.dumps([float(r['x'].sum()), float(r['y'].sum()), r['obj_p']]))"
            % os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    outs = []
    for th in ("1", "3"):
        env = dict(os.environ, OMP_NUM_THREADS=th)
        outs.append(subprocess.check_output([sys.executable, "-c", code], env=env))
    assert outs[0] == outs[1]


# -- Sec. 6: diagonal QP ----------------------------------------------------------
def test_qp_kkt_zero_at_constructed_optimum(oracle_mod):
    """A constructed diagonal QP (the LP optimum with c shifted by -Q x*) has
    zero KKT residuals at (x*, y*) and the objective c^T x* + x*^T Q x* / 2.
    A dropped Q x term in the dual residual, or a missing half-quadratic in
    either objective, leaves a residual or a gap here."""
    lp = lpgen.constructed_qp(300, 500, 150, 4, seed=3)
    P = oracle_mod.Problem(lp)
    for tau in (1e-3, 0.5, 10.0):
        k = P.kkt(lp.x_star, lp.y_star, tau=tau)
        assert max(k[0], k[1], k[2]) < 1e-13, k
        assert np.isclose(k[3], lp.obj_star, rtol=1e-13)
        assert np.isclose(k[4], lp.obj_star, rtol=1e-11)
    # without Q the same point is not optimal (its dual residual is Q x*)
    k0 = oracle_mod.Problem(lp, q=np.zeros(lp.n)).kkt(lp.x_star, lp.y_star, tau=1.0)
    assert k0[1] > 1e-3


def test_qp_step_minimises_the_prox_subproblem(oracle_mod):
    """The QP primal step (Sec. 6) is the minimiser over the box of
    q x^2 / 2 + g x + (x - x_k)^2 / (2 tau), checked per column with scipy's
    bounded scalar minimiser; with q = 0 it is the LP step bit for bit."""
    from scipy.optimize import minimize_scalar
    lp = lpgen.constructed_qp(40, 60, 20, 3, seed=5)
    P = oracle_mod.Problem(lp)
    P0 = oracle_mod.Problem(lp, q=np.zeros(lp.n))
    PL = oracle_mod.Problem(dataclasses.replace(lp, q=None))
    d = P.scaled()
    rng = np.random.default_rng(0)
    x = rng.uniform(0, 3, lp.n) / d["dc"]
    y = rng.standard_normal(lp.m)
    tau, sigma = 0.37, 0.9
    o = P.step(x, y, x, y, 0, tau, sigma)
    A = sp.csr_matrix((d["v"], lp.col_idx, lp.row_ptr), shape=(lp.m, lp.n))
    g = d["c"] - A.T @ y
    qs = d["dc"] ** 2 * lp.q
    for j in range(lp.n):
        f = lambda v: 0.5 * qs[j] * v * v + g[j] * v + (v - x[j]) ** 2 / (2 * tau)
        r = minimize_scalar(f, bounds=(d["vlo"][j], d["vhi"][j]), method="bounded",
                            options=dict(xatol=1e-12))
        assert abs(o["xh"][j] - r.x) <= 1e-7 * (1 + abs(r.x)), j
    o0, oL = P0.step(x, y, x, y, 0, tau, sigma), PL.step(x, y, x, y, 0, tau, sigma)
    for k in ("xh", "yh", "xn", "yn"):
        assert np.array_equal(o0[k], oL[k])


def _lasso_cd(A, b, lam, sweeps=20000):
    """Textbook cyclic coordinate descent for the LASSO (soft thresholding)."""
    A = A.toarray()
    n = A.shape[1]
    x = np.zeros(n)
    r = b.copy()
    cs = (A * A).sum(axis=0)
    for _ in range(sweeps):
        big = 0.0
        for j in range(n):
            if cs[j] == 0.0:
                continue
            rho = A[:, j] @ r + cs[j] * x[j]
            xn = np.sign(rho) * max(abs(rho) - lam, 0.0) / cs[j]
            if xn != x[j]:
                r += A[:, j] * (x[j] - xn)
                big = max(big, abs(xn - x[j]))
                x[j] = xn
        if big < 1e-15:
            break
    return x


@pytest.mark.parametrize("seed", [1, 2])
def test_lasso_qp_matches_coordinate_descent(oracle_mod, seed):
    """The LASSO of App. J as a diagonal QP, solved by the oracle to 1e-9,
    against cyclic coordinate descent on the LASSO itself: the same LASSO
    objective and the same x."""
    lp = lpgen.lasso_qp(60, 25, 4, seed=seed)
    A, b, lam = lp.lasso["A"], lp.lasso["b"], lp.lasso["lam"]
    P = oracle_mod.Problem(lp, oracle_mod.Params(eps=1e-9))
    r = P.solve(max_iters=2_000_000)
    assert r["status"] == 1
    nf = A.shape[1]
    x = r["x"][:nf]
    f = lambda v: 0.5 * float(np.sum((A @ v - b) ** 2)) + lam * float(np.abs(v).sum())
    xc = _lasso_cd(A, b, lam)
    assert abs(f(x) - f(xc)) <= 1e-7 * (1 + f(xc))
    assert np.allclose(x, xc, atol=1e-5)
    assert abs(r["obj_p"] - f(xc)) <= 1e-7 * (1 + f(xc))


def test_constructed_qp_solves_to_its_optimum(oracle_mod):
    lp = lpgen.constructed_qp(300, 500, 150, 4, seed=3)
    r = oracle_mod.Problem(lp).solve(max_iters=300_000)
    assert r["status"] == 1
    assert abs(r["obj_p"] - lp.obj_star) <= 1e-7 * (1 + abs(lp.obj_star))


# -- A7 off the optimum: App. B.4's formulas evaluated directly -----------------
def _mixed_bounds_lp(seed, m=60, n=90):
    """A sparse LP with every row type of Sec. 2.1 ('=', '>=', '<=', ranged,
    free) and every variable-bound type (box, upper only, lower only, free),
    with entries spread over four orders of magnitude so that scaling moves
    every D_r and D_c entry away from one."""
    rng = np.random.default_rng(seed)
    A = sp.random(m, n, density=0.08, random_state=rng, format="csr",
                  data_rvs=lambda k: rng.standard_normal(k) * 10.0 ** rng.uniform(-2, 2, k))
    A = A.toarray()
    A[np.arange(m), np.arange(m) % n] += 1.0          # no empty row
    kind = np.arange(m) % 5
    b = rng.standard_normal(m)
    lo = np.select([kind == 0, kind == 1, kind == 2, kind == 3, kind == 4],
                   [b, b, -np.inf, b - 1.0, -np.inf])
    hi = np.select([kind == 0, kind == 1, kind == 2, kind == 3, kind == 4],
                   [b, np.inf, b, b + 2.0, np.inf])
    vk = np.arange(n) % 4
    vlo = np.select([vk == 0, vk == 1, vk == 2, vk == 3], [-1.0, -np.inf, -3.0, -np.inf])
    vhi = np.select([vk == 0, vk == 1, vk == 2, vk == 3], [2.0, 5.0, np.inf, np.inf])
    return lpgen.from_dense(A, rng.standard_normal(n), lo, hi, vlo, vhi, name="mixed")


def _point_in_x_and_y(lp, seed):
    rng = np.random.default_rng(seed)
    x = np.clip(3.0 * rng.standard_normal(lp.n), lp.var_lo, lp.var_hi)
    y = 2.0 * rng.standard_normal(lp.m)
    lo_f, hi_f = np.isfinite(lp.con_lo), np.isfinite(lp.con_hi)
    y = np.where(lo_f & hi_f, y, np.where(lo_f, np.abs(y), np.where(hi_f, -np.abs(y), 0.0)))
    return x, y


def _kkt_app_b4(lp, x, y, tau):
    """r_primal, r_dual, r_gap and both objectives, written from App. B.4 and
    Sec. 2.1 as printed: proj_S and proj_X are clips, p(y; l, u) =
    u^T y+ - l^T y- (an infinite bound meets a zero part), and s is the
    projection's displacement divided by tau.  tau may be a vector (a
    per-column step)."""
    A = lp.scipy_csr().toarray()
    ax = A @ x
    finite = np.concatenate([lp.con_lo[np.isfinite(lp.con_lo)],
                             lp.con_hi[np.isfinite(lp.con_hi)]])
    r_primal = np.linalg.norm(ax - np.clip(ax, lp.con_lo, lp.con_hi)) / (1 + np.linalg.norm(finite))
    u = x - tau * (lp.c - A.T @ y)
    pu = np.clip(u, lp.var_lo, lp.var_hi)
    r_dual = np.linalg.norm((pu - x) / tau) / (1 + np.linalg.norm(lp.c))
    s = (pu - u) / tau
    yp, ym = np.maximum(-y, 0.0), np.maximum(y, 0.0)          # (-y)+ and (-y)-
    p_neg_y = (np.sum(lp.con_hi[yp > 0] * yp[yp > 0])
               - np.sum(lp.con_lo[ym > 0] * ym[ym > 0]))      # p(-y; l_c, u_c)
    cx = lp.c @ x
    dual_obj = -p_neg_y + s @ x
    r_gap = abs(cx + p_neg_y - s @ x) / (1 + max(abs(cx), abs(dual_obj)))
    return np.array([r_primal, r_dual, r_gap, cx, dual_obj])


@pytest.mark.parametrize("seed", [0, 1])
@pytest.mark.parametrize("tau", [1e-3, 0.3, 5.0])
def test_kkt_off_optimum_matches_app_b4_unscaled(oracle_mod, seed, tau):
    """With scaling off (D_r = D_c = I) the oracle's KKT at a random
    non-optimal point of X x Y equals App. B.4 evaluated directly, for every
    row and bound type: the residual norms, the gap, and both objectives.
    The oracle forms the dual residual as (c - A^T y) - s; here it is the
    printed ||proj_X(x - tau(c - A^T y)) - x|| / tau, another route."""
    lp = _mixed_bounds_lp(seed)
    x, y = _point_in_x_and_y(lp, seed + 10)
    P = oracle_mod.Problem(lp, _prm(oracle_mod, ruiz_iters=0, use_pc=0, eta=1.0, omega0=1.0))
    d = P.scaled()
    assert np.all(d["dr"] == 1.0) and np.all(d["dc"] == 1.0)
    got = P.kkt(x, y, tau=tau)
    ref = _kkt_app_b4(lp, x, y, tau)
    assert np.all(ref[:3] > 1e-3), ref                    # far from optimal
    assert np.allclose(got, ref, rtol=1e-13, atol=0), (got, ref)


@pytest.mark.parametrize("tau", [1e-3, 0.3, 5.0])
def test_kkt_through_scaling_is_app_b4_in_original_space(oracle_mod, tau):
    """The scaled-path KKT (the reading that evaluates at the scaled T(z) and
    maps back: A x = D_r^-1 A~ x~, s = D_c^-1 s~) against the original-space
    formulas.  The primal residual is the printed one.  The primal step of
    the scaled problem with step tau, mapped back, is the original problem's
    step with the per-column step tau D_c^2, so r_dual and r_gap are App. B.4
    with that vector of steps.  A dropped or inverted D_c anywhere in the
    mapping, or D_r in place of D_c, fails here."""
    lp = _mixed_bounds_lp(3)
    x, y = _point_in_x_and_y(lp, 13)
    P = oracle_mod.Problem(lp, _prm(oracle_mod, eta=1.0, omega0=1.0))
    dc = P.scaled()["dc"]
    assert dc.max() / dc.min() > 10.0                    # scaling is far from I
    got = P.kkt(x, y, tau=tau)
    ref = _kkt_app_b4(lp, x, y, tau * dc ** 2)
    assert np.isclose(got[0], _kkt_app_b4(lp, x, y, tau)[0], rtol=1e-12, atol=0)
    assert np.allclose(got, ref, rtol=1e-12, atol=0), (got, ref)
    # a uniform step would not do once the clamps bind (at tau = 1e-3 hardly
    # any does, and then r_dual is ||c - A^T y|| under either step)
    if tau >= 0.3:
        assert not np.isclose(got[1], _kkt_app_b4(lp, x, y, tau)[1], rtol=1e-3)


# -- A8: the fixed-point residual is the P-norm of z - T(z) ------------------------
def test_restart_residual_is_the_p_norm_of_the_step(oracle_mod):
    """r at a check equals sqrt(dz^T P dz) with dz = z - T(z) and the
    block matrix P = [[omega/eta I, A~^T], [A~, 1/(eta omega) I]] of App. B
    assembled explicitly (scaled space), at the first check (k = 0) and at
    the check of iteration 63."""
    lp = lpgen.constructed_lp(40, 70, 20, 3, seed=21)
    P = oracle_mod.Problem(lp)
    d = P.scaled()
    At = sp.csr_matrix((d["v"], lp.col_idx, lp.row_ptr), shape=(lp.m, lp.n)).toarray()
    for t_check in (0, 63):
        st = P.init_state()
        if t_check:
            P.run(st, t_check)                         # iterations 0 .. t_check-1
        x, y = st["x"].copy(), st["y"].copy()
        xa, ya = st["xa"].copy(), st["ya"].copy()
        S = st["state"]
        w = S.omega
        o = P.step(x, y, xa, ya, S.k, P.eta / w, P.eta * w)
        P.run(st, 1)                                   # the check itself
        e = st["log"][-1]
        assert e["t"] == t_check
        dz = np.concatenate([x - o["xh"], y - o["yh"]])
        Pm = np.block([[w / P.eta * np.eye(lp.n), At.T], [At, np.eye(lp.m) / (P.eta * w)]])
        assert np.isclose(e["r"], np.sqrt(dz @ Pm @ dz), rtol=1e-11), (e["r"], np.sqrt(dz @ Pm @ dz))


# -- A8: the restart rule, in both directions -------------------------------------
def _replay_restart_rule(log, beta_suf, beta_nec, beta_art):
    """Decisions of App. B.2 recomputed from each check's (t, k, r) alone:
    r0 is r at the epoch's k = 0 check, the 'previous' residual is the
    previous check of the same epoch, and the three tests run in the order
    sufficient, necessary, artificial."""
    out, r0, r_prev = [], None, None
    for e in log:
        if e["k"] == 0:
            r0, r_prev = e["r"], e["r"]
            out.append(0)
            continue
        r = e["r"]
        if r <= beta_suf * r0:
            kind = 1
        elif r <= beta_nec * r0 and r > r_prev:
            kind = 2
        elif e["k"] >= beta_art * e["t"]:
            kind = 3
        else:
            kind = 0
        out.append(kind)
        r_prev = r
    return out


@pytest.mark.parametrize("kw", [dict(), dict(beta_suf=0.5), dict(beta_nec=0.95),
                                dict(beta_art=0.1), dict(beta_suf=0.0, beta_nec=0.0)])
def test_restart_rule_both_directions(oracle_mod, kw):
    """Every check's decision, restart or not, equals the rule replayed from
    the logged residuals, so a rule that never fires one kind, or fires when
    it should not, fails.  The default constants fire all three kinds on
    config 0; the other constants move the thresholds."""
    prm = _prm(oracle_mod, max_iters=20000, **kw)
    lp = lpgen.config0()
    r = oracle_mod.Problem(lp, prm).solve()
    log = r["state"]["log"]
    want = _replay_restart_rule(log, prm.beta_suf, prm.beta_nec, prm.beta_art)
    if r["status"] == 1:
        want[-1] = 0                                   # the converged check
    assert [e["restart"] for e in log] == want
    if not kw:
        assert {1, 2, 3} <= set(want)
    # after a restart the next iteration opens an epoch with a check
    for a, b in zip(log, log[1:]):
        if a["restart"]:
            assert b["k"] == 0 and b["t"] == a["t"] + 1


def test_restart_rule_forced_firing(oracle_mod):
    """Constants that force each kind: beta_art = 0 restarts at every check
    after an epoch's first (artificial unless a decay test fired first);
    beta_suf = 1e9 makes every such check a sufficient-decay restart."""
    lp = lpgen.config0()
    for kw, kind in ((dict(beta_suf=0.0, beta_nec=0.0, beta_art=0.0), 3),
                     (dict(beta_suf=1e9), 1)):
        r = oracle_mod.Problem(lp, _prm(oracle_mod, max_iters=2000, eps=0.0, **kw)).solve()
        log = r["state"]["log"]
        assert len(log) > 10
        for e in log:
            assert e["restart"] == (0 if e["k"] == 0 else kind), (kw, e)


# -- start point: scaled, clamped into X, projected onto Y (Sec. 2.1) -------------
def test_init_state_projects_the_given_start(oracle_mod):
    """A given (x0, y0) is mapped to the scaled space and projected: x onto
    the box, y onto Y_i of Sec. 2.1 per row type ({0} free, R- '<=' only,
    R+ '>=' only, R with both bounds finite, '=' and ranged)."""
    lp = _mixed_bounds_lp(5)
    P = oracle_mod.Problem(lp)
    d = P.scaled()
    rng = np.random.default_rng(6)
    x0 = 10.0 * rng.standard_normal(lp.n)
    y0 = 5.0 * rng.standard_normal(lp.m)
    st = P.init_state(x0, y0)
    x_want = np.clip(x0, lp.var_lo, lp.var_hi) / d["dc"]
    lo_f, hi_f = np.isfinite(lp.con_lo), np.isfinite(lp.con_hi)
    y_proj = np.where(lo_f & hi_f, y0, np.where(lo_f, np.maximum(y0, 0.0),
                                               np.where(hi_f, np.minimum(y0, 0.0), 0.0)))
    y_want = y_proj / d["dr"]
    assert np.allclose(st["x"], x_want, rtol=1e-15, atol=0)
    assert np.allclose(st["y"], y_want, rtol=1e-15, atol=0)
    assert np.array_equal(st["xa"], st["x"]) and np.array_equal(st["ya"], st["y"])
    # every row type and both signs of y0 occur, so each branch is exercised
    for lo_ok, hi_ok in ((True, True), (True, False), (False, True), (False, False)):
        rows = (lo_f == lo_ok) & (hi_f == hi_ok)
        assert np.any(rows & (y0 > 0)) and np.any(rows & (y0 < 0))
    S = st["state"]
    assert S.omega == P.omega0 and S.k == 0 and S.t == 0 and S.restarts == 0
    # no start given: the origin projected (0 inside every box here but the
    # lower-only boxes [-3, inf) and the free ones contain 0 too)
    st0 = P.init_state()
    assert np.array_equal(st0["x"], np.clip(0.0, d["vlo"], d["vhi"]))
    assert np.all(st0["y"] == 0.0)
