"""GPU parity of the diagonal-QP extension (Sec. 6) against the CPU oracle.

The primal step minimises the separable quadratic subproblem over the box in
closed form; the KKT evaluation carries Q x and the half-quadratic objective
terms.  Inputs: the constructed QP (an LP optimum with c shifted by -Q x*)
and the LASSO of App. J on a synthetic sparse feature matrix.  Bars as in
the LP parity tests: iterates within 1e-10 (relative 2-norm) after a fixed
number of iterations from the same start and step sizes, identical restart
decisions, solves to the stated KKT tolerance.
"""
import dataclasses

import numpy as np
import pytest

import lpgen
from tests.test_gpu_parity import D, O, fixed_run, gpu_params, rel  # noqa: F401 (fixtures)

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("slices", [0, 8])
def test_qp_iterate_parity_constructed(D, O, slices):
    lp = lpgen.constructed_qp(2000, 4000, 1000, 5, seed=21)
    fixed_run(D, O, lp, 500, gpu_kw=dict(gather_slices=slices))


@pytest.mark.parametrize("slices", [0, 16])
def test_qp_iterate_parity_lasso(D, O, slices):
    """LASSO rows hold one sample's features plus -1 for its residual; the
    features' popularity is Zipf-like, so some columns are long."""
    lp = lpgen.lasso_qp(3000, 1500, 12, seed=4)
    fixed_run(D, O, lp, 400, gpu_kw=dict(gather_slices=slices))


def test_qp_kkt_matches_oracle(D, O):
    lp = lpgen.constructed_qp(2000, 4000, 1000, 5, seed=22)
    G = D.Problem(lp, gpu_params(D))
    P = O.Problem(lp)
    rng = np.random.default_rng(1)
    ge = np.isinf(lp.con_hi)              # '>=' rows: y >= 0 keeps the dual objective finite
    for _ in range(3):
        x = rng.uniform(0, 10, lp.n)
        y = rng.standard_normal(lp.m)
        y[ge] = np.abs(y[ge])
        for tau in (0.01, 1.0):
            g = G.kkt(x, y, tau=tau)
            o = P.kkt(x, y, tau=tau)
            for i in range(5):
                assert abs(g[i] - o[i]) <= 1e-11 * (1 + abs(o[i])), (i, g[i], o[i])
    # zero at the constructed optimum; without Q the same point is not optimal
    k = G.kkt(lp.x_star, lp.y_star, tau=1.0)
    assert max(k[0], k[1], k[2]) < 1e-12
    G.set_objective_diag(None)
    assert G.kkt(lp.x_star, lp.y_star, tau=1.0)[1] > 1e-3


def test_qp_solves_to_constructed_optimum(D, O):
    lp = lpgen.constructed_qp(2000, 4000, 1000, 5, seed=23)
    r = D.Problem(lp, gpu_params(D, eps=1e-8)).solve()
    assert r["status"] == D.CONVERGED
    assert max(r["r_primal"], r["r_dual"], r["r_gap"]) <= 1e-8
    assert abs(r["obj_primal"] - lp.obj_star) <= 1e-6 * (1 + abs(lp.obj_star))
    o = O.Problem(lp, O.Params(eps=1e-8)).solve()
    assert abs(r["obj_primal"] - o["obj_p"]) <= 1e-6 * (1 + abs(o["obj_p"]))


def test_lasso_solve_matches_oracle_objective(D, O):
    """LASSO at the paper's tolerance 1e-6 (App. J): the LASSO objective of
    the GPU's x agrees with the oracle's."""
    lp = lpgen.lasso_qp(3000, 1500, 12, seed=5)
    A, b, lam = lp.lasso["A"], lp.lasso["b"], lp.lasso["lam"]
    f = lambda v: 0.5 * float(np.sum((A @ v - b) ** 2)) + lam * float(np.abs(v).sum())
    r = D.Problem(lp, gpu_params(D, eps=1e-6, max_iters=400_000)).solve()
    assert r["status"] == D.CONVERGED
    o = O.Problem(lp, O.Params(eps=1e-6)).solve(max_iters=400_000)
    assert o["status"] == 1
    nf = A.shape[1]
    fg, fo = f(r["x"][:nf]), f(o["x"][:nf])
    assert abs(fg - fo) <= 1e-4 * (1 + abs(fo))


def test_qp_off_again_is_the_lp(D, O):
    """Setting diag(Q) and removing it gives the LP's iterates bit for bit."""
    lp = lpgen.constructed_qp(500, 1000, 250, 4, seed=24)
    plain = dataclasses.replace(lp, q=None)
    G1 = D.Problem(plain, gpu_params(D))
    G1.init()
    G1.iterate(200)
    G2 = D.Problem(lp, gpu_params(D))
    G2.set_objective_diag(None)
    G2.init()
    G2.iterate(200)
    s1, s2 = G1.state(), G2.state()
    for k in ("x", "y"):
        assert np.array_equal(s1[k], s2[k])


def test_qp_argument_errors(D):
    lp = lpgen.constructed_qp(100, 200, 50, 3, seed=25)
    G = D.Problem(lp, gpu_params(D))
    bad = lp.q.copy()
    bad[3] = -1.0
    with pytest.raises(RuntimeError, match="diag"):
        G.set_objective_diag(bad)
    bad[3] = np.nan
    with pytest.raises(RuntimeError, match="diag"):
        G.set_objective_diag(bad)
    with pytest.raises(ValueError):
        G.set_objective_diag(lp.q[:-1])


@pytest.mark.parametrize("name,maker", [
    ("constructed-qp", lambda: lpgen.constructed_qp(2000, 4000, 1000, 5, seed=26)),
    ("lasso", lambda: lpgen.lasso_qp(3000, 1500, 12, seed=6))])
def test_qp_fp32_mixed_iterates_against_fp64_oracle(D, O, name, maker):
    """FP32-mixed QP iterates against the FP64 oracle after one 64-iteration
    epoch from the same start and step sizes, to the FP32 bar of the LP
    tests (1e-5 relative)."""
    lp = maker()
    P0 = O.Problem(lp)
    eta, w0 = P0.eta, P0.omega0
    P = O.Problem(lp, O.Params(eta=eta, omega0=w0, eps=0.0))
    st = P.init_state()
    P.run(st, 64)
    G = D.Problem(lp, gpu_params(D, eta=eta, omega0=w0, eps=0.0, precision=D.FP32_MIXED,
                                 fp32_switch_tol=0.0, fp32_stall_checks=10**6, fp32_diverge=0.0))
    G.init()
    G.iterate(64)
    gs = G.state()
    assert [e["restart"] for e in G.log()] == [e["restart"] for e in st["log"]]
    errs = {k: rel(gs[k], st[k]) for k in ("xh", "yh")}
    print(f"{name}: FP32-mixed QP vs FP64 oracle after 64 iterations: {errs}")
    assert max(errs.values()) <= 1e-5, errs


def test_qp_fp32_mixed_solves_to_1e8(D, O):
    lp = lpgen.constructed_qp(2000, 4000, 1000, 5, seed=27)
    r = D.Problem(lp, gpu_params(D, eps=1e-8, precision=D.FP32_MIXED)).solve()
    assert r["status"] == D.CONVERGED
    assert max(r["r_primal"], r["r_dual"], r["r_gap"]) <= 1e-8
    assert r["fp32_iters"] > 0
    assert abs(r["obj_primal"] - lp.obj_star) <= 1e-6 * (1 + abs(lp.obj_star))


def test_qp_diag_from_device_memory(D):
    """diag(Q) handed over as device memory gives the same iterates as the
    host copy."""
    import torch
    lp = lpgen.constructed_qp(500, 1000, 250, 4, seed=28)
    G1 = D.Problem(lp, gpu_params(D))
    G1.init()
    G1.iterate(150)
    G2 = D.Problem(lp, gpu_params(D), q=False)
    qd = torch.tensor(lp.q, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    rc = D.lib().dpdlp_set_objective_diag(G2.h, qd.data_ptr(), D.MEM_DEVICE, None)
    assert rc == 0, D.dpdlp_last_error()
    G2.init()
    G2.iterate(150)
    s1, s2 = G1.state(), G2.state()
    for k in ("x", "y", "xh", "yh"):
        assert np.array_equal(s1[k], s2[k])


def test_qp_set_mid_run_matches_oracle(D, O):
    """diag(Q) set after 100 LP iterations takes effect from the next
    iteration (the replayed graph of the LP step is dropped): 100 more
    iterations match the oracle, which switches at the same point."""
    lp = lpgen.constructed_qp(1000, 2000, 500, 4, seed=29)
    plain = dataclasses.replace(lp, q=None)
    P0 = O.Problem(plain)
    eta, w0 = P0.eta, P0.omega0
    P = O.Problem(plain, O.Params(eta=eta, omega0=w0, eps=0.0))
    st = P.init_state()
    P.run(st, 100)
    O.lib().ora_set_qdiag(P._h, lp.q.ctypes.data)
    P.run(st, 100)
    G = D.Problem(plain, gpu_params(D, eta=eta, omega0=w0, eps=0.0))
    G.init()
    G.iterate(100)
    G.set_objective_diag(lp.q)
    G.iterate(100)
    gs = G.state()
    for k in ("x", "y", "xh", "yh"):
        assert rel(gs[k], st[k]) <= 1e-10, (k, rel(gs[k], st[k]))
