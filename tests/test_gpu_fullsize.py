"""Parity at the full sizes of the benchmark workloads, in the launch
configuration bench.py times (default parameters: 2048-nonzero tiles, XCD
remap on, block permutation B = 256, automatic XCD slicing, which slices
c1's dual step), plus slicing off and slicing of both steps.

c1 (m 2M, n 4M, 40M nonzeros), c2 (m 6000, n 9M, 18M nonzeros), c1 in the
FP32-mixed form (c3) and the LASSO QP of the benchmark (m 2M, n 2M, 22.9M
nonzeros): both sides run the first iterations from the same start with the
same eta and omega0 (the step size comes from a short power estimate of the
oracle, so no oracle input comes from the GPU); the oracle computes every
output, and all of them are compared: the iterate, the anchor, T(z), the
restart log and the KKT values of the check iterations."""
import functools

import numpy as np
import pytest

import lpgen

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module")
def D():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    import paper_2601_07628_amd as D
    return D


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@functools.lru_cache(maxsize=1)
def _oracle_run(name, n_iters):
    """The oracle's first n_iters iterations on a benchmark workload, with
    the step size from a short power estimate (kept for the next test)."""
    import oracle
    lp = {"c1": lpgen.config1, "c2": lpgen.config2, "staircase": lpgen.config1_staircase,
          "lasso": lambda: lpgen.lasso_qp(1_000_000, 500_000, 20, seed=7)}[name]()
    P0 = oracle.Problem(lp, oracle.Params(eta=1.0, omega0=0.0, eps=0.0))
    sig, _ = P0.sigma_max_power(max_iters=8, tol=0.0)
    eta, w0 = 0.9 / sig, P0.omega0
    del P0
    P = oracle.Problem(lp, oracle.Params(eta=eta, omega0=w0, eps=0.0))
    st = P.init_state()
    P.run(st, n_iters)
    del P
    return lp, eta, w0, st


def _gpu_run(D, lp, eta, w0, n_iters, **kw):
    prm = D.dpdlp_params_default()
    prm.eta, prm.omega0, prm.eps = eta, w0, 0.0
    for k, v in kw.items():
        setattr(prm, k, v)
    G = D.Problem(lp, prm)
    G.init()
    G.iterate(n_iters)
    return G, G.state()


def _fullsize(D, name, n_iters, slices=0):
    lp, eta, w0, st = _oracle_run(name, n_iters)
    G, gs = _gpu_run(D, lp, eta, w0, n_iters, gather_slices=slices)
    for k in ("x", "y", "xa", "ya", "xh", "yh"):
        assert rel(gs[k], st[k]) <= 1e-10, (k, rel(gs[k], st[k]))
        scale = max(np.abs(st[k]).max(initial=0.0), 1e-300)
        assert np.abs(gs[k] - st[k]).max(initial=0.0) <= 1e-10 * scale, (k, "element-wise")
    lg, lo = G.log(), st["log"]
    assert len(lg) == len(lo) and len(lo) >= 1
    for g, o in zip(lg, lo):
        assert g["t"] == o["t"] and g["k"] == o["k"] and g["restart"] == o["restart"]
        for q in ("r_primal", "r_dual", "r_gap", "r"):
            assert abs(g[q] - o[q]) <= 1e-9 * abs(o[q]) + 1e-300, (q, g[q], o[q])
    assert abs(gs["scalars"]["omega"] - st["state"].omega) <= 1e-9 * st["state"].omega


@pytest.mark.parametrize("slices", [0, -1, 8])
def test_c1_fullsize_parity(D, slices):
    """The first 140 iterations of c1 (checks at t = 0, 63 and 127; the
    iterations between checks replayed as HIP graphs), with slicing off,
    automatic and forced on both steps."""
    _fullsize(D, "c1", 140, slices)


def test_c3_fullsize_fp32_mixed_against_fp64_oracle(D):
    """c3: the FP32-mixed form on the full c1 instance against the FP64
    oracle over the same 140 iterations, held in FP32 (switch rule off):
    the same restart decisions, and T(z) within 1e-5 relative (FP32
    rounding of A~, of the iterates and of the sums, about 6e-8 each; the
    measured error is printed)."""
    lp, eta, w0, st = _oracle_run("c1", 140)
    G, gs = _gpu_run(D, lp, eta, w0, 140, precision=D.FP32_MIXED, fp32_switch_tol=0.0,
                     fp32_stall_checks=10**6, fp32_diverge=0.0)
    r = G.result(want_xy=False)
    assert r["fp32_iters"] == 140
    lg, lo = G.log(), st["log"]
    assert [(e["t"], e["k"], e["restart"]) for e in lg] == \
        [(e["t"], e["k"], e["restart"]) for e in lo]
    errs = {k: rel(gs[k], st[k]) for k in ("xh", "yh")}
    kkt = [abs(g[q] - o[q]) / o[q] for g, o in zip(lg, lo) for q in ("r_primal", "r_dual", "r_gap")]
    print(f"c3 (FP32-mixed) vs FP64 oracle after 140 iterations: {errs}; "
          f"KKT values within {max(kkt):.2e} relative")
    assert max(errs.values()) <= 1e-5, errs
    assert max(kkt) <= 1e-2


def test_staircase_fullsize_parity(D):
    """The 40M-nonzero staircase LP that bench.py solves to 1e-8: 140
    iterations with the default parameters (its dual step sliced)."""
    _fullsize(D, "staircase", 140, -1)


def test_c2_fullsize_parity(D):
    """100 iterations of the transportation LP (checks at t = 0 and 63)."""
    _fullsize(D, "c2", 100)


def test_lasso_qp_fullsize_parity(D):
    """The diagonal QP at the size bench.py times (the LASSO of App. J on
    1M samples x 500k features, 22.9M nonzeros; default parameters),
    70 iterations: one full check block plus the next check."""
    _fullsize(D, "lasso", 70, -1)


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
def test_c2_solves_to_1e8_at_the_oracle_objective(D, precision):
    """The transportation LP solved to relative KKT 1e-8 (App. B.4) with the
    default parameters, in FP64 and in FP32-mixed form, reaches the FP64
    oracle's objective at 1e-8 (tests/golden/oracle_objectives.json, written
    by make_oracle_objectives.py from the oracle alone).  Both points have a
    relative gap and relative residuals of at most 1e-8, so their objectives
    differ by a few times 1e-8 (1 + |obj|) at most; the bar is 1e-7."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "oracle_objectives.json")) as f:
        ref = json.load(f)["c2"]
    lp = lpgen.config2()
    prm = D.dpdlp_params_default()
    prm.eps = 1e-8
    if precision == "fp32_mixed":
        prm.precision = D.FP32_MIXED
    G = D.Problem(lp, prm)
    r = G.solve()
    assert r["status"] == D.CONVERGED
    assert max(r["r_primal"], r["r_dual"], r["r_gap"]) <= 1e-8
    # the automatic rule slices the dual step (x-bar, 72 MB) in both
    # precisions and leaves the primal step (y, 48 KB) unsliced
    assert (r["slices_primal"], r["slices_dual"]) == (0, 8)
    err = abs(r["obj_primal"] - ref["obj_primal"]) / (1 + abs(ref["obj_primal"]))
    print(f"c2 {precision}: {r['iters']} iterations ({r['fp32_iters']} in FP32), objective "
          f"{r['obj_primal']:.10g} against the oracle's {ref['obj_primal']:.10g} "
          f"(relative {err:.2e})")
    assert err <= 1e-7, err
    if precision == "fp64":
        # the same method to the same tolerance (the step sizes differ
        # slightly: Lanczos on the GPU, power iteration in the oracle)
        assert abs(r["iters"] - ref["iters"]) <= 0.25 * ref["iters"], (r["iters"], ref["iters"])


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
def test_c1_solves_to_1e4_at_the_oracle_objective(D, precision):
    """c1, and c3 (its FP32-mixed form), solved to relative KKT 1e-4 with the
    default parameters, reach the objective of the oracle's own 1e-4 solve
    (tests/golden/oracle_objectives.json).  Two points at 1e-4 each have a
    relative gap and residuals of at most 1e-4, so the bar is the other
    solve tests' 10 eps (1 + |obj|); measured: 2.3e-6 (FP64, the same 7,296
    iterations as the oracle) and 2.5e-4 (FP32-mixed)."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "oracle_objectives.json")) as f:
        ref = json.load(f)["c1"]
    lp = lpgen.config1()
    prm = D.dpdlp_params_default()
    prm.eps = 1e-4
    prm.time_limit = 60.0
    if precision == "fp32_mixed":
        prm.precision = D.FP32_MIXED
    G = D.Problem(lp, prm)
    r = G.solve()
    assert r["status"] == D.CONVERGED
    assert max(r["r_primal"], r["r_dual"], r["r_gap"]) <= 1e-4
    err = abs(r["obj_primal"] - ref["obj_primal"]) / (1 + abs(ref["obj_primal"]))
    print(f"c1 {precision} to 1e-4: {r['iters']} iterations ({r['fp32_iters']} in FP32), "
          f"objective {r['obj_primal']:.10g} against the oracle's {ref['obj_primal']:.10g} "
          f"(relative {err:.2e})")
    assert err <= 10 * 1e-4, err


@pytest.mark.parametrize("name,n_iters", [("lasso", 70), ("c2", 100)])
def test_fullsize_fp32_mixed_against_fp64_oracle(D, name, n_iters):
    """The LASSO QP and c2 at full size in the FP32-mixed form, held in FP32
    (c2's dual step sliced, as in FP64), against the FP64 oracle over the
    iterations of their FP64 parity tests: the same restart decisions and
    T(z) within 1e-5 relative, the bar of the c3 test (FP32 rounding of A~,
    the iterates and the sums, about 6e-8 per operation)."""
    lp, eta, w0, st = _oracle_run(name, n_iters)
    G, gs = _gpu_run(D, lp, eta, w0, n_iters, gather_slices=-1, precision=D.FP32_MIXED,
                     fp32_switch_tol=0.0, fp32_stall_checks=10**6, fp32_diverge=0.0)
    assert G.result(want_xy=False)["fp32_iters"] == n_iters
    lg, lo = G.log(), st["log"]
    assert [(e["t"], e["k"], e["restart"]) for e in lg] == \
        [(e["t"], e["k"], e["restart"]) for e in lo]
    errs = {k: rel(gs[k], st[k]) for k in ("xh", "yh")}
    print(f"{name} (FP32-mixed) vs FP64 oracle after {n_iters} iterations: {errs}")
    assert max(errs.values()) <= 1e-5, errs
