"""Parity at the full sizes of the benchmark workloads, in the launch
configuration bench.py times (default parameters: 2048-nonzero tiles, XCD
remap on, block permutation B = 256, automatic XCD slicing, which slices
c1's dual step), plus slicing off and slicing of both steps.

c1 (m 2M, n 4M, 40M nonzeros), c2 (m 6000, n 9M, 18M nonzeros) and the
LASSO QP of the benchmark (m 2M, n 2M, 22.9M nonzeros): both
sides run the first iterations from the same start with the same eta and
omega0 (the step size comes from a short power estimate of the oracle, so no
oracle input comes from the GPU); the oracle computes every output, and all
of them are compared: the iterate, the anchor, T(z), the restart log and the
KKT values of the check iterations."""
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


def _fullsize(D, lp, n_iters, slices=0):
    import oracle
    P0 = oracle.Problem(lp, oracle.Params(eta=1.0, omega0=0.0, eps=0.0))
    sig, _ = P0.sigma_max_power(max_iters=8, tol=0.0)
    eta, w0 = 0.9 / sig, P0.omega0
    del P0
    P = oracle.Problem(lp, oracle.Params(eta=eta, omega0=w0, eps=0.0))
    st = P.init_state()
    P.run(st, n_iters)
    prm = D.dpdlp_params_default()
    prm.eta, prm.omega0, prm.eps, prm.gather_slices = eta, w0, 0.0, slices
    G = D.Problem(lp, prm)
    G.init()
    G.iterate(n_iters)
    gs = G.state()
    for k in ("x", "y", "xa", "ya", "xh", "yh"):
        assert rel(gs[k], st[k]) <= 1e-10, (k, rel(gs[k], st[k]))
    lg, lo = G.log(), st["log"]
    assert len(lg) == len(lo) and len(lo) >= 1
    for g, o in zip(lg, lo):
        assert g["t"] == o["t"] and g["k"] == o["k"] and g["restart"] == o["restart"]
        for q in ("r_primal", "r_dual", "r_gap", "r"):
            assert abs(g[q] - o[q]) <= 1e-9 * abs(o[q]) + 1e-300, (q, g[q], o[q])


@pytest.mark.parametrize("slices", [0, -1, 8])
def test_c1_fullsize_parity(D, slices):
    _fullsize(D, lpgen.config1(), 3, slices)


def test_c1_fullsize_two_check_blocks_with_graph_replay(D):
    """140 iterations of c1 in the default configuration: checks at t = 0,
    63 and 127, and iterations 64..126 replayed as one HIP graph; every output
    and the restart log against the oracle."""
    _fullsize(D, lpgen.config1(), 140, -1)


def test_c2_fullsize_parity(D):
    _fullsize(D, lpgen.config2(), 3)


def test_lasso_qp_fullsize_parity(D):
    """The diagonal QP at the size bench.py times (the LASSO of App. J on
    1M samples x 500k features, 22.9M nonzeros; default parameters),
    70 iterations: one full check block plus the next check."""
    _fullsize(D, lpgen.lasso_qp(1_000_000, 500_000, 20, seed=7), 70, -1)
