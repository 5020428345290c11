"""Pins of the FP64 reference of the warm-start network (CPU only): its
gradient against central finite differences of its own loss, and closed
forms (zero heads return the reference point; zero loss at the target)."""
import numpy as np
import pytest
import scipy.sparse as sp

import lpgen
from oracle import gnn_ref


def _setup(layers=2, seed=0):
    base = lpgen.constructed_lp(20, 30, 10, 3, seed=seed)
    inst = lpgen.perturbed(base, seed + 100)
    rng = np.random.default_rng(seed)
    dr = rng.uniform(0.5, 2.0, base.m)
    dc = rng.uniform(0.5, 2.0, base.n)
    A = (sp.diags(dr) @ base.scipy_csr() @ sp.diags(dc)).tocsr()
    b_ref = gnn_ref.row_b(base.con_lo, base.con_hi)
    Xc, Xr = gnn_ref.features(inst.c, inst.con_lo, inst.con_hi, inst.var_lo, inst.var_hi,
                              base.c, b_ref, base.x_star, base.y_star, dr, dc)
    p = 0.08 * rng.standard_normal(gnn_ref.n_params(layers))
    tx = rng.standard_normal(base.n)
    ty = rng.standard_normal(base.m)
    return A, Xc, Xr, base.x_star / dc, base.y_star / dr, tx, ty, p


def test_gradient_matches_finite_differences():
    layers = 2
    A, Xc, Xr, xs, ys, tx, ty, p = _setup(layers)
    L0, g = gnn_ref.loss_and_grad(p, layers, A, Xc, Xr, xs, ys, tx, ty)
    rng = np.random.default_rng(7)
    idx = rng.choice(p.size, 60, replace=False)
    idx = np.concatenate([idx, [p.size - 1, p.size - 129, 0, 2 * 16 * 128]])
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        Lp, _ = gnn_ref.loss_and_grad(pp, layers, A, Xc, Xr, xs, ys, tx, ty)
        Lm, _ = gnn_ref.loss_and_grad(pm, layers, A, Xc, Xr, xs, ys, tx, ty)
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-5 * (abs(fd) + abs(g[i])) + 1e-8, (i, fd, g[i])


def test_zero_heads_return_reference_and_pack_roundtrip():
    layers = 3
    A, Xc, Xr, xs, ys, tx, ty, p = _setup(layers, seed=1)
    d = gnn_ref.unpack(p, layers)
    d["w_x"][:] = 0
    d["w_y"][:] = 0
    q = gnn_ref.pack(d)
    assert q.size == gnn_ref.n_params(layers)
    px, py, _ = gnn_ref.forward(q, layers, A, Xc, Xr, xs, ys)
    assert np.array_equal(px, xs) and np.array_equal(py, ys)
    L, g = gnn_ref.loss_and_grad(q, layers, A, Xc, Xr, xs, ys, xs, ys)
    assert L == 0.0 and not np.any(g)
