"""FP64 numpy reference of the warm-start network (forward and gradient).

TEST INFRASTRUCTURE ONLY: the GPU library's BF16/MFMA training kernels are
checked against this.  It shares no code with the GPU library; the scaling
(D_r, D_c, A~) it uses comes from the CPU oracle's own preparation.

The warm start is not part of the D-PDLP paper (the paper takes (x0, y0) as
an input of Algorithm 1); the network is this project's design:

  column features  [c~, c~ - c~ref, x~ref, has_lo, has_hi, lo~ or 0, hi~ or 0, 1, 0 x 8]
  row features     [b~, b~ - b~ref, y~ref, is_eq, has_lo, has_hi, 0, 1, 0 x 8]
      with x~ = x / D_c, y~ = y / D_r, c~ = D_c c, b~ = D_r b, lo~ = lo / D_c
      clipped to [-1e4, 1e4], and b the finite lower bound, else the finite
      upper bound, else 0;
  H_c = relu(X_c W_cin), H_r = relu(X_r W_rin);
  per layer:  H_r = relu([H_r, A~ H_c] W_r),  H_c = relu([H_c, A~^T H_r] W_c);
  x~0 = x~ref + H_c w_x,  y~0 = y~ref + H_r w_y;
  loss = mean((x~0 - x~*)^2) + mean((y~0 - y~*)^2).
Parameter vector layout: W_cin [16x128], W_rin [16x128], per layer W_c
[256x128], W_r [256x128], then w_x [128], w_y [128].
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

H = 128
F = 16


def n_params(layers: int) -> int:
    return 2 * F * H + layers * 2 * (2 * H * H) + 2 * H


def unpack(p: np.ndarray, layers: int) -> dict:
    p = np.asarray(p, np.float64)
    o = 0

    def take(shape):
        nonlocal o
        k = int(np.prod(shape))
        out = p[o:o + k].reshape(shape)
        o += k
        return out

    d = {"W_cin": take((F, H)), "W_rin": take((F, H)), "W_c": [], "W_r": []}
    for _ in range(layers):
        d["W_c"].append(take((2 * H, H)))
        d["W_r"].append(take((2 * H, H)))
    d["w_x"] = take((H,))
    d["w_y"] = take((H,))
    assert o == p.size
    return d


def pack(d: dict) -> np.ndarray:
    parts = [d["W_cin"].ravel(), d["W_rin"].ravel()]
    for wc, wr in zip(d["W_c"], d["W_r"]):
        parts += [wc.ravel(), wr.ravel()]
    parts += [d["w_x"].ravel(), d["w_y"].ravel()]
    return np.concatenate(parts)


def row_b(lo, hi):
    return np.where(np.isfinite(lo), lo, np.where(np.isfinite(hi), hi, 0.0))


def features(c, con_lo, con_hi, var_lo, var_hi, c_ref, b_ref, x_ref, y_ref, dr, dc):
    n, m = c.size, con_lo.size
    Xc = np.zeros((n, F))
    Xc[:, 0] = dc * c
    Xc[:, 1] = dc * (c - c_ref)
    Xc[:, 2] = x_ref / dc
    flo, fhi = np.isfinite(var_lo), np.isfinite(var_hi)
    Xc[:, 3] = flo
    Xc[:, 4] = fhi
    Xc[:, 5] = np.where(flo, np.clip(np.where(flo, var_lo, 0) / dc, -1e4, 1e4), 0.0)
    Xc[:, 6] = np.where(fhi, np.clip(np.where(fhi, var_hi, 0) / dc, -1e4, 1e4), 0.0)
    Xc[:, 7] = 1.0
    b = row_b(con_lo, con_hi)
    Xr = np.zeros((m, F))
    Xr[:, 0] = dr * b
    Xr[:, 1] = dr * (b - b_ref)
    Xr[:, 2] = y_ref / dr
    glo, ghi = np.isfinite(con_lo), np.isfinite(con_hi)
    Xr[:, 3] = glo & ghi & (con_lo == con_hi)
    Xr[:, 4] = glo
    Xr[:, 5] = ghi
    Xr[:, 7] = 1.0
    return Xc, Xr


def relu(z):
    return np.maximum(z, 0.0)


def forward(p, layers, A: sp.csr_matrix, Xc, Xr, xref_s, yref_s, rnd=None):
    """rnd (optional) is applied to every stored activation (H and the
    products S), e.g. a rounding to the storage format of an implementation;
    the gradient then treats it as the identity."""
    rnd = rnd or (lambda v: v)
    W = unpack(p, layers)
    At = A.T.tocsr()
    cache = {"INc": [], "INr": [], "Hc": [], "Hr": []}
    Hc = rnd(relu(Xc @ W["W_cin"]))
    Hr = rnd(relu(Xr @ W["W_rin"]))
    cache["Hc0"], cache["Hr0"] = Hc, Hr
    for l in range(layers):
        INr = np.hstack([Hr, rnd(A @ Hc)])
        Hr = rnd(relu(INr @ W["W_r"][l]))
        INc = np.hstack([Hc, rnd(At @ Hr)])
        Hc = rnd(relu(INc @ W["W_c"][l]))
        cache["INr"].append(INr)
        cache["INc"].append(INc)
        cache["Hr"].append(Hr)
        cache["Hc"].append(Hc)
    px = xref_s + Hc @ W["w_x"]
    py = yref_s + Hr @ W["w_y"]
    return px, py, cache


def loss_and_grad(p, layers, A: sp.csr_matrix, Xc, Xr, xref_s, yref_s, tx_s, ty_s, rnd=None):
    """Loss and its gradient with respect to the flat parameter vector."""
    W = unpack(p, layers)
    At = A.T.tocsr()
    px, py, cache = forward(p, layers, A, Xc, Xr, xref_s, yref_s, rnd)
    n, m = px.size, py.size
    rx, ry = px - tx_s, py - ty_s
    loss = (rx @ rx) / n + (ry @ ry) / m
    dpx, dpy = 2 * rx / n, 2 * ry / m
    G = {"W_c": [None] * layers, "W_r": [None] * layers}
    Hc_L, Hr_L = cache["Hc"][-1], cache["Hr"][-1]
    G["w_x"] = Hc_L.T @ dpx
    G["w_y"] = Hr_L.T @ dpy
    dHc = np.outer(dpx, W["w_x"])
    dHr = np.outer(dpy, W["w_y"])
    for l in range(layers - 1, -1, -1):
        Hc, Hr = cache["Hc"][l], cache["Hr"][l]
        INc, INr = cache["INc"][l], cache["INr"][l]
        dZc = dHc * (Hc > 0)
        G["W_c"][l] = INc.T @ dZc
        dINc = dZc @ W["W_c"][l].T
        dHr = dHr + A @ dINc[:, H:]             # S_c = A~^T H_r
        dZr = dHr * (Hr > 0)
        G["W_r"][l] = INr.T @ dZr
        dINr = dZr @ W["W_r"][l].T
        dHc = dINc[:, :H] + At @ dINr[:, H:]    # S_r = A~ H_c
        dHr = dINr[:, :H]
    dZc0 = dHc * (cache["Hc0"] > 0)
    dZr0 = dHr * (cache["Hr0"] > 0)
    G["W_cin"] = Xc.T @ dZc0
    G["W_rin"] = Xr.T @ dZr0
    return loss, pack(G)
