"""Plain-Python oracle of the distributed method's cost model.

TEST INFRASTRUCTURE ONLY: the reference the library's host functions
``dpdlp_cost_step``, ``dpdlp_grid_select`` and ``dpdlp_auto_devices`` are
checked against.  The library never imports it.

* ``t_step`` is the per-iteration time model of Sec. 3.3, with its four
  terms as App. E.2 derives them (matrix stream, vector traffic, ring
  all-reduce payload, topology latency), in seconds.
* ``grid`` is the grid choice of Sec. 4.1: among the factor pairs
  R x C = N, the one whose R / C is closest to m / n.  The paper does not say
  how closeness is measured.  A plain difference |R/C - m/n| would give a
  1 x 4 grid for the sdm instance of App. E.4, which the paper runs on
  2 x 2; the log-ratio |log(R/C) - log(m/n)| reproduces every grid of
  App. E.4.  Ties (equal up to 1e-12) take the smaller R.
* ``auto`` is the AUTO rule of Sec. 5.1: evaluate the model for each
  candidate count on its grid and keep the fastest (ties: fewer devices).

Parameters follow App. E.3.  The paper's hardware values are H100's:
b_mem 3350 GB/s, b_net 450 GB/s (Sec. 5.1 prints 400 GB/s; the worked
examples of App. E.4 use 450), beta_sync 10 us, n_hop 1; c_spmv 24, c_vec 90,
c_net 8 bytes.
"""
from __future__ import annotations

import math

H100 = dict(b_mem=3350e9, b_net=450e9, beta_sync=10e-6, n_hop=1.0,
            c_spmv=24.0, c_vec=90.0, c_net=8.0)


def t_step(m, n, nnz, R, C, b_mem, b_net, beta_sync, n_hop, c_spmv, c_vec, c_net):
    """The four terms of the per-iteration model and their sum (seconds)."""
    N = R * C
    spmv = c_spmv * nnz / (b_mem * N)
    vec = c_vec / b_mem * (n / C + m / R)
    net = c_net / b_net * ((n * R + m * C - (m + n)) / N)
    sync = n_hop * beta_sync * ((1 if R > 1 else 0) + (1 if C > 1 else 0))
    return dict(spmv=spmv, vec=vec, net=net, sync=sync, total=spmv + vec + net + sync)


def grid(m, n, N):
    best = None
    for R in range(1, N + 1):
        if N % R:
            continue
        C = N // R
        d = abs(math.log(R / C) - math.log(m / n))
        if best is None or d < best[0] - 1e-12:      # near-ties keep the smaller R
            best = (d, R, C)
    return best[1], best[2]


def auto(m, n, nnz, counts=(1, 2, 4, 8), **hw):
    best = None
    for N in counts:
        R, C = grid(m, n, N)
        t = t_step(m, n, nnz, R, C, **hw)["total"]
        if best is None or t < best[0] or (t == best[0] and N < best[1]):
            best = (t, N, R, C)
    return dict(ndev=best[1], R=best[2], C=best[3], t_step=best[0])
