"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Both sides get the same seeded inputs from lpgen and the same parameters
(eta and omega0 are passed explicitly where iterates are compared, so the two
power iterations' rounding cannot split the trajectories).  Bars:
  * iterates after a fixed number of iterations: relative 2-norm <= 1e-10
    (the GPU sums in a different order; PDHG is nonexpansive, so rounding
    differences stay at the 1e-15..1e-13 level over these runs);
  * the restart-decision log: identical decisions, except a decision whose r
    lies within 1e-9 r0 of its threshold (a tie); both sides are then run
    again up to the tied check and compared there in full;
  * solves: relative KKT <= eps, and the objective within the tolerance that
    eps implies of the oracle's.
"""
import numpy as np
import pytest

import lpgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    import paper_2601_07628_amd as D
    return D


@pytest.fixture(scope="module")
def O():
    import oracle
    oracle.lib()
    return oracle


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def oracle_params(O, **kw):
    return O.Params(**kw)


def gpu_params(D, **kw):
    p = D.dpdlp_params_default()
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def near_tie(e, beta_suf=0.2, beta_nec=0.8, beta_art=0.36):
    r, r0 = e["r"], e["r0"]
    tol = 1e-9 * max(r0, 1e-300)
    return (abs(r - beta_suf * r0) <= tol or abs(r - beta_nec * r0) <= tol)


def compare_logs(lg, lo):
    """Index of the first record whose restart decision differs at a near tie
    (None if the logs agree); any other difference fails."""
    n = min(len(lg), len(lo))
    for i in range(n):
        g, o = lg[i], lo[i]
        assert g["t"] == o["t"] and g["k"] == o["k"], (i, g, o)
        if g["restart"] != o["restart"]:
            assert near_tie(o), (i, g, o)
            return i
    assert len(lg) == len(lo)
    return None


def compare_iterates(gs, st, tol):
    """Iterates, anchors and T(z) against the oracle: relative 2-norm, and
    element by element (each entry within tol of the vector's largest
    entry), so one wrong small entry cannot hide in the norm."""
    for k in ("x", "y", "xa", "ya", "xh", "yh"):
        assert rel(gs[k], st[k]) <= tol, (k, rel(gs[k], st[k]))
        scale = max(np.abs(st[k]).max(initial=0.0), 1e-300)
        worst = np.abs(gs[k] - st[k]).max(initial=0.0)
        assert worst <= tol * scale, (k, "element-wise", worst / scale)
    assert gs["scalars"]["t"] == st["state"].t
    assert gs["scalars"]["k"] == st["state"].k
    # omega moves only at restarts, by log(dx/dy) with dx, dy the distances
    # of T(z) to the anchor.  Those distances are of the order of the KKT
    # error at that restart and are differences of iterates that agree to
    # about 1e-15 relative, so omega agrees to about 1e-15 / KKT (the bar
    # keeps a factor 10); where that floor exceeds 1e-2 the iterate has
    # converged to rounding level and omega follows rounding noise.
    rest = [e for e in st.get("log", []) if e["restart"]]
    if rest:
        floor = min(max(e["r_primal"], e["r_dual"], e["r_gap"]) for e in rest)
        tol_w = max(1e-9, 1e-14 / max(floor, 1e-300))
        if tol_w < 1e-2:
            w_g, w_o = gs["scalars"]["omega"], st["state"].omega
            assert abs(w_g - w_o) <= tol_w * w_o, ("omega", w_g, w_o, tol_w)


def fixed_run(D, O, lp, n_iters, gpu_kw=None, ora_kw=None, tol=1e-10, eps=0.0):
    """Run both sides n_iters iterations with shared eta/omega0 and compare
    the restart logs, the iterates and the primal weight.  If a restart
    decision differs at a near tie (r within 1e-9 r0 of a threshold), both
    sides are run again up to the iteration before the tied check and
    compared there in full, so a tie never skips the comparison; returns
    whether the whole run agreed.  With eps > 0 both sides stop at the
    check that reaches it (the same one, since the logs agree)."""
    P0 = O.Problem(lp)
    eta, w0 = P0.eta, P0.omega0
    ora_kw = dict(ora_kw or {})
    gkw = dict(eta=eta, omega0=w0, eps=eps)
    gkw.update(ora_kw)
    gkw.update(gpu_kw or {})

    def run_both(n):
        P = O.Problem(lp, oracle_params(O, eta=eta, omega0=w0, eps=eps, **ora_kw))
        st = P.init_state()
        P.run(st, n)
        G = D.Problem(lp, gpu_params(D, **gkw))
        G.init()
        G.iterate(n)
        return G, P, st, G.state()

    G, P, st, gs = run_both(n_iters)
    tie = compare_logs(G.log(), st["log"])
    if tie is None:
        compare_iterates(gs, st, tol)
        return G, P, st, gs, True
    t_tie = int(st["log"][tie]["t"])
    print(f"near tie at check {tie} (t = {t_tie}): compared up to t = {t_tie}")
    G, P, st, gs = run_both(t_tie)
    assert compare_logs(G.log(), st["log"]) is None
    compare_iterates(gs, st, tol)
    return G, P, st, gs, False


# ---- building blocks -----------------------------------------------------------
def test_scaling_matches_oracle(D, O):
    lp = lpgen.huge_share_lp(m=20000, n=40000, seed=7)
    G = D.Problem(lp, gpu_params(D, eta=1.0, omega0=1.0))
    P = O.Problem(lp, oracle_params(O, eta=1.0, omega0=1.0))
    sg, so = G.scaling(), P.scaled()
    assert rel(sg["dr"], so["dr"]) < 1e-13
    assert rel(sg["dc"], so["dc"]) < 1e-13


@pytest.mark.parametrize("transpose", [False, True])
@pytest.mark.parametrize("slices", [-1, 8, 16])
def test_spmv_matches_oracle(D, O, transpose, slices):
    """A~ v and A~^T v against the oracle, unsliced (the automatic rule does
    not slice this size) and through the sliced partial + combine kernels."""
    import torch
    lp = lpgen.huge_share_lp(m=30000, n=60000, seed=8)
    G = D.Problem(lp, gpu_params(D, eta=1.0, omega0=1.0, gather_slices=slices))
    P = O.Problem(lp, oracle_params(O, eta=1.0, omega0=1.0))
    rng = np.random.default_rng(0)
    v = rng.standard_normal(lp.m if transpose else lp.n)
    out = G.spmv(torch.from_numpy(v).cuda(), transpose=transpose).cpu().numpy()
    ref = P.spmv(v, transpose=transpose)
    # element-wise: each entry is the same sum in another order
    assert np.allclose(out, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("maker", [lpgen.config0,
                                   lambda: lpgen.huge_share_lp(m=2000, n=4000, seed=9),
                                   lambda: lpgen.transport_lp(40, 60, seed=3)])
@pytest.mark.parametrize("slices", [-1, 8])
def test_sigma_max_matches_dense_two_norm(D, O, maker, slices):
    """The Lanczos estimate of sigma_max(A~) against the 2-norm of the
    oracle's scaled matrix (dense SVD).  It is a lower bound (up to rounding)
    within 1e-5 (the step size keeps a 2e-3 margin; the scaled matrices
    have clustered top singular values, and c0's start vectors include one
    nearly orthogonal to the top singular vector), and at least as close as
    the oracle's power-iteration estimate."""
    lp = maker()
    G = D.Problem(lp, gpu_params(D, gather_slices=slices))
    P = O.Problem(lp)
    s = G.scaling()
    assert abs(s["omega0"] - P.omega0) <= 1e-12 * P.omega0
    d = P.scaled()
    import scipy.sparse as sp
    Ad = sp.csr_matrix((d["v"], lp.col_idx, lp.row_ptr), shape=(lp.m, lp.n)).toarray()
    ref = np.linalg.norm(Ad, 2)
    assert s["sigma_max"] <= ref * (1 + 1e-12), (s["sigma_max"], ref)
    assert s["sigma_max"] >= ref * (1 - 1e-5), (s["sigma_max"], ref)
    assert s["sigma_max"] >= P.sigma_max * (1 - 1e-12), (s["sigma_max"], P.sigma_max)
    G.init()
    r = G.result(want_xy=False)
    assert 2 <= r["power_iters"] <= 600


@pytest.mark.parametrize("slices", [-1, 8])
def test_kkt_matches_oracle(D, O, slices):
    """KKT triple and objectives, unsliced and through the sliced check
    passes (two-right-hand-side partials, combine with per-block sums)."""
    lp = lpgen.config0()
    G = D.Problem(lp, gpu_params(D, gather_slices=slices))
    P = O.Problem(lp)
    k = G.kkt(lp.x_star, lp.y_star, tau=0.5)
    assert max(k[:3]) < 1e-13
    rng = np.random.default_rng(1)
    x = np.clip(lp.x_star + rng.standard_normal(lp.n), 0, 10)
    y = lp.y_star + 0.1 * rng.standard_normal(lp.m)
    y[500:] = np.maximum(y[500:], 0)
    kg = G.kkt(x, y, tau=0.3)
    ko = P.kkt(x, y, tau=0.3)
    assert np.allclose(kg, ko, rtol=1e-11, atol=0)


# ---- fixed-iteration iterate parity ----------------------------------------------
@pytest.mark.parametrize("name,maker,n_iters", [
    ("c0", lpgen.config0, 1000),
    ("c4", lpgen.config4, 600),
    ("huge-share-small", lambda: lpgen.huge_share_lp(m=20000, n=40000, seed=9), 400),
    ("transport-60x4000", lambda: lpgen.transport_lp(60, 4000, seed=3), 400),
])
def test_iterate_parity(D, O, name, maker, n_iters):
    fixed_run(D, O, maker(), n_iters)


@pytest.mark.parametrize("name,maker", [
    ("c0-perturbed", lambda: lpgen.perturbed(lpgen.config0(), 7)),
    ("c4-member-384", lambda: lpgen.config4_family(384)),
])
def test_iterate_parity_10k(D, O, name, maker):
    """10,000 iterations with identical restart logs and iterates.  Members
    of the perturbed families are used because after 10,000 iterations their
    KKT error is still about 3e-7, far above rounding: the unperturbed c0 and
    c4 reach rounding level (1e-14 and 3e-13) after about 4,600 and 2,000
    iterations, where restart decisions are made by rounding noise."""
    _, _, st, _, same = fixed_run(D, O, maker(), 10_000)
    assert st["state"].t == 10_000 and sum(e["restart"] > 0 for e in st["log"]) >= 5


@pytest.mark.parametrize("name,maker,eps", [("c0", lpgen.config0, 1e-12),
                                            ("c4", lpgen.config4, 1e-11)])
def test_iterate_parity_to_tight_tolerance(D, O, name, maker, eps):
    """The unperturbed instances run to the tightest tolerance they reach
    above rounding level (up to 10,000 iterations); both sides stop at the
    same check with the same iterates."""
    _, _, st, _, same = fixed_run(D, O, maker(), 10_000, eps=eps)
    assert same and st["state"].status == 1


@pytest.mark.parametrize("name,maker,n_iters", [
    ("c0", lpgen.config0, 500),
    ("huge-share-small", lambda: lpgen.huge_share_lp(m=20000, n=40000, seed=9), 300),
    ("transport-60x4000", lambda: lpgen.transport_lp(60, 4000, seed=3), 300),
])
@pytest.mark.parametrize("slices", [8, 16])
@pytest.mark.parametrize("gsort", [0, 1])
def test_iterate_parity_xcd_sliced(D, O, name, maker, n_iters, slices, gsort):
    """The XCD-sliced fused steps (per-slice partial sums added in slice
    order), with each tile's nonzeros in storage order or sorted by gathered
    index (products put back in segment order in LDS), change only the
    summation order."""
    fixed_run(D, O, maker(), n_iters, gpu_kw=dict(gather_slices=slices, gather_sort=gsort))


def test_sliced_fp32_mixed_and_determinism(D, O):
    lp = lpgen.config4()
    kw = dict(precision=D.FP32_MIXED, gather_slices=8)
    r1 = D.Problem(lp, gpu_params(D, **kw)).solve()
    r2 = D.Problem(lp, gpu_params(D, **kw)).solve()
    assert r1["status"] == 1 and max(r1["r_primal"], r1["r_dual"], r1["r_gap"]) <= 1e-8
    assert np.array_equal(r1["x"], r2["x"]) and np.array_equal(r1["y"], r2["y"])
    o = O.Problem(lp).solve()
    assert abs(r1["obj_primal"] - o["obj_p"]) <= 1e-7 * (1 + abs(o["obj_p"]))


@pytest.mark.parametrize("remap,block,order", [(0, 256, 0), (1, 0, 0), (1, 256, 1), (1, 256, 2), (0, 0, 3)])
def test_iterate_parity_launch_variants(D, O, remap, block, order):
    """XCD remap off, permutation off and the hot-first order change only the
    summation order."""
    fixed_run(D, O, lpgen.config0(), 500,
              gpu_kw=dict(xcd_remap=remap, perm_block=block, perm_order=order))


@pytest.mark.parametrize("order,slices", [(1, -1), (2, -1), (3, -1), (3, 8)])
def test_hot_first_order_skewed_lp(D, O, order, slices):
    """Hot-first order on a Zipf-degree LP with heavy rows (config-1 shape at
    1/40 scale): the most frequent rows and columns move to the front, some
    columns split over tiles; with S = 8 slices the slices are unequal in
    nonzeros.  Iterates and restart log match the oracle."""
    lp = lpgen.huge_share_lp(50000, 100000, seed=11)
    fixed_run(D, O, lp, 200, gpu_kw=dict(perm_order=order, gather_slices=slices))


@pytest.mark.parametrize("block,slices", [(1, -1), (1, 16), (0, 8), (0, 16)])
def test_permutation_variants_skewed_lp(D, O, block, slices):
    """A full random permutation (blocks of 1) and no permutation, with XCD
    slicing, on a config-1 shaped LP at 1/40 scale: without a permutation
    the heavy rows fill the first slice of y.  Only the summation order
    changes."""
    lp = lpgen.huge_share_lp(50000, 100000, seed=11)
    fixed_run(D, O, lp, 200, gpu_kw=dict(perm_block=block, gather_slices=slices))


@pytest.mark.parametrize("block", [0, 1, 256])
def test_permutation_variants_staircase_lp(D, O, block):
    """The staircase LP (local gathers in the natural order) under each
    permutation, sliced into 8."""
    lp = lpgen.staircase_lp(20000, 40000, stages=40, per_col=10, seed=3)
    fixed_run(D, O, lp, 200, gpu_kw=dict(perm_block=block, gather_slices=8))


def test_perm_order_rejects_unknown(D):
    with pytest.raises(RuntimeError, match="perm_order"):
        D.Problem(lpgen.config0(), gpu_params(D, perm_order=4))


def test_split_segments_long_row_and_column(D, O):
    """A 9000-nonzero row and a 7000-nonzero column are split over several
    tiles (the last piece finishes the segment)."""
    rng = np.random.default_rng(5)
    m, n = 3000, 9000
    rows = [np.zeros(9000, np.int64), rng.integers(0, m, 30000)]
    cols = [np.arange(9000), rng.integers(0, n, 30000)]
    rows.append(np.arange(7000) % m)
    cols.append(np.full(7000, 17))
    r = np.concatenate(rows); c = np.concatenate(cols)
    key = np.unique(r * n + c)
    r, c = key // n, key % n
    A = np.zeros(0)
    vals = rng.standard_normal(r.size)
    import scipy.sparse as sp
    M = sp.csr_matrix((vals, (r, c)), shape=(m, n))
    M.sort_indices()
    lo = np.where(np.arange(m) % 2 == 0, -1.0, -np.inf)
    hi = np.where(np.arange(m) % 3 == 0, 1.0, np.inf)
    lp = lpgen.LP(m, n, M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data,
                  rng.standard_normal(n), lo, hi, -np.ones(n), np.ones(n), name="split")
    fixed_run(D, O, lp, 300)
    fixed_run(D, O, lp, 300, gpu_kw=dict(tile_nnz=512))
    fixed_run(D, O, lp, 300, gpu_kw=dict(tile_nnz=512, gather_slices=8))
    # 16 slices of equal nonzero counts: the long row holds more than one
    # slice's share, so the slice after it is empty
    fixed_run(D, O, lp, 300, gpu_kw=dict(tile_nnz=512, gather_slices=16))


@pytest.mark.parametrize("slices", [-1, 8, 16])
def test_edge_cases_empty_rows_cols_free_rows(D, O, slices):
    """Empty rows and columns, free rows; sliced: most slices hold no
    nonzero at all (5 columns, 4 rows over 8 or 16 slices)."""
    A = np.array([[1.0, 0, 1, 0, 0], [0, 0, 0, 0, 0], [1, 0, -1, 0, 2], [0, 0, 0, 0, 0]])
    lp = lpgen.from_dense(A, [1.0, 2.0, -1.0, -3.0, 0.5], [1.0, -np.inf, -1.0, -np.inf],
                          [1.0, np.inf, np.inf, np.inf], [0] * 5, [5] * 5)
    fixed_run(D, O, lp, 200, gpu_kw=dict(gather_slices=slices))
    G = D.Problem(lp, gpu_params(D, eps=1e-10, gather_slices=slices))
    r = G.solve()
    o = O.Problem(lp, oracle_params(O, eps=1e-10)).solve()
    assert r["status"] == 1 and o["status"] == 1
    assert abs(r["obj_primal"] - o["obj_p"]) < 1e-8


def test_matrix_without_nonzeros(D, O):
    """A = 0 (3 rows, none of them binding, one an equality 0 = 0): a
    box-only LP, x_j = l_j where c_j > 0 and u_j where c_j < 0; tiles of
    empty segments only.  Iterates against the oracle, then the solve
    against the closed form."""
    rng = np.random.default_rng(12)
    n = 40
    c = rng.standard_normal(n)
    lo, hi = -rng.uniform(0, 2, n), rng.uniform(0, 2, n)
    lp = lpgen.from_dense(np.zeros((3, n)), c, [-np.inf, -1.0, 0.0], [np.inf, 1.0, 0.0], lo, hi)
    assert lp.nnz == 0
    fixed_run(D, O, lp, 150)
    r = D.Problem(lp, gpu_params(D, eps=1e-10)).solve()
    assert r["status"] == D.CONVERGED
    assert np.abs(r["x"] - np.where(c > 0, lo, hi)).max() <= 1e-9
    assert abs(r["obj_primal"] - np.sum(np.where(c > 0, c * lo, c * hi))) <= 1e-9


@pytest.mark.parametrize("orient,slices", [("row", 8), ("column", -1)])
def test_segment_split_into_hundreds_of_pieces(D, O, orient, slices):
    """One dense row (dual step) or column (primal step) of 300,000 nonzeros
    (147 pieces of 2048, or about 18 per slice when sliced) beside 2,000
    short ones: the pieces' carries are added in piece order by
    k_split_fix."""
    import scipy.sparse as sp
    rng = np.random.default_rng(13)
    big, n_short = 300_000, 2000
    dense = sp.csr_matrix(rng.uniform(0.5, 1.5, (1, big)))
    short = sp.random(n_short, big, density=4.0 / big, random_state=14, format="csr",
                      data_rvs=lambda k: rng.standard_normal(k))
    A = sp.vstack([dense, short]).tocsr()
    if orient == "column":
        A = A.T.tocsr()
    A.sort_indices()
    m, n = A.shape
    x0 = rng.uniform(0.0, 1.0, n)
    b = A @ x0
    lo, hi = b - 0.5, b + 0.5
    if orient == "row":
        lo[0], hi[0] = -np.inf, b[0] + 1.0
    lp = lpgen.LP(m, n, A.indptr.astype(np.int32), A.indices.astype(np.int32),
                  A.data.copy(), rng.standard_normal(n), lo, hi, np.zeros(n), np.ones(n),
                  name=f"long-{orient}")
    fixed_run(D, O, lp, 200, gpu_kw=dict(gather_slices=slices))


@pytest.mark.parametrize("slices", [-1, 8])
def test_single_row_and_single_column(D, O, slices):
    """One row of 5000 nonzeros and one column of 4000 (split over tiles;
    sliced: split within a slice, and 1-wide index ranges)."""
    rng = np.random.default_rng(11)
    n = 5000                                   # one row of 5000 nonzeros (split)
    w = rng.uniform(1, 10, n)
    lp = lpgen.from_dense(w[None, :], -rng.uniform(1, 10, n), [-np.inf], [0.4 * w.sum()],
                          np.zeros(n), np.ones(n))
    fixed_run(D, O, lp, 300, gpu_kw=dict(gather_slices=slices))
    m = 4000                                   # one column of 4000 nonzeros (split)
    a = rng.standard_normal(m)
    lp = lpgen.from_dense(a[:, None], [1.0], a * 0.5 - 1, a * 0.5 + 1, [-2.0], [2.0])
    fixed_run(D, O, lp, 300, gpu_kw=dict(gather_slices=slices))


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("slices", [-1, 8])
def test_tiny_lps(D, O, seed, slices):
    fixed_run(D, O, lpgen.tiny_lp(seed), 500, gpu_kw=dict(gather_slices=slices))


# ---- solves ----------------------------------------------------------------------
@pytest.mark.parametrize("eps", [1e-4, 1e-8])
def test_solve_c0_objective_and_kkt(D, O, eps):
    lp = lpgen.config0()
    G = D.Problem(lp, gpu_params(D, eps=eps))
    r = G.solve()
    o = O.Problem(lp, oracle_params(O, eps=eps)).solve()
    assert r["status"] == 1 and o["status"] == 1
    assert max(r["r_primal"], r["r_dual"], r["r_gap"]) <= eps
    tol = 10 * eps * (1 + abs(o["obj_p"]))
    assert abs(r["obj_primal"] - o["obj_p"]) <= tol
    assert abs(r["obj_primal"] - lp.obj_star) <= tol
    # the library's KKT of its own output agrees with the oracle's evaluation
    k = O.Problem(lp).kkt(r["x"], r["y"], tau=r["eta"] / r["omega"])
    assert max(k[:3]) <= 1.5 * eps


def test_solve_c4_1e8(D, O):
    lp = lpgen.config4()
    G = D.Problem(lp)
    r = G.solve()
    o = O.Problem(lp).solve()
    assert r["status"] == 1 and o["status"] == 1
    assert abs(r["obj_primal"] - o["obj_p"]) <= 1e-7 * (1 + abs(o["obj_p"]))
    assert abs(r["iters"] - o["iters"]) <= 0.2 * o["iters"] + 64


def test_fp32_mixed_reaches_1e8(D, O):
    lp = lpgen.config4()
    G = D.Problem(lp, gpu_params(D, precision=D.FP32_MIXED))
    r = G.solve()
    o = O.Problem(lp).solve()
    assert r["status"] == 1
    assert max(r["r_primal"], r["r_dual"], r["r_gap"]) <= 1e-8
    assert r["fp32_iters"] > 0
    assert abs(r["obj_primal"] - o["obj_p"]) <= 1e-7 * (1 + abs(o["obj_p"]))


def test_fp32_divergence_switches_to_fp64_from_best_point(D, O):
    """On config 4 the FP32 phase stalls near KKT 1e-4: the primal weight
    falls, the primal step grows, and FP32 rounding of c - A^T y grows with
    it.  The switch rule (KKT 10x above the phase's best) hands over to FP64
    at the best check point, so the solve to 1e-4 takes at most twice the
    FP64 iterations and reaches the oracle's objective."""
    lp = lpgen.config4()
    r64 = D.Problem(lp, gpu_params(D, eps=1e-4)).solve()
    G = D.Problem(lp, gpu_params(D, eps=1e-4, precision=D.FP32_MIXED, fp32_switch_tol=0.0))
    r = G.solve()
    assert r["status"] == 1 and r64["status"] == 1
    assert max(r["r_primal"], r["r_dual"], r["r_gap"]) <= 1e-4
    assert r["iters"] <= 2 * r64["iters"], (r["iters"], r64["iters"])
    kkt = lambda e: max(e["r_primal"], e["r_dual"], e["r_gap"])
    lg = G.log()
    fp32_checks = [e for e in lg if e["t"] < r["fp32_iters"]]
    best = [min(kkt(e) for e in fp32_checks[:i + 1]) for i in range(len(fp32_checks))]
    # the switch came from the divergence rule: the last FP32 check is 10x
    # above the best before it, and no earlier one is
    assert r["fp32_iters"] < r["iters"]
    assert kkt(fp32_checks[-1]) > 10 * best[-2]
    for i in range(1, len(fp32_checks) - 1):
        assert kkt(fp32_checks[i]) <= 10 * best[i - 1], i
    # FP64 resumed at the best point: its first check is near that KKT
    first64 = next(e for e in lg if e["t"] >= r["fp32_iters"])
    assert kkt(first64) <= 10 * best[-2]
    ibest = int(np.argmin([kkt(e) for e in fp32_checks[:-1]]))
    assert first64["omega"] == fp32_checks[ibest]["omega"]
    o = O.Problem(lp, O.Params(eps=1e-4)).solve()
    assert abs(r["obj_primal"] - o["obj_p"]) <= 1e-3 * (1 + abs(o["obj_p"]))

    # The FP64 phase is plain FP64 PDHG from the best point with the best
    # point's primal weight and the PID state at the switch: the oracle,
    # started there, takes the same restart decisions and primal weights,
    # and its fixed-point residuals r (App. B.2, measured in the P-norm of
    # that weight) match the GPU's.
    G2 = D.Problem(lp, gpu_params(D, eps=1e-4, precision=D.FP32_MIXED, fp32_switch_tol=0.0))
    G2.init()
    G2.iterate(int(r["fp32_iters"]))
    s = G2.state()
    sc = s["scalars"]
    assert sc["t"] == r["fp32_iters"] and sc["k"] == 0 and sc["omega"] == first64["omega"]
    scal = G2.scaling()
    P = O.Problem(lp, O.Params(eps=0.0, eta=scal["eta"], omega0=sc["omega"]))
    ost = P.init_state(scal["dc"] * s["xa"], scal["dr"] * s["ya"])
    S = ost["state"]
    for f in ("omega", "pid_int", "pid_prev", "pid_started", "restarts", "t", "k"):
        setattr(S, f, sc[f])
    n_more = 640
    P.run(ost, n_more)
    G2.set_params(eps=0.0)
    G2.iterate(n_more)
    lg2 = [e for e in G2.log() if e["t"] >= r["fp32_iters"]]
    lo2 = ost["log"]
    assert len(lg2) == len(lo2) and len(lo2) >= 4
    assert any(e["restart"] for e in lo2), "no restart in the compared window"
    # The oracle's scaled problem and its start point (mapped back through
    # its own D_r, D_c, which agree with the GPU's to about 1e-13) differ
    # from the GPU's by about 1e-13 relative, so r = ||z - T(z)||_P, a
    # difference of vectors of size ||z||_P, agrees to about 1e-13 ||z||_P.
    # The primal weight moves at a restart by the log of the ratio of the
    # distances to the anchor, which are of the size of r, so it agrees to
    # about 1e-13 ||z||_P / r of the restarts before it.
    w, eta = sc["omega"], scal["eta"]
    zP = np.sqrt((w / eta) * np.dot(s["xa"], s["xa"]) + np.dot(s["ya"], s["ya"]) / (eta * w))
    r_min = np.inf
    for g, e in zip(lg2, lo2):
        assert (g["t"], g["k"], g["restart"]) == (e["t"], e["k"], e["restart"]), (g, e)
        tol_w = 1e-9 + (1e-12 * zP / r_min if np.isfinite(r_min) else 0.0)
        assert abs(g["omega"] - e["omega"]) <= tol_w * e["omega"], (g, e, tol_w)
        assert abs(g["r"] - e["r"]) <= 1e-12 * zP + 1e-9 * e["r"], (g, e, zP)
        if e["restart"]:
            r_min = min(r_min, e["r"])
    gs = G2.state()
    for k in ("x", "y", "xh", "yh"):
        assert rel(gs[k], ost[k]) <= 1e-9, (k, rel(gs[k], ost[k]))


# ---- determinism, checkpoint / resume ------------------------------------------------
def test_bitwise_deterministic(D):
    lp = lpgen.huge_share_lp(m=20000, n=40000, seed=12)
    outs = []
    for _ in range(2):
        G = D.Problem(lp, gpu_params(D, eps=0.0))
        G.init()
        G.iterate(300)
        outs.append(G.state())
    for k in ("x", "y", "xh", "yh"):
        assert np.array_equal(outs[0][k], outs[1][k]), k


def test_checkpoint_resume_is_exact(D):
    lp = lpgen.config0()
    G = D.Problem(lp, gpu_params(D, eps=0.0))
    G.init()
    G.iterate(700)
    ref = G.state()
    G2 = D.Problem(lp, gpu_params(D, eps=0.0))
    G2.init()
    G2.iterate(300)
    snap = G2.state()
    G3 = D.Problem(lp, gpu_params(D, eps=0.0))
    G3.load_state(snap)
    G3.iterate(400)
    got = G3.state()
    for k in ("x", "y", "xa", "ya", "xh", "yh"):
        assert np.array_equal(got[k], ref[k]), k


def test_warm_start_at_optimum_converges_at_once(D):
    lp = lpgen.config0()
    G = D.Problem(lp)
    r = G.solve(x0=lp.x_star, y0=lp.y_star)
    assert r["status"] == 1 and r["iters"] <= 2


def test_bad_input_is_rejected_on_gpu(D):
    lp = lpgen.config0()
    lp.col_idx = lp.col_idx.copy()
    lp.col_idx[5] = lp.n + 3
    with pytest.raises(D.DpdlpError) as e:
        D.Problem(lp)
    assert e.value.code == D.E_BAD_CSR


@pytest.mark.parametrize("kw,msg", [(dict(gather_slices=12), "gather_slices"),
                                    (dict(gather_slices=72), "gather_slices"),
                                    (dict(perm_order=-1), "perm_order")])
def test_bad_parameters_are_rejected(D, kw, msg):
    """Slice counts that are not a multiple of 8 up to 64, and unknown
    orders, are errors with a message; the partly built handle is freed."""
    with pytest.raises(D.DpdlpError, match=msg) as e:
        D.Problem(lpgen.config0(), gpu_params(D, **kw))
    assert e.value.code == D.E_INVALID_ARG


@pytest.mark.parametrize("kw,qp", [(dict(), False), (dict(precision=1), False),
                                   (dict(gather_slices=8), False), (dict(), True),
                                   (dict(precision=1, gather_slices=8), True)])
def test_graph_replay_matches_eager_bitwise(D, kw, qp):
    """Runs between checks replayed as one HIP graph give bitwise the same
    solve as eager launches (dozens of replays with restarts, checks and host
    synchronizations between them), for the LP and for the diagonal QP's
    primal step (FP64 unsliced, FP32-mixed sliced)."""
    lp = lpgen.constructed_qp(2000, 4000, 1000, 5, seed=21) if qp else lpgen.config4()
    outs = []
    for graphs in (0, 1):
        G = D.Problem(lp, gpu_params(D, use_graphs=graphs, **kw))
        r = G.solve()
        outs.append((r, G.log()))
    (r0, l0), (r1, l1) = outs
    assert r0["status"] == 1 and r0["iters"] == r1["iters"]
    assert np.array_equal(r0["x"], r1["x"]) and np.array_equal(r0["y"], r1["y"])
    assert [e["restart"] for e in l0] == [e["restart"] for e in l1]


@pytest.mark.parametrize("name,maker", [
    ("c0", lpgen.config0),
    ("huge-share-small", lambda: lpgen.huge_share_lp(m=20000, n=40000, seed=9)),
    ("transport-60x4000", lambda: lpgen.transport_lp(60, 4000, seed=3))])
def test_fp32_mixed_iterates_against_fp64_oracle(D, O, name, maker):
    """The FP32-mixed form's error against the FP64 oracle after 64
    iterations from the same start with the same step sizes (one epoch, the
    same restart decision): FP32 rounding of A~, the iterates and the
    accumulations, about 6e-8 per operation, keeps the iterates within 1e-5
    relative.  The measured error is printed."""
    lp = maker()
    P0 = O.Problem(lp)
    eta, w0 = P0.eta, P0.omega0
    P = O.Problem(lp, oracle_params(O, eta=eta, omega0=w0, eps=0.0))
    st = P.init_state()
    P.run(st, 64)
    G = D.Problem(lp, gpu_params(D, eta=eta, omega0=w0, eps=0.0, precision=D.FP32_MIXED,
                                 fp32_switch_tol=0.0, fp32_stall_checks=10**6, fp32_diverge=0.0))
    G.init()
    G.iterate(64)
    gs = G.state()
    assert [e["restart"] for e in G.log()] == [e["restart"] for e in st["log"]]
    errs = {k: rel(gs[k], st[k]) for k in ("xh", "yh")}
    print(f"{name}: FP32-mixed vs FP64 oracle after 64 iterations: {errs}")
    assert max(errs.values()) <= 1e-5, errs


def test_time_gather_probe(D):
    """The random-gather probe that bench.py sets beside the fused steps:
    it runs in both precisions and slice counts, reports a positive rate,
    and rejects bad arguments with a message."""
    for prec in (D.FP64, D.FP32_MIXED):
        for S in (8, 16):
            r = D.dpdlp_time_gather(1 << 20, S, 3_000_001, precision=prec, reps=3)
            assert r["avg_ms"] > 0 and r["gathers_per_s"] > 1e9, (prec, S, r)
    for bad in (dict(n_vec=1 << 20, slices=12, n_gathers=1000),
                dict(n_vec=7, slices=8, n_gathers=1000),
                dict(n_vec=1 << 20, slices=8, n_gathers=0)):
        with pytest.raises(D.DpdlpError, match="dpdlp_time_gather") as e:
            D.dpdlp_time_gather(**bad)
        assert e.value.code == D.E_INVALID_ARG


def test_bad_memory_kind_is_rejected_before_any_pointer_is_read(D):
    """A memory kind other than host (0) or device (1) is an INVALID_ARG
    error at every entry point that takes one, raised before a pointer is
    read, so host arrays passed with a wrong kind cannot fault the GPU."""
    import ctypes as C
    lp = lpgen.config0()
    arrs = D.host_arrays(lp)
    bad = 7
    out = C.c_void_p()
    rc = D._lib.dpdlp_problem_create(C.byref(D._csr_struct(arrs, lp.m, lp.n, bad)),
                                     C.byref(gpu_params(D)), None, C.byref(out))
    assert rc == D.E_INVALID_ARG and "mem_kind" in D.dpdlp_last_error()
    G = D.Problem(lp, gpu_params(D))
    x, y = np.zeros(lp.n), np.zeros(lp.m)
    k = np.zeros(5)
    res = D.Result()
    calls = {
        "init": lambda: D._lib.dpdlp_init(G.h, x.ctypes.data, y.ctypes.data, bad, None),
        "solve": lambda: D._lib.dpdlp_solve(G.h, None, None, x.ctypes.data, y.ctypes.data, bad,
                                            C.byref(res), None),
        "get_result": lambda: D._lib.dpdlp_get_result(G.h, x.ctypes.data, y.ctypes.data, bad,
                                                      C.byref(res), None),
        "kkt": lambda: D._lib.dpdlp_kkt(G.h, x.ctypes.data, y.ctypes.data, 1.0, bad,
                                        k.ctypes.data, None),
        "update_data": lambda: D._lib.dpdlp_problem_update_data(G.h, arrs["c"].ctypes.data, None,
                                                                None, None, None, bad, None),
    }
    for name, call in calls.items():
        assert call() == D.E_INVALID_ARG, name
        assert "mem_kind" in D.dpdlp_last_error(), name
    # the handle still works afterwards
    r = G.solve()
    assert r["status"] == D.CONVERGED
