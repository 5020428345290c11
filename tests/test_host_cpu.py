"""CPU-only tests of the library's host logic and of its C ABI surface.

No GPU compute: the library is loaded, every symbol the header declares is
checked, and the host-only preprocessing entry points (validation, the
block-wise random permutation of Sec. 4.2, the nonzero-aware tiles of
Sec. 4.3) are exercised.
"""
import os
import re

import numpy as np
import pytest

import lpgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def D():
    import paper_2601_07628_amd as D
    return D


def test_library_exports_every_declared_symbol(D):
    hdr = open(os.path.join(ROOT, "include", "dpdlp.h")).read()
    declared = set(re.findall(r"\b(dpdlp_[a-z_0-9]+)\s*\(", hdr))
    assert declared, "no declarations found"
    assert declared == set(D.EXPORTS), declared ^ set(D.EXPORTS)
    for name in declared:
        assert hasattr(D.lib(), name), name


def test_params_defaults_match_oracle_defaults(D):
    import oracle
    p = D.dpdlp_params_default()
    o = oracle.Params()
    for k in ("eps", "max_iters", "check_period", "ruiz_iters", "gamma", "beta_suf",
              "beta_nec", "beta_art", "kp", "ki", "kd", "eta", "omega0", "eta_safety",
              "power_max_iters", "use_pc", "power_tol", "pc_alpha"):
        assert getattr(p, k) == getattr(o, k), k
    assert p.perm_block == 256            # B = 256 (Sec. 4.2)


def test_validate_accepts_good_lps(D):
    for lp in (lpgen.config0(), lpgen.tiny_lp(3), lpgen.transport_lp(20, 30)):
        assert D.dpdlp_validate(lp) == 0


def _lp(**over):
    lp = lpgen.from_dense([[1.0, 2.0, 0.0], [0.0, 1.0, 3.0]], [1, 1, 1], [1, -np.inf],
                          [1, 4.0], [0, 0, 0], [1, 1, 1])
    for k, v in over.items():
        setattr(lp, k, np.asarray(v))
    return lp


@pytest.mark.parametrize("over,code", [
    (dict(row_ptr=[0, 3, 2]), -2),                  # not monotone
    (dict(row_ptr=[1, 2, 4]), -2),                  # row_ptr[0] != 0
    (dict(col_idx=[0, 1, 1, 5]), -2),               # column out of range
    (dict(col_idx=[0, 0, 1, 2]), -2),               # duplicate (0,0)
    (dict(val=[1.0, np.nan, 1.0, 3.0]), -2),        # NaN value
    (dict(con_lo=[2.0, -np.inf], con_hi=[1.0, 4.0]), -3),   # lo > hi
    (dict(var_lo=[0, np.inf, 0]), -3),              # lo = +inf
    (dict(var_hi=[1, np.nan, 1]), -3),              # NaN bound
    (dict(c=[1.0, np.inf, 1.0]), -3),               # non-finite c
])
def test_validate_rejects_bad_input(D, over, code):
    assert D.dpdlp_validate(_lp(**over)) == code
    assert D.dpdlp_last_error()


def test_block_permutation_structure(D):
    for count, block in [(1000, 256), (256, 256), (257, 256), (5000, 100), (10, 0)]:
        p = D.dpdlp_block_permutation(count, block, 12345)
        assert sorted(p.tolist()) == list(range(count))            # a permutation
        if block <= 0 or count <= block:
            assert np.array_equal(p, np.arange(count))
            continue
        # walk the new order: every original block appears whole, in order
        a = 0
        while a < count:
            assert p[a] % block == 0
            L = min(block, count - p[a])
            assert np.array_equal(p[a:a + L], np.arange(p[a], p[a] + L))
            a += L
    p1 = D.dpdlp_block_permutation(100000, 256, 1)
    p2 = D.dpdlp_block_permutation(100000, 256, 2)
    assert not np.array_equal(p1, p2)                               # seeded
    assert np.array_equal(p1, D.dpdlp_block_permutation(100000, 256, 1))


def _check_tiles(t, ptr, tile_nnz):
    nseg = ptr.size - 1
    # coverage: tiles walk the segments in order, nonzeros exactly once
    pos_seg, pos_nnz = 0, 0
    for row in t:
        sb, se, nb, ne, wl, pc, npc, _ = row.tolist()
        assert nb == pos_nnz and ne - nb <= tile_nnz
        if npc == 0:
            assert sb == pos_seg and se > sb and se - sb <= 1024
            assert nb == ptr[sb] and ne == ptr[se]
            assert 0 <= wl <= 6
            pos_seg = se
        else:
            assert se == sb + 1 and ptr[sb + 1] - ptr[sb] > tile_nnz
            assert nb == ptr[sb] + pc * tile_nnz
            if pc == npc - 1:
                assert ne == ptr[sb + 1]
                pos_seg = se
            else:
                assert sb == pos_seg
        pos_nnz = ne
    assert pos_seg == nseg and pos_nnz == ptr[-1]


@pytest.mark.parametrize("tile_nnz", [0, 512])
def test_tiles_cover_and_balance(D, tile_nnz):
    cap = tile_nnz or 2048
    rng = np.random.default_rng(0)
    lens = np.concatenate([rng.integers(0, 30, 5000), [0] * 3000, [5000, 2049, 2048],
                           rng.integers(100, 400, 50), [1] * 4000])
    ptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    t = D.dpdlp_build_tiles(ptr, tile_nnz)
    _check_tiles(t, ptr, cap)
    # nonzero-aware: every tile but the ones closed by a segment boundary is
    # at least half full (greedy packing), and none exceeds the cap
    nz = t[:, 3] - t[:, 2]
    assert nz.max() <= cap


def test_tiles_on_generated_instances(D):
    for lp in (lpgen.config0(), lpgen.huge_share_lp(m=20000, n=40000, seed=3),
               lpgen.transport_lp(50, 3000)):
        ptr = lp.row_ptr
        _check_tiles(D.dpdlp_build_tiles(ptr), ptr, 2048)
        cp = np.concatenate([[0], np.cumsum(np.bincount(lp.col_idx, minlength=lp.n))])
        _check_tiles(D.dpdlp_build_tiles(cp.astype(np.int32)), cp, 2048)


def test_create_without_gpu_fails_loudly(D):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(D.DpdlpError):
        D.Problem(lpgen.config0())


@pytest.mark.parametrize("prog", ["slice_format_check", "bidiag_check"])
def test_host_cpp_checks(tmp_path, prog):
    """Host-side C++ checks built with g++ and the sanitizers (no GPU code):
    the compact sliced format with the combine's indexing, and the Lanczos
    bidiagonal helpers (see the sources under tests/host_cpp/)."""
    import shutil
    import subprocess
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    csrc = os.path.join(root, "paper_2601_07628_amd", "csrc")
    exe = str(tmp_path / prog)
    cmd = [gxx, "-O1", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", os.path.join(root, "include"), "-I", csrc,
           os.path.join(root, "tests", "host_cpp", prog + ".cpp"),
           os.path.join(csrc, "dpdlp_host.cpp"), "-o", exe, "-lpthread"]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout[-2000:] + out.stderr[-2000:]
    assert out.stdout.strip().endswith("ok")


def test_row_bounds_from_row_types(D):
    """Ax (=, >=, <=) b rows as [lo, hi] bounds; bad input is rejected."""
    b = np.array([1.5, -2.0, 3.0, 0.0])
    lo, hi = D.dpdlp_row_bounds(b, [0, 1, 2, 1])
    assert np.array_equal(lo, [1.5, -2.0, -np.inf, 0.0])
    assert np.array_equal(hi, [1.5, np.inf, 3.0, np.inf])
    assert D.dpdlp_validate(lpgen.from_dense(np.eye(4), np.ones(4), lo, hi, np.zeros(4), np.ones(4))) == 0
    with pytest.raises(D.DpdlpError, match="row type"):
        D.dpdlp_row_bounds(b, [0, 1, 3, 1])
    with pytest.raises(D.DpdlpError, match="finite"):
        D.dpdlp_row_bounds([np.inf], [1])


def test_bench_refuses_more_than_one_gpu():
    """bench.py --gpus N with N > 1 exits with a message before touching a GPU
    (the library has no multi-GPU path)."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
