"""dpdlp_kkt_noalloc (the KKT evaluation that allocates nothing) against
dpdlp_kkt of a prepared problem handle, through the C ABI: the same KKT
values (App. B.4) at perturbed points, on consecutive calls that share the
library's fixed scratch array, the second and third on smaller inputs."""
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


def _device_lp(D, lp):
    import torch
    csr = {k: torch.from_numpy(v).cuda() for k, v in D.host_arrays(lp).items()}
    A = lp.scipy_csr().tocsc()
    csc = dict(col_ptr=torch.from_numpy(A.indptr.astype(np.int32)).cuda(),
               row_idx=torch.from_numpy(A.indices.astype(np.int32)).cuda(),
               val=torch.from_numpy(A.data.astype(np.float64)).cuda())
    return csr, csc


def _point(lp, seed):
    """A point off the optimum, inside X, with y projected onto Y."""
    rng = np.random.default_rng(seed)
    x = np.clip(lp.x_star + rng.standard_normal(lp.n), lp.var_lo, lp.var_hi)
    y = lp.y_star + 0.1 * rng.standard_normal(lp.m)
    y = np.where(np.isinf(lp.con_hi), np.maximum(y, 0.0), y)
    y = np.where(np.isinf(lp.con_lo), np.minimum(y, 0.0), y)
    return x, y


def test_kkt_noalloc_matches_kkt_on_consecutive_calls(D):
    import torch
    cases = [(lpgen.config4(), 0.3), (lpgen.config0(), 0.7),
             (lpgen.constructed_qp(300, 700, 150, 4, seed=5), 0.2)]
    for i, (lp, tau) in enumerate(cases):
        G = D.Problem(lp)
        dc = torch.from_numpy(G.scaling()["dc"]).cuda()
        x, y = _point(lp, 10 + i)
        ref = G.kkt(x, y, tau=tau)
        csr, csc = _device_lp(D, lp)
        q = getattr(lp, "q", None)
        qd = None if q is None else torch.from_numpy(np.asarray(q, np.float64)).cuda()
        out = torch.full((5,), np.nan, dtype=torch.float64, device="cuda")
        D.dpdlp_kkt_noalloc(lp.m, lp.n, csr, csc, torch.from_numpy(x).cuda(),
                            torch.from_numpy(y).cuda(), tau, out, col_scale=dc, q=qd,
                            stream=torch.cuda.current_stream())
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        print(f"{lp.name}: no-alloc {got}, handle {ref}")
        assert np.all(ref[:3] > 1e-6)          # a point off the optimum
        assert np.allclose(got, ref, rtol=1e-11, atol=0), (i, got, ref)
        G.close()


def test_kkt_noalloc_rejects_bad_input(D):
    """Argument checks run on the host before any device access."""
    import torch
    lp = lpgen.config0()
    csr, csc = _device_lp(D, lp)
    x = torch.zeros(lp.n, dtype=torch.float64, device="cuda")
    y = torch.zeros(lp.m, dtype=torch.float64, device="cuda")
    out = torch.zeros(5, dtype=torch.float64, device="cuda")
    with pytest.raises(D.DpdlpError, match="16777216") as e:
        D.dpdlp_kkt_noalloc(16_777_217, lp.n, csr, csc, x, y, 0.5, out)
    assert e.value.code == D.E_INVALID_ARG
    with pytest.raises(D.DpdlpError, match="tau"):
        D.dpdlp_kkt_noalloc(lp.m, lp.n, csr, csc, x, y, 0.0, out)
    host = D.host_arrays(lp)
    s = D._csr_struct(host, lp.m, lp.n, D.MEM_HOST)
    rc = D.lib().dpdlp_kkt_noalloc(s, D._ptr(csc["col_ptr"]), D._ptr(csc["row_idx"]),
                                   D._ptr(csc["val"]), None, None, D._ptr(x), D._ptr(y), 0.5,
                                   D._ptr(out), None)
    assert rc == D.E_INVALID_ARG and "device memory" in D.dpdlp_last_error()
