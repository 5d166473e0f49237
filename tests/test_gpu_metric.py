"""Variable-metric search directions on the GPU (Remark in Sec. 3: the metric
L_k with the p-Laplacian's coefficient frozen at the current iterate, solved
by conjugate gradients preconditioned with the FFT operator L_h) against the
oracle's variable-metric PSD."""
import numpy as np
import pytest

import oracle
import psd_inputs
from parity_bounds import check_alphas, rounding_scale

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def psd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1607_01475_amd import psd as _psd
    _psd.load_library()
    return _psd


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


# a fixed number of inner iterations makes both sides run the same sequence of
# directions (up to rounding), so the iterates compare at matched counts
@pytest.mark.parametrize("dim,n,p", [(2, 64, 4.0), (2, 48, 3.0), (3, 32, 4.0), (3, 48, 6.0)])
def test_variable_metric_matches_oracle(psd, dim, n, p):
    L, s, eps, m = 12.8 * n / 64, 0.01, 0.1, 8
    f = psd_inputs.small_field(dim, n, L, 51, K=6)
    O = oracle.Problem(dim, n, L, p=p, s=s, eps=eps)
    ref = oracle.solve_variable_metric(O, f, tol=1e-10, max_iter=100, inner_rtol=0.0, inner_iters=m)
    P = psd.Problem(dim, n, L, 4, p, s, eps)
    with psd.Solver(P, tol=1e-10, max_iter=100, metric="variable", inner_rtol=0.0, inner_iters=m,
                    history=True) as S:
        u = torch.zeros_like(dev(f))
        st = S.solve([dev(f)], [u])[0]
        hist = S.history(0)
    print(f"case vm {dim}D n={n} p={p}: gpu iters {st.iters} oracle {ref['iters']}", flush=True)
    assert st.status == 0 and abs(st.iters - ref["iters"]) <= 1
    # step sizes: the per-update rounding bound of the other parity tests
    # (residual rounding over ||r_{k-1}||, plus the sums' sqrt(N) floor)
    check_alphas(hist[:, 0], ref["alphas"], ref["res_hist"], ref["res0"], rounding_scale(O, ref["u"]), f.size)
    kk = max(ref["iters"] - 1, 1)
    ref_k = oracle.solve_variable_metric(O, f, tol=0.0, max_iter=kk, inner_rtol=0.0, inner_iters=m)
    with psd.Solver(P, tol=0.0, max_iter=kk, metric="variable", inner_rtol=0.0, inner_iters=m) as S:
        u = torch.zeros_like(dev(f))
        S.solve([dev(f)], [u])
    e = rel(host(u), ref_k["u"])
    print(f"  matched k={kk}: rel {e:.2e}", flush=True)
    assert e <= 1e-11


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_variable_metric_reaches_the_minimiser(psd, precision):
    # the unique minimiser (Sec. 3) with fewer outer iterations than the
    # constant metric; the inner solve to a relative tolerance
    dim, n, L = 3, 48, 12.8
    f = psd_inputs.small_field(dim, n, L, 52, K=6)
    O = oracle.Problem(dim, n, L, p=4.0, s=0.01, eps=0.1)
    ref = O.solve(f, tol=1e-12, max_iter=300)
    P = psd.Problem(dim, n, L, 4, 4.0, 0.01, 0.1)
    iters = {}
    for metric in ("constant", "variable"):
        with psd.Solver(P, tol=1e-10, max_iter=300, precision=precision, metric=metric,
                        inner_rtol=1e-6, inner_iters=100) as S:
            u = torch.zeros_like(dev(f))
            st = S.solve([dev(f)], [u])[0]
        assert st.status == 0 and st.res_inf <= 1e-10
        iters[metric] = st.iters
        assert rel(host(u), ref["u"]) <= 1e-9
    print(f"case vm {precision}: outer iterations {iters}", flush=True)
    assert iters["variable"] < iters["constant"]
