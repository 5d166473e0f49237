"""Sixth-order mixed system in 3D (Sec. 5.4 with the 3D operators of the Remark
in Sec. 5.2): residuals, energy and PSD solves of the GPU against the oracle,
with non-zero means of f and g (Sec. 4 conservation)."""
import numpy as np
import pytest

import oracle
import psd_inputs
from parity_bounds import check_alphas, rounding_scale

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

S6, EPS6, LAM6, L6 = 0.02, 0.1, 1.0, 12.8


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


def inputs(n, seed=61, fbar=-0.2, gbar=0.3):
    f = psd_inputs.small_field(3, n, L6, seed, K=5) + fbar
    g = psd_inputs.small_field(3, n, L6, seed + 1, K=5) + gbar
    return f, g


@pytest.mark.parametrize("n", [32, 48])
def test_residuals_and_energy_3d_order6(psd, n):
    print(f"case 3D order 6 operators n={n}", flush=True)
    f, g = inputs(n)
    u = psd_inputs.small_field(3, n, L6, 63, K=4) + g.mean()
    w = psd_inputs.small_field(3, n, L6, 64, K=4)
    O = oracle.Problem(3, n, L6, order=6, p=4.0, s=S6, eps=EPS6, lam=LAM6)
    P = psd.Problem(3, n, L6, 6, 4.0, S6, EPS6, LAM6)
    with psd.Solver(P) as S:
        r1, r2 = torch.empty_like(dev(f)), torch.empty_like(dev(f))
        S.residual_mixed(0, dev(f), dev(g), dev(u), dev(w), r1=r1, r2=r2)
        e1, e2 = O.mixed_residuals(f, g, u, w)
        assert np.abs(host(r1) - e1).max() <= 1e-12 * max(1, np.abs(e1).max())
        assert np.abs(host(r2) - e2).max() <= 1e-12 * max(1, np.abs(e2).max())
        r = torch.empty_like(r1)
        S.residual(0, dev(f), dev(u), g=dev(g), r=r)
        rho = O.residual(f, u, g)
        assert np.abs(host(r) - rho).max() <= 1e-12 * np.abs(rho).max()
        E = S.energy(0, dev(f), dev(u), g=dev(g))
        assert abs(E - O.energy(f, u, g)) <= 1e-12 * abs(E)


@pytest.mark.parametrize("n", [32, 48])
def test_solve_parity_3d_order6(psd, n):
    f, g = inputs(n)
    O = oracle.Problem(3, n, L6, order=6, p=4.0, s=S6, eps=EPS6, lam=LAM6)
    ref = O.solve(f, g=g, tol=1e-10, max_iter=400, history=True)
    P = psd.Problem(3, n, L6, 6, 4.0, S6, EPS6, LAM6)
    with psd.Solver(P, tol=1e-10, max_iter=400, history=True) as S:
        u = torch.full_like(dev(f), float(g.mean()))
        w = torch.zeros_like(u)
        st = S.solve([dev(f)], [u], g=[dev(g)], w=[w])[0]
        hist = S.history(0)
    print(f"case 3D order 6 n={n}: gpu iters {st.iters} oracle {ref['iters']}", flush=True)
    assert st.status == 0 and abs(st.iters - ref["iters"]) <= 1
    r1, r2 = O.mixed_residuals(f, g, host(u), host(w))
    assert np.abs(r1).max() <= 2e-10 and np.abs(r2).max() <= 2e-10
    check_alphas(hist[:, 0], ref["hist"][:, 0], ref["hist"][:, 1],
                 np.abs(O.residual(f, np.full_like(f, g.mean()), g)).max(),
                 rounding_scale(O, ref["u"], ref["w"]), f.size)
    kk = ref["iters"]
    with psd.Solver(P, tol=0.0, max_iter=kk) as S:
        u = torch.full_like(dev(f), float(g.mean()))
        w = torch.zeros_like(u)
        st = S.solve([dev(f)], [u], g=[dev(g)], w=[w])[0]
    ref_k = O.solve(f, g=g, tol=0.0, max_iter=kk)
    ug, wg = host(u), host(w)
    print(f"  matched k={kk}: u {rel(ug, ref_k['u']):.2e} w {rel(wg, ref_k['w']):.2e}", flush=True)
    assert st.iters == kk
    assert rel(ug, ref_k["u"]) <= 1e-11 and rel(wg, ref_k["w"]) <= 1e-11
    assert abs(ug.mean() - g.mean()) <= 1e-13 * (1 + abs(g.mean()))
    assert abs(wg.mean() - (S6 * LAM6 * g.mean() - f.mean())) <= 1e-12 * (1 + np.abs(wg).max())


def test_mixed_batched_3d_order6(psd):
    """Mixed precision, graph-captured, two 3D sizes in one handle."""
    sizes = [32, 48]
    data = [inputs(n, seed=70 + 2 * i, fbar=0.1 * i, gbar=-0.2 + 0.3 * i) for i, n in enumerate(sizes)]
    probs = [psd.Problem(3, n, L6, 6, 4.0, S6, EPS6, LAM6) for n in sizes]
    with psd.Solver(probs, tol=1e-10, max_iter=400, precision="mixed", graph_chunk=4) as S:
        us = [torch.full_like(dev(f), float(g.mean())) for f, g in data]
        ws = [torch.zeros_like(u) for u in us]
        stats = S.solve([dev(f) for f, _ in data], us, g=[dev(g) for _, g in data], w=ws)
    for (f, g), n, u, w, st in zip(data, sizes, us, ws, stats):
        O = oracle.Problem(3, n, L6, order=6, p=4.0, s=S6, eps=EPS6, lam=LAM6)
        ug, wg = host(u), host(w)
        print(f"case 3D order 6 mixed n={n}: iters {st.iters}", flush=True)
        assert st.status == 0 and st.res_inf <= 1e-10
        r1, r2 = O.mixed_residuals(f, g, ug, wg)
        assert np.abs(r1).max() <= 2e-10 and np.abs(r2).max() <= 2e-10
        ref = O.solve(f, g=g, tol=1e-10, max_iter=400)
        assert rel(ug, ref["u"]) <= 1e-9
