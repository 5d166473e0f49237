"""GPU adjoint (Hessian-CG through the C ABI) against the oracle adjoint,
central finite differences and, at full size, the defining equation."""
import numpy as np
import pytest

import oracle
import psd_inputs

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


@pytest.mark.parametrize("dim,n,precision", [(2, 64, "fp64"), (3, 32, "fp64"), (3, 32, "mixed")])
def test_adjoint_matches_oracle(psd, dim, n, precision):
    print(f"case adjoint dim={dim} n={n} {precision}", flush=True)
    L = 12.8 * n / 64
    f = psd_inputs.small_field(dim, n, L, 81, K=5)
    ut = psd_inputs.small_field(dim, n, L, 82, K=5)
    O = oracle.Problem(dim, n, L, p=4.0, s=0.01, eps=0.1)
    P = psd.Problem(dim, n, L, 4, 4.0, 0.01, 0.1)
    with psd.Solver(P, tol=1e-13, max_iter=500, precision=precision) as S:
        u = torch.zeros_like(dev(f))
        S.solve([dev(f)], [u])
        gu = O.hd * (host(u) - ut)
        lam, ds, de, it = S.adjoint([u], [dev(gu)], rtol=1e-13, max_iter=500)
    ref = O.adjoint(host(u), gu, rtol=1e-14)
    rel = np.abs(host(lam[0]) - ref["dJdf"]).max() / np.abs(ref["dJdf"]).max()
    print(f"  cg iters gpu {it[0]} oracle {ref['iters']} rel {rel:.2e}", flush=True)
    assert rel < 1e-9
    assert abs(ds[0] - ref["dJds"]) < 1e-9 * abs(ref["dJds"])
    assert abs(de[0] - ref["dJdeps"]) < 1e-9 * abs(ref["dJdeps"])


def test_autograd_matches_finite_differences(psd):
    n, L, s, eps = 32, 6.4, 0.01, 0.1
    f_np = psd_inputs.small_field(3, n, L, 91, K=5)
    ut = dev(psd_inputs.small_field(3, n, L, 92, K=5))
    h3 = (L / n) ** 3

    def J_of(ff, ss, ee):
        with psd.Solver(psd.Problem(3, n, L, 4, 4.0, ss, ee), tol=1e-13, max_iter=500) as S:
            u = torch.zeros_like(ff)
            st = S.solve([ff], [u])[0]
            assert st.status == 0
        return 0.5 * h3 * float(((u - ut) ** 2).sum())

    P = psd.Problem(3, n, L, 4, 4.0, s, eps)
    with psd.Solver(P, tol=1e-13, max_iter=500, precision="mixed") as S:
        f = dev(f_np).requires_grad_(True)
        st = torch.tensor(s, dtype=torch.float64, device="cuda", requires_grad=True)
        et = torch.tensor(eps, dtype=torch.float64, device="cuda", requires_grad=True)
        u = psd.solve_differentiable(f, st, et, S, adj_rtol=1e-13)
        J = 0.5 * h3 * ((u - ut) ** 2).sum()
        J.backward()
    gf, gs, ge = f.grad.detach(), float(st.grad), float(et.grad)
    tau = 1e-4
    dirn = dev(psd_inputs.white_noise(f_np.shape, 93))
    fd_f = (J_of(dev(f_np) + tau * dirn, s, eps) - J_of(dev(f_np) - tau * dirn, s, eps)) / (2 * tau)
    an_f = float((gf * dirn).sum())
    fd_s = (J_of(dev(f_np), s * (1 + tau), eps) - J_of(dev(f_np), s * (1 - tau), eps)) / (2 * tau * s)
    fd_e = (J_of(dev(f_np), s, eps * (1 + tau)) - J_of(dev(f_np), s, eps * (1 - tau))) / (2 * tau * eps)
    print(f"fd f {fd_f:.10e} {an_f:.10e}; s {fd_s:.10e} {gs:.10e}; eps {fd_e:.10e} {ge:.10e}", flush=True)
    assert abs(an_f - fd_f) <= 1e-6 * abs(fd_f)
    assert abs(gs - fd_s) <= 1e-6 * abs(fd_s)
    assert abs(ge - fd_e) <= 1e-6 * abs(fd_e)


def test_adjoint_full_size_defining_equation(psd):
    """Config C5 shape (128^3, batch 2 here): the GPU lam satisfies H lam = g,
    checked with the oracle's Hessian-vector product (one application)."""
    ws = psd_inputs.config5(batch=2)
    P = [psd.Problem(3, w.n, w.L, 4, w.p, w.s, w.eps) for w in ws]
    with psd.Solver(P, tol=1e-12, max_iter=500, precision="mixed", graph_chunk=4) as S:
        fs = [dev(w.f) for w in ws]
        us = [torch.zeros_like(f) for f in fs]
        stats = S.solve(fs, us)
        assert all(st.status == 0 for st in stats)
        h3 = (ws[0].L / ws[0].n) ** 3
        gs = [h3 * (u - dev(w.u_target)) for u, w in zip(us, ws)]
        lam, ds, de, it = S.adjoint(us, gs, rtol=1e-12, max_iter=500)
    print(f"C5 cg iters {it}", flush=True)
    w = ws[0]
    O = oracle.Problem(3, w.n, w.L, p=w.p, s=w.s, eps=w.eps)
    Hl = O.hessvec(host(us[0]), host(lam[0]))
    g = host(gs[0])
    assert np.linalg.norm(Hl - g) <= 1e-10 * np.linalg.norm(g)


def test_adjoint_full_size_finite_differences(psd):
    """Config C5 shape (one 128^3 instance): dJ/df along a random direction,
    dJ/ds and dJ/deps from psd_adjoint against central differences of J
    through FP64 forward solves to 1e-13 (relative steps 1e-4)."""
    w = psd_inputs.config5(batch=1)[0]
    h3 = (w.L / w.n) ** 3
    f = dev(w.f)
    ut = dev(w.u_target)

    def J_of(ff, ss, ee):
        with psd.Solver(psd.Problem(3, w.n, w.L, 4, w.p, ss, ee), tol=1e-13, max_iter=500) as S:
            u = torch.zeros_like(ff)
            st = S.solve([ff], [u])[0]
            assert st.status == 0
        return 0.5 * h3 * float(((u - ut) ** 2).sum())

    P = psd.Problem(3, w.n, w.L, 4, w.p, w.s, w.eps)
    with psd.Solver(P, tol=1e-13, max_iter=500) as S:
        u = torch.zeros_like(f)
        st = S.solve([f], [u])[0]
        assert st.status == 0
        lam, ds, de, it = S.adjoint([u], [h3 * (u - ut)], rtol=1e-13, max_iter=500)
    tau = 1e-4
    dirn = dev(psd_inputs.white_noise(w.f.shape, 94))
    fd_f = (J_of(f + tau * dirn, w.s, w.eps) - J_of(f - tau * dirn, w.s, w.eps)) / (2 * tau)
    an_f = float((lam[0] * dirn).sum())
    fd_s = (J_of(f, w.s * (1 + tau), w.eps) - J_of(f, w.s * (1 - tau), w.eps)) / (2 * tau * w.s)
    fd_e = (J_of(f, w.s, w.eps * (1 + tau)) - J_of(f, w.s, w.eps * (1 - tau))) / (2 * tau * w.eps)
    print(f"C5 shape: cg {it[0]}; f {fd_f:.10e} {an_f:.10e}; s {fd_s:.10e} {ds[0]:.10e}; "
          f"eps {fd_e:.10e} {de[0]:.10e}", flush=True)
    assert abs(an_f - fd_f) <= 1e-6 * abs(fd_f)
    assert abs(ds[0] - fd_s) <= 1e-6 * abs(fd_s)
    assert abs(de[0] - fd_e) <= 1e-6 * abs(fd_e)
