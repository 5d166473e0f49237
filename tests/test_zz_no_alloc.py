"""psd_solve_noalloc (workspace in the library's static scratch array) against
psd_create + psd_solve + psd_destroy on the same inputs.

Both run the same kernels with the same default tiling and the host-driven
loop, so the results must agree bit for bit: iteration counts, final
iterates, w (order 6) and the residual norms.  Each case is two calls in a
row on one GPU, the second with a smaller grid, so the second call runs on
the array as the first left it.  The iterates are also held to the oracle at
the converged count.
"""
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


# (dim, n, order, precision, mean of g, mean of f): pairs of calls, larger grid first
SEQUENCES = {
    "2d_o4_fp64": [(2, 128, 4, "fp64", 0.0, 0.0), (2, 64, 4, "fp64", 0.0, 0.0)],
    "3d_o4_mixed": [(3, 48, 4, "mixed", 0.0, 0.0), (3, 32, 4, "mixed", 0.0, 0.0)],
    "2d_o6_fp64_means": [(2, 96, 6, "fp64", 0.3, -0.2), (2, 64, 6, "fp64", -0.1, 0.4)],
}


def inputs(dim, n, order, gbar, fbar, seed):
    L = 12.8
    f = psd_inputs.small_field(dim, n, L, seed, K=5) + fbar
    g = psd_inputs.small_field(dim, n, L, seed + 1, K=5) + gbar if order == 6 else None
    return L, f, g


@pytest.mark.parametrize("name", list(SEQUENCES))
def test_noalloc_matches_handle_solve(psd, name):
    for call, (dim, n, order, prec, gbar, fbar) in enumerate(SEQUENCES[name]):
        print(f"case {name} call {call}: dim={dim} n={n} order={order} {prec}", flush=True)
        L, f, g = inputs(dim, n, order, gbar, fbar, 300 + 10 * call)
        lam, s = (1.0, 0.02) if order == 6 else (0.0, 0.01)
        P = psd.Problem(dim, n, L, order, 4.0, s, 0.1, lam)
        u0 = np.full_like(f, g.mean()) if order == 6 else np.zeros_like(f)
        gd = dev(g) if g is not None else None
        # reference: the allocating entry points
        with psd.Solver(P, tol=1e-10, max_iter=300, precision=prec) as S:
            u_ref = dev(u0)
            w_ref = torch.zeros_like(u_ref) if order == 6 else None
            st_ref = S.solve([dev(f)], [u_ref], g=[gd] if gd is not None else None,
                             w=[w_ref] if w_ref is not None else None)[0]
        u = dev(u0)
        w = torch.zeros_like(u) if order == 6 else None
        st = psd.solve_noalloc(P, dev(f), u, g=gd, w=w, tol=1e-10, max_iter=300, precision=prec)
        assert st.status == 0 and st_ref.status == 0
        assert st.iters == st_ref.iters
        assert st.res_inf == st_ref.res_inf and st.res_l2 == st_ref.res_l2
        assert np.array_equal(host(u), host(u_ref))
        if order == 6:
            assert np.array_equal(host(w), host(w_ref))
        # and the oracle at the converged count
        O = oracle.Problem(dim, n, L, order=order, p=4.0, s=s, eps=0.1, lam=lam)
        ref = O.solve(f, g=g, tol=0.0, max_iter=st.iters)
        e = np.abs(host(u) - ref["u"]).max() / np.abs(ref["u"]).max()
        print(f"  iters {st.iters} rel vs oracle {e:.2e}", flush=True)
        assert e <= (1e-11 if prec == "fp64" else 1e-9)


def test_noalloc_rejects_what_it_cannot_run(psd):
    # workspace larger than the static array: an argument error, nothing runs
    P = psd.Problem(3, 256, 12.8, 4, 4.0, 0.01, 0.1)
    f = torch.zeros((256,) * 3, dtype=torch.float64, device="cuda")
    u = torch.zeros_like(f)
    with pytest.raises(psd.PSDError) as ei:
        psd.solve_noalloc(P, f, u)
    assert ei.value.status == psd.PSD_ERR_ARG and "scratch" in str(ei.value)
    # graph capture, profiling and autotuning need allocations: refused
    import ctypes
    lib = psd.load_library()
    P2 = psd.Problem(2, 64, 12.8)
    f2 = torch.zeros((64, 64), dtype=torch.float64, device="cuda")
    u2 = torch.zeros_like(f2)
    opt = psd._Options(1e-10, 10, psd.PSD_FP64, 4, 0, 0, 0)
    rc = lib.psd_solve_noalloc(ctypes.byref(P2.c()), ctypes.byref(opt), None, ctypes.c_void_p(f2.data_ptr()),
                               None, ctypes.c_void_p(u2.data_ptr()), None, None)
    assert rc == psd.PSD_ERR_ARG


def test_noalloc_leaves_device_memory_unchanged(psd):
    n = 64
    P = psd.Problem(2, n, 12.8, 4, 4.0, 0.01, 0.1)
    f = dev(psd_inputs.small_field(2, n, 12.8, 5, K=5))
    u = torch.zeros_like(f)
    psd.solve_noalloc(P, f, u)          # warm-up (module and runtime set-up)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    u.zero_()
    st = psd.solve_noalloc(P, f, u)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert st.status == 0
    assert free1 == free0
