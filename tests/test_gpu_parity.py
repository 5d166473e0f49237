"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bars (from the arithmetic, stated per test): FP64 operators to ~1e-13
relative; FP64 solves to 1e-11 relative max-norm at residual <= 1e-10 with
iteration counts within +-1, and at matched iteration counts to ~1e-12.
"""
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


def log(msg):
    print(msg, flush=True)


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


# --------------------------------------------------------------------------
# operator parity
# --------------------------------------------------------------------------
CASES = [(2, 64, 4.0), (2, 96, 4.0), (2, 48, 3.0), (2, 128, 2.0), (3, 32, 4.0), (3, 48, 4.0),
         (3, 64, 2.5)]


@pytest.mark.parametrize("dim,n,p", CASES)
def test_residual_energy_grad_parity(psd, dim, n, p):
    log(f"case residual dim={dim} n={n} p={p}")
    L = 12.8 * n / 64
    P = psd.Problem(dim, n, L, 4, p, 0.01, 0.1)
    O = oracle.Problem(dim, n, L, p=p, s=0.01, eps=0.1)
    f = psd_inputs.small_field(dim, n, L, 11)
    u = psd_inputs.small_field(dim, n, L, 12, K=5) + 0.01 * psd_inputs.white_noise(f.shape, 13)
    with psd.Solver(P) as S:
        r = torch.empty_like(dev(f))
        rinf = S.residual(0, dev(f), dev(u), r=r)
        r_ref = O.residual(f, u)
        scale = np.abs(O.N4(u)).max()
        assert np.abs(host(r) - r_ref).max() <= 1e-13 * scale
        assert abs(rinf - np.abs(r_ref).max()) <= 1e-13 * scale
        E = S.energy(0, dev(f), dev(u))
        assert abs(E - O.energy(f, u)) <= 1e-13 * abs(E)
        g = S.grad(0, dev(f), dev(u))
        assert np.abs(host(g) + r_ref).max() <= 1e-13 * scale


def test_residual_parity_order6(psd):
    n, L = 96, 12.8
    P = psd.Problem(2, n, L, 6, 4.0, 0.02, 0.1, 1.0)
    O = oracle.Problem(2, n, L, order=6, p=4.0, s=0.02, eps=0.1, lam=1.0)
    f = psd_inputs.small_field(2, n, L, 21)
    g = psd_inputs.small_field(2, n, L, 22)
    u = psd_inputs.small_field(2, n, L, 23, K=5) + g.mean()
    w = psd_inputs.small_field(2, n, L, 24, K=5)
    with psd.Solver(P) as S:
        r = torch.empty_like(dev(f))
        S.residual(0, dev(f), dev(u), g=dev(g), r=r)
        rho = O.residual(f, u, g)
        assert np.abs(host(r) - rho).max() <= 1e-12 * np.abs(rho).max()
        r1, r2 = torch.empty_like(r), torch.empty_like(r)
        S.residual_mixed(0, dev(f), dev(g), dev(u), dev(w), r1=r1, r2=r2)
        e1, e2 = O.mixed_residuals(f, g, u, w)
        assert np.abs(host(r1) - e1).max() <= 1e-12 * max(1, np.abs(e1).max())
        assert np.abs(host(r2) - e2).max() <= 1e-12 * max(1, np.abs(e2).max())
        E = S.energy(0, dev(f), dev(u), g=dev(g))
        assert abs(E - O.energy(f, u, g)) <= 1e-12 * abs(E)


# --------------------------------------------------------------------------
# solve parity (FP64)
# --------------------------------------------------------------------------
SOLVES = [(2, 64, 4.0, 12.8, 0.01, 0.1), (2, 96, 4.0, 12.8, 0.01, 0.1), (2, 128, 3.0, 25.6, 0.005, 0.05),
          (3, 32, 4.0, 12.8, 0.01, 0.1), (3, 48, 4.0, 12.8, 0.01, 0.1),
          # wide (64-column) line-search tiles, one of them partial
          (3, 96, 4.0, 12.8, 0.01, 0.1),
          # 3D general p: line search by (q, q') evaluations and the host root rule
          (3, 32, 3.0, 12.8, 0.01, 0.1),
          # p = 6: quintic q (Sec. 6.1), one line-search pass; the oracle finds
          # the same root by (q, q') grid evaluations
          (2, 64, 6.0, 12.8, 0.01, 0.1), (2, 96, 6.0, 3.2, 0.001, 0.1), (3, 32, 6.0, 12.8, 0.01, 0.1)]


@pytest.mark.parametrize("dim,n,p,L,s,eps", SOLVES)
def test_solve_parity_fp64(psd, dim, n, p, L, s, eps):
    log(f"case solve dim={dim} n={n} p={p}")
    f = psd_inputs.small_field(dim, n, L, 31, K=6)
    O = oracle.Problem(dim, n, L, p=p, s=s, eps=eps)
    ref = O.solve(f, tol=1e-10, max_iter=300, history=True)
    P = psd.Problem(dim, n, L, 4, p, s, eps)
    with psd.Solver(P, tol=1e-10, max_iter=300, history=True) as S:
        u = torch.zeros_like(dev(f))
        st = S.solve([dev(f)], [u])[0]
        hist = S.history(0)
    assert st.status == 0 and st.res_inf <= 1e-10
    assert abs(st.iters - ref["iters"]) <= 1
    ug = host(u)
    if st.iters == ref["iters"]:
        assert rel(ug, ref["u"]) <= 1e-11
    # step sizes agree (same iterate sequence up to rounding): per-update
    # bound from the residual's rounding scale (parity_bounds)
    check_alphas(hist[:, 0], ref["hist"][:, 0], ref["hist"][:, 1], np.abs(f).max(),
                 rounding_scale(O, ref["u"]), f.size, log)
    if p in (4.0, 6.0):
        # the energy decrease integrated from the GPU's polynomial q against
        # the oracle's energies before and after each update (Sec. 2.2, 6.1)
        k = min(len(hist), len(ref["hist"]))
        E = np.concatenate([[O.energy(f, np.zeros_like(f))], ref["hist"][:k, 3]])
        dE_ref = np.diff(E)
        err = np.abs(hist[:k, 3] - dE_ref)
        log(f"  dE: worst |diff| {err.max():.2e} (|E0| {abs(E[0]):.2e})")
        assert (err <= 1e-12 * abs(E[0]) + 1e-9 * np.abs(dE_ref)).all()
    # matched iteration count
    kk = max(ref["iters"] - 2, 1)
    with psd.Solver(P, tol=0.0, max_iter=kk) as S:
        u = torch.zeros_like(dev(f))
        st = S.solve([dev(f)], [u])[0]
    ref_k = O.solve(f, tol=0.0, max_iter=kk)
    assert st.iters == kk and st.status == 1
    assert rel(host(u), ref_k["u"]) <= 1e-11
    # the converged GPU iterate solves the oracle's discrete equation
    assert np.abs(O.residual(f, ug)).max() <= 1.5e-10


@pytest.mark.parametrize("p,k", [(6.0, 6), (3.0, 4)])
def test_wide_tiles_general_p_matched_count(psd, p, k):
    """p = 6 (quintic) and p = 3 (root search by (q, q') passes) in 3D at
    n = 64 (64-wide line-search tiles): k FP64 updates and their step sizes
    against k oracle updates (the oracle's general-p root rule at 64^3 takes
    minutes to convergence, so the count is fixed)."""
    n, L, s, eps = 64, 12.8, 0.01, 0.1
    f = psd_inputs.small_field(3, n, L, 31, K=6)
    O = oracle.Problem(3, n, L, p=p, s=s, eps=eps)
    ref = O.solve(f, tol=0.0, max_iter=k, history=True)
    P = psd.Problem(3, n, L, 4, p, s, eps)
    with psd.Solver(P, tol=0.0, max_iter=k, history=True) as S:
        u = torch.zeros_like(dev(f))
        st = S.solve([dev(f)], [u])[0]
        hist = S.history(0)
    log(f"case p={p:g} 3D n={n}: {st.iters} updates, rel {rel(host(u), ref['u']):.2e}")
    assert st.iters == k
    assert rel(host(u), ref["u"]) <= 1e-11
    check_alphas(hist[:, 0], ref["hist"][:, 0], ref["hist"][:, 1], np.abs(f).max(),
                 rounding_scale(O, ref["u"]), f.size, log)


def test_solve_parity_config1(psd):
    w = psd_inputs.config1()
    O = oracle.Problem(2, w.n, w.L, p=w.p, s=w.s, eps=w.eps)
    ref = O.solve(w.f, tol=1e-10, max_iter=300)
    with psd.Solver(psd.Problem(2, w.n, w.L, 4, w.p, w.s, w.eps), tol=1e-10, max_iter=300) as S:
        u = torch.zeros_like(dev(w.f))
        st = S.solve([dev(w.f)], [u])[0]
    log(f"config1: gpu iters {st.iters} oracle iters {ref['iters']}")
    assert st.status == 0 and abs(st.iters - ref["iters"]) <= 1
    if st.iters == ref["iters"]:
        assert rel(host(u), ref["u"]) <= 1e-11


def order6_inputs(n, L, seed, gbar=0.0, fbar=0.0):
    """Seeded sixth-order right-hand sides; gbar, fbar shift the means (the
    mean handling of Sec. 4 and Sec. 5.4 runs only when they are non-zero)."""
    f = psd_inputs.small_field(2, n, L, seed, K=6) + fbar
    g = psd_inputs.small_field(2, n, L, seed + 1, K=6) + gbar
    return f, g


# n = 192 takes the radix-3 transform; n = 96 has non-zero means of f and g
@pytest.mark.parametrize("n,gbar,fbar", [(64, 0.0, 0.0), (96, 0.3, -0.2), (192, 0.0, 0.0)])
def test_solve_parity_order6(psd, n, gbar, fbar):
    L, s, eps, lam = 12.8, 0.02, 0.1, 1.0
    f, g = order6_inputs(n, L, 41, gbar, fbar)
    O = oracle.Problem(2, n, L, order=6, p=4.0, s=s, eps=eps, lam=lam)
    ref = O.solve(f, g=g, tol=1e-10, max_iter=300, history=True)
    P = psd.Problem(2, n, L, 6, 4.0, s, eps, lam)
    with psd.Solver(P, tol=1e-10, max_iter=300, history=True) as S:
        u = torch.full_like(dev(f), float(g.mean()))
        w = torch.zeros_like(u)
        st = S.solve([dev(f)], [u], g=[dev(g)], w=[w])[0]
        hist = S.history(0)
    log(f"order6 n={n} gbar={gbar} fbar={fbar}: gpu iters {st.iters} oracle iters {ref['iters']}")
    # the GPU stops on max(|r1|, |r2|) of the mixed system, the oracle on the
    # reduced residual rho: equal in exact arithmetic (carried w consistent)
    assert st.status == 0 and abs(st.iters - ref["iters"]) <= 1
    r1, r2 = O.mixed_residuals(f, g, host(u), host(w))
    assert np.abs(r1).max() <= 2e-10 and np.abs(r2).max() <= 2e-10
    check_alphas(hist[:, 0], ref["hist"][:, 0], ref["hist"][:, 1],
                 np.abs(O.residual(f, np.full_like(f, g.mean()), g)).max(),
                 rounding_scale(O, ref["u"], ref["w"]), f.size, log)
    # matched iteration count: u and the carried w against the oracle's u and
    # w = T_h[g - u] + s lam gbar - fbar (Sec. 4)
    kk = ref["iters"]
    with psd.Solver(P, tol=0.0, max_iter=kk) as S:
        u = torch.full_like(dev(f), float(g.mean()))
        w = torch.zeros_like(u)
        st = S.solve([dev(f)], [u], g=[dev(g)], w=[w])[0]
    ref_k = O.solve(f, g=g, tol=0.0, max_iter=kk)
    assert st.iters == kk and st.status == 1
    ug, wg = host(u), host(w)
    log(f"  matched k={kk}: u {rel(ug, ref_k['u']):.2e} w {rel(wg, ref_k['w']):.2e}")
    assert rel(ug, ref_k["u"]) <= 1e-11
    assert rel(wg, ref_k["w"]) <= 1e-11
    # conservation (Sec. 4): mean(u) = gbar, mean(w) = s lam gbar - fbar
    assert abs(ug.mean() - g.mean()) <= 1e-13 * (1 + abs(g.mean()))
    assert abs(wg.mean() - (s * lam * g.mean() - f.mean())) <= 1e-12 * (1 + np.abs(wg).max())


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_order6_nonzero_means(psd, precision):
    """Sixth-order instances of three sizes with different non-zero means of f
    and g in one handle (graph-captured): each against its own oracle solve,
    with the conservation of Sec. 4."""
    sizes, L, s, eps, lam = [64, 96, 192], 12.8, 0.02, 0.1, 1.0
    means = [(0.25, -0.4), (-0.3, 0.15), (0.1, 0.5)]
    data = [order6_inputs(n, L, 140 + 2 * i, gb, fb) for i, (n, (gb, fb)) in enumerate(zip(sizes, means))]
    probs = [psd.Problem(2, n, L, 6, 4.0, s, eps, lam) for n in sizes]
    log(f"case batched order 6 with means, {precision}")
    with psd.Solver(probs, tol=1e-10, max_iter=300, precision=precision, graph_chunk=4) as S:
        us = [torch.full_like(dev(f), float(g.mean())) for f, g in data]
        ws = [torch.zeros_like(u) for u in us]
        stats = S.solve([dev(f) for f, _ in data], us, g=[dev(g) for _, g in data], w=ws)
    for (f, g), n, u, w, st in zip(data, sizes, us, ws, stats):
        O = oracle.Problem(2, n, L, order=6, p=4.0, s=s, eps=eps, lam=lam)
        ref = O.solve(f, g=g, tol=1e-10, max_iter=300)
        ug, wg = host(u), host(w)
        assert st.status == 0 and st.res_inf <= 1e-10
        r1, r2 = O.mixed_residuals(f, g, ug, wg)
        assert np.abs(r1).max() <= 2e-10 and np.abs(r2).max() <= 2e-10
        same_k = precision == "fp64" and st.iters == ref["iters"]
        if precision == "fp64":
            assert abs(st.iters - ref["iters"]) <= 1
        assert rel(ug, ref["u"]) <= (1e-11 if same_k else 1e-9)
        assert rel(wg, ref["w"]) <= (1e-11 if same_k else 1e-9)
        assert abs(ug.mean() - g.mean()) <= 1e-13 * (1 + abs(g.mean()))
        assert abs(wg.mean() - (s * lam * g.mean() - f.mean())) <= 1e-12 * (1 + np.abs(wg).max())


# --------------------------------------------------------------------------
# mixed precision, graphs, batching
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dim,n,p", [(2, 128, 4.0), (3, 48, 4.0), (3, 32, 3.0), (2, 128, 6.0), (3, 48, 6.0)])
def test_mixed_precision_reaches_fp64_answer(psd, dim, n, p):
    L = 12.8
    f = psd_inputs.small_field(dim, n, L, 51, K=6)
    O = oracle.Problem(dim, n, L, p=p, s=0.01, eps=0.1)
    ref = O.solve(f, tol=1e-12, max_iter=300)
    P = psd.Problem(dim, n, L, 4, p, 0.01, 0.1)
    with psd.Solver(P, tol=1e-10, max_iter=300, precision="mixed") as S:
        u = torch.zeros_like(dev(f))
        st = S.solve([dev(f)], [u])[0]
    log(f"mixed dim={dim} n={n}: iters {st.iters} (oracle to 1e-12: {ref['iters']})")
    assert st.status == 0 and st.res_inf <= 1e-10
    # FP64 residual verified by the oracle; error against the FP64 answer
    assert np.abs(O.residual(f, host(u))).max() <= 1.5e-10
    assert rel(host(u), ref["u"]) <= 1e-9


# p = 3 and 2.5: general p, the root search runs a fixed number of evaluation
# passes per captured iteration; while none is cut short the graph replays
# give the host-driven loop's iterates bit for bit
@pytest.mark.parametrize("precision,p,dim,n", [("fp64", 4.0, 3, 48), ("mixed", 4.0, 3, 48), ("mixed", 6.0, 3, 48),
                                              ("fp64", 3.0, 3, 48), ("mixed", 2.5, 2, 48),
                                              # 64-wide line-search tiles
                                              ("mixed", 4.0, 3, 64), ("mixed", 3.0, 3, 64)])
def test_graph_mode_matches_stream_mode(psd, precision, p, dim, n):
    L = 12.8
    f = psd_inputs.small_field(dim, n, L, 61, K=6)
    P = psd.Problem(dim, n, L, 4, p, 0.01, 0.1)
    out = []
    for chunk in (0, 4):
        with psd.Solver(P, tol=1e-10, max_iter=300, precision=precision, graph_chunk=chunk) as S:
            for rep in range(2):
                u = torch.zeros_like(dev(f))
                st = S.solve([dev(f)], [u])[0]
                assert st.status == 0 and st.ls_truncated == 0
                out.append((st.iters, host(u)))
    assert all(o[0] == out[0][0] for o in out)
    for o in out[1:]:
        assert np.array_equal(o[1], out[0][1])  # deterministic, bitwise


def test_batched_instances_match_single(psd):
    sizes = [64, 96, 128, 64]
    probs, fs = [], []
    for i, n in enumerate(sizes):
        probs.append(psd.Problem(2, n, 12.8, 6, 4.0, 0.02, 0.1, 1.0))
        fs.append((psd_inputs.small_field(2, n, 12.8, 70 + 2 * i, K=6),
                   psd_inputs.small_field(2, n, 12.8, 71 + 2 * i, K=6)))
    with psd.Solver(probs, tol=1e-10, max_iter=300, precision="mixed", graph_chunk=4) as S:
        us = [torch.full_like(dev(f), float(g.mean())) for f, g in fs]
        ws = [torch.zeros_like(u) for u in us]
        stats = S.solve([dev(f) for f, _ in fs], us, g=[dev(g) for _, g in fs], w=ws)
    for (f, g), n, u, w, st in zip(fs, sizes, us, ws, stats):
        O = oracle.Problem(2, n, 12.8, order=6, p=4.0, s=0.02, eps=0.1, lam=1.0)
        assert st.status == 0 and st.res_inf <= 1e-10
        r1, r2 = O.mixed_residuals(f, g, host(u), host(w))
        assert np.abs(r1).max() <= 2e-10 and np.abs(r2).max() <= 2e-10
        ref = O.solve(f, g=g, tol=1e-11, max_iter=300)
        assert rel(host(u), ref["u"]) <= 1e-9


@pytest.mark.parametrize("dim,n,mode", [(2, 256, "one_iteration"), (2, 256, "solve"),
                                        (2, 128, "one_iteration"), (2, 128, "solve"),
                                        (3, 128, "one_iteration")])
def test_register_transforms_mixed(psd, dim, n, mode):
    """FP32 lines of 128 and 256 points take the register four-step transform
    (y passes and the fused last axis; 2D grids include the one-column Nyquist
    block): one mixed iteration from zero against the oracle's to FP32
    accuracy, and a full mixed solve against the oracle's solution."""
    L = 0.1 * n
    # the noise puts energy in every mode, the Nyquist lines included
    f = psd_inputs.small_field(dim, n, L, 41, K=8, noise=0.05)
    O = oracle.Problem(dim, n, L, p=4.0, s=0.01, eps=0.1)
    P = psd.Problem(dim, n, L, 4, 4.0, 0.01, 0.1)
    log(f"case {dim}D n={n} mixed {mode}")
    if mode == "one_iteration":
        with psd.Solver(P, tol=0.0, max_iter=1, precision="mixed") as S:
            u = torch.zeros_like(dev(f))
            S.solve([dev(f)], [u])
        ref = O.solve(f, tol=0.0, max_iter=1)
        # FP32 residual and spectrum: the step is exact to about 1e-7 relative
        assert rel(host(u), ref["u"]) <= 2e-6
    else:
        with psd.Solver(P, tol=1e-10, max_iter=300, precision="mixed", graph_chunk=4) as S:
            u = torch.zeros_like(dev(f))
            st = S.solve([dev(f)], [u])[0]
        assert st.status == 0 and st.res_inf <= 1e-10
        ref = O.solve(f, tol=1e-10, max_iter=300)
        assert rel(host(u), ref["u"]) <= 1e-9
        assert np.abs(O.residual(f, host(u))).max() <= 1.5e-10


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_degenerate_inputs(psd, precision):
    """Degenerate cases: f = 0 from u0 = 0 (the residual is zero at the
    start: no iteration), a restart from a converged answer (no iteration,
    the answer untouched), and the smallest grid (2D 16^2) against the oracle."""
    n, L = 16, 3.2
    P = psd.Problem(2, n, L, 4, 4.0, 0.01, 0.1)
    log(f"case degenerate {precision}")
    with psd.Solver(P, tol=1e-10, max_iter=50, precision=precision) as S:
        z = torch.zeros((n, n), dtype=torch.float64, device="cuda")
        u = torch.zeros_like(z)
        st = S.solve([z], [u])[0]
        assert st.status == 0 and st.iters == 0 and st.res_inf == 0.0
        assert not bool(u.abs().max() > 0)
    f = psd_inputs.small_field(2, n, L, 71, K=4, noise=0.05)
    O = oracle.Problem(2, n, L, p=4.0, s=0.01, eps=0.1)
    ref = O.solve(f, tol=1e-10, max_iter=300)
    with psd.Solver(P, tol=1e-10, max_iter=300, precision=precision) as S:
        u = torch.zeros_like(dev(f))
        st = S.solve([dev(f)], [u])[0]
        assert st.status == 0 and st.res_inf <= 1e-10
        if precision == "fp64":
            assert abs(st.iters - ref["iters"]) <= 1
        assert rel(host(u), ref["u"]) <= (1e-11 if precision == "fp64" and st.iters == ref["iters"] else 1e-9)
        # restart from the converged answer
        u_conv = host(u).copy()
        st2 = S.solve([dev(f)], [u])[0]
        assert st2.status == 0 and st2.iters == 0
        assert np.array_equal(host(u), u_conv)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_mode_edge_cases(psd, precision):
    """Graph-mode solves read the device states of one batch of replays while
    the next batch runs: a zero residual at the start (no update, the iterate
    untouched), a restart from a converged answer, and a stop at max_iter in
    the middle of a captured chunk (status PSD_NOT_CONVERGED, the same
    iterate as the host-driven loop after max_iter updates, bit for bit)."""
    n, L = 48, 9.6
    P = psd.Problem(2, n, L, 4, 4.0, 0.01, 0.1)
    log(f"case graph edge {precision}")
    with psd.Solver(P, tol=1e-10, max_iter=50, precision=precision, graph_chunk=4) as S:
        z = torch.zeros((n, n), dtype=torch.float64, device="cuda")
        u = torch.zeros_like(z)
        st = S.solve([z], [u])[0]
        assert st.status == 0 and st.iters == 0 and st.res_inf == 0.0
        assert not bool(u.abs().max() > 0)
    f = psd_inputs.small_field(2, n, L, 73, K=5)
    with psd.Solver(P, tol=1e-10, max_iter=300, precision=precision, graph_chunk=4) as S:
        u = torch.zeros_like(dev(f))
        st = S.solve([dev(f)], [u])[0]
        assert st.status == 0 and st.res_inf <= 1e-10
        u_conv = host(u).copy()
        st2 = S.solve([dev(f)], [u])[0]
        assert st2.status == 0 and st2.iters == 0
        assert np.array_equal(host(u), u_conv)
    out = []
    for chunk in (0, 4):
        with psd.Solver(P, tol=1e-30, max_iter=7, precision=precision, graph_chunk=chunk) as S:
            u = torch.zeros_like(dev(f))
            st = S.solve([dev(f)], [u])[0]
            assert st.status == 1 and st.iters == 7
            out.append(host(u))
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_3d_sizes_match_oracle(psd, precision):
    """3D instances of different n in one handle: every FFT pass runs as one
    launch over both sizes (per-block length switch); narrow line-search tiles."""
    sizes = [32, 48]
    probs = [psd.Problem(3, n, 12.8, 4, 4.0, 0.01, 0.1) for n in sizes]
    fs = [psd_inputs.small_field(3, n, 12.8, 90 + i, K=5) for i, n in enumerate(sizes)]
    log(f"case batched 3D sizes {sizes} {precision}")
    with psd.Solver(probs, tol=1e-10, max_iter=300, precision=precision, graph_chunk=4) as S:
        us = [torch.zeros_like(dev(f)) for f in fs]
        stats = S.solve([dev(f) for f in fs], us)
    for f, n, u, st in zip(fs, sizes, us, stats):
        O = oracle.Problem(3, n, 12.8, p=4.0, s=0.01, eps=0.1)
        assert st.status == 0 and st.res_inf <= 1e-10
        ref = O.solve(f, tol=1e-10, max_iter=300)
        if precision == "fp64":
            assert abs(st.iters - ref["iters"]) <= 1
        assert rel(host(u), ref["u"]) <= (1e-11 if precision == "fp64" and st.iters == ref["iters"] else 1e-9)
        assert np.abs(O.residual(f, host(u))).max() <= 1.5e-10


def test_autotuned_tiling_gives_same_solution(psd):
    n, L = 64, 12.8
    f = psd_inputs.small_field(3, n, L, 101, K=6)
    P = psd.Problem(3, n, L, 4, 4.0, 0.01, 0.1)
    res = []
    for tune in (False, True):
        with psd.Solver(P, tol=1e-10, max_iter=300, precision="mixed", autotune=tune) as S:
            t = S.tuning()
            # residual / line-search z-chunks run whole groups of six plane steps
            # (the residual's chunk + 2, the line search's chunk)
            assert t[0] >= 12 and (t[0] + 2) % 6 == 0 and t[1] >= 12 and t[1] % 6 == 0
            u = torch.zeros_like(dev(f))
            st = S.solve([dev(f)], [u])[0]
            res.append((st.iters, host(u), t))
    log(f"autotune: tuning {res[1][2]}")
    assert abs(res[0][0] - res[1][0]) <= 1
    assert rel(res[1][1], res[0][1]) <= 1e-10
