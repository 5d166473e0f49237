"""Full-size checks of the benchmark configurations (C1-C5 shapes).

At full size the oracle cannot run every solve, so these compare on what it
can compute: the oracle residual of the GPU result (one evaluation), matched
iteration prefixes, and complete oracle solves for sampled instances.
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


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("p", [4.0, 3.0])
def test_config2_1024(psd, p):
    w = psd_inputs.config2(p)
    print(f"case C2 p={p}", flush=True)
    O = oracle.Problem(2, w.n, w.L, p=w.p, s=w.s, eps=w.eps)
    P = psd.Problem(2, w.n, w.L, 4, w.p, w.s, w.eps)
    out = {}
    for prec in ("fp64", "mixed"):
        with psd.Solver(P, tol=1e-10, max_iter=500, precision=prec) as S:
            u = torch.zeros_like(dev(w.f))
            st = S.solve([dev(w.f)], [u])[0]
        assert st.status == 0, st
        out[prec] = (st.iters, host(u))
        # the FP64 residual of the GPU result, evaluated by the oracle
        assert np.abs(O.residual(w.f, out[prec][1])).max() <= 1.5e-10
    print(f"  iters fp64 {out['fp64'][0]} mixed {out['mixed'][0]}", flush=True)
    assert rel(out["mixed"][1], out["fp64"][1]) <= 1e-9
    # matched prefix: 3 iterations of both
    with psd.Solver(P, tol=0.0, max_iter=3) as S:
        u = torch.zeros_like(dev(w.f))
        S.solve([dev(w.f)], [u])
    ref = O.solve(w.f, tol=0.0, max_iter=3)
    assert rel(host(u), ref["u"]) <= 1e-11


def test_config3_256(psd):
    w = psd_inputs.config3()
    O = oracle.Problem(3, w.n, w.L, p=w.p, s=w.s, eps=w.eps)
    P = psd.Problem(3, w.n, w.L, 4, w.p, w.s, w.eps)
    us = {}
    for prec, chunk in (("fp64", 0), ("mixed", 4)):
        with psd.Solver(P, tol=1e-10, max_iter=500, precision=prec, graph_chunk=chunk) as S:
            u = torch.zeros_like(dev(w.f))
            st = S.solve([dev(w.f)], [u])[0]
        assert st.status == 0 and st.res_inf <= 1e-10
        us[prec] = host(u)
        print(f"case C3 {prec}: iters {st.iters}", flush=True)
    assert rel(us["mixed"], us["fp64"]) <= 1e-9
    # one oracle residual evaluation of the FP64 GPU answer at full size
    assert np.abs(O.residual(w.f, us["fp64"])).max() <= 1.5e-10
    # one oracle PSD iteration from zero vs one GPU iteration
    with psd.Solver(P, tol=0.0, max_iter=1) as S:
        u = torch.zeros_like(dev(w.f))
        S.solve([dev(w.f)], [u])
    ref = O.solve(w.f, tol=0.0, max_iter=1)
    assert rel(host(u), ref["u"]) <= 1e-12
    # the same iteration in mixed precision (FP32 residual and spectrum; the
    # 256-point y and z passes run the register four-step transform)
    with psd.Solver(P, tol=0.0, max_iter=1, precision="mixed") as S:
        u = torch.zeros_like(dev(w.f))
        S.solve([dev(w.f)], [u])
    assert rel(host(u), ref["u"]) <= 2e-6


def test_config4_batch64(psd):
    ws = psd_inputs.config4()
    P = [psd.Problem(2, w.n, w.L, 6, w.p, w.s, w.eps, w.lam) for w in ws]
    with psd.Solver(P, tol=1e-10, max_iter=500, precision="mixed", graph_chunk=4) as S:
        fs = [dev(w.f) for w in ws]
        gs = [dev(w.g) for w in ws]
        us = [torch.full_like(f, float(w.g.mean())) for f, w in zip(fs, ws)]
        wv = [torch.zeros_like(u) for u in us]
        stats = S.solve(fs, us, g=gs, w=wv)
    iters = [st.iters for st in stats]
    print(f"case C4: iters min {min(iters)} max {max(iters)}", flush=True)
    for w, u, ww, st in zip(ws, us, wv, stats):
        assert st.status == 0 and st.res_inf <= 1e-10
        O = oracle.Problem(2, w.n, w.L, order=6, p=w.p, s=w.s, eps=w.eps, lam=w.lam)
        r1, r2 = O.mixed_residuals(w.f, w.g, host(u), host(ww))
        assert np.abs(r1).max() <= 2e-10 and np.abs(r2).max() <= 2e-10
    # complete oracle solves for two sampled instances (smallest grids)
    order = sorted(range(len(ws)), key=lambda i: ws[i].n)[:2]
    for i in order:
        w = ws[i]
        O = oracle.Problem(2, w.n, w.L, order=6, p=w.p, s=w.s, eps=w.eps, lam=w.lam)
        ref = O.solve(w.f, g=w.g, tol=1e-11, max_iter=500)
        assert rel(host(us[i]), ref["u"]) <= 1e-9
