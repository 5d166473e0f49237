"""Every stencil tiling and row-transform layout the autotuner may pick gives
the oracle's iterates.

The 3D residual and line-search kernels march z-chunks of planes in whole
groups of six steps; the chunk, the block order (natural or XCD-grouped) and
the line-search tile width (32 or 64 cells) are tuning choices, and so is the
number of lines per block of the row transforms (layouts 0, 1, 2).  Each
candidate is forced through the tuning cache (PSD_TUNE_CACHE) and four FP64
PSD updates are compared with four oracle updates (1e-11 relative), at n = 96
(chunks that end mid-grid) and n = 128.  The chunk 46 of the residual is the
one the autotuner picks at 256^3 (whole grid in one round of resident blocks),
so its last chunk is partial at every n tested here.  A 2D case covers the
row layouts at 1024 points per line (one and four lines per block).
"""
import os

import numpy as np
import pytest

import oracle
import psd_inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# (residual z-chunk, line-search z-chunk, XCD order residual, XCD order line search, tile width,
#  row-transform layout)
TILINGS = [(16, 12, 0, 0, 32, 1), (28, 24, 1, 0, 64, 0), (40, 36, 0, 1, 64, 2), (46, 36, 1, 1, 64, 1),
           (64, 60, 0, 0, 32, 2), (46, 36, 1, 1, 32, 0), (64, 36, 1, 1, 64, 1), (28, 60, 0, 1, 32, 2),
           (16, 54, 1, 1, 64, 0)]
KUPD = 4


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


@pytest.mark.parametrize("n", [96, 128])
def test_forced_tilings_match_oracle(psd, n, tmp_path, monkeypatch):
    L = 12.8
    f = psd_inputs.small_field(3, n, L, 211, K=8, noise=0.01)
    O = oracle.Problem(3, n, L, p=4.0, s=0.01, eps=0.1)
    ref = O.solve(f, tol=0.0, max_iter=KUPD)["u"]
    arch = torch.cuda.get_device_properties(0).gcnArchName
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("PSD_TUNE_CACHE", str(cache))
    P = psd.Problem(3, n, L, 4, 4.0, 0.01, 0.1)
    for t in TILINGS:
        cache.write_text(f"{arch} d3 o4 fp64 n{n}|{' '.join(str(v) for v in t)}\n")
        with psd.Solver(P, tol=0.0, max_iter=KUPD, autotune=True) as S:
            got = S.tuning()
            u = torch.zeros_like(dev(f))
            st = S.solve([dev(f)], [u])[0]
        e = np.abs(host(u) - ref).max() / np.abs(ref).max()
        print(f"case n={n} tiling {t}: handle {got} rel {e:.2e}", flush=True)
        assert tuple(got) == t
        assert st.iters == KUPD
        assert e <= 1e-11


@pytest.mark.parametrize("layout", [0, 1, 2])
def test_row_layouts_2d(psd, layout, tmp_path, monkeypatch):
    """2D at 1024^2 (p = 4, mixed form: FP32 row transforms): every row layout
    gives the same iterates as the oracle within the mixed-form bound after
    three updates, and the layout is the one forced."""
    w = psd_inputs.config2(4.0)
    arch = torch.cuda.get_device_properties(0).gcnArchName
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("PSD_TUNE_CACHE", str(cache))
    cache.write_text(f"{arch} d2 o4 mixed n{w.n}|16 12 0 0 32 {layout}\n")
    P = psd.Problem(2, w.n, w.L, 4, w.p, w.s, w.eps)
    with psd.Solver(P, tol=1e-10, max_iter=500, precision="mixed", autotune=True) as S:
        got = S.tuning()
        u = torch.zeros_like(dev(w.f))
        st = S.solve([dev(w.f)], [u])[0]
    O = oracle.Problem(2, w.n, w.L, p=w.p, s=w.s, eps=w.eps)
    print(f"case 2D 1024 row layout {layout}: handle {got}, iters {st.iters}", flush=True)
    assert got[5] == layout
    assert st.status == 0 and st.res_inf <= 1e-10
    assert np.abs(O.residual(w.f, host(u))).max() <= 1.5e-10
