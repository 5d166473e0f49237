"""Host-only checks of the C ABI: the library loads, exports every symbol
declared in include/psd.h, and validates problems without a GPU."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1607_01475_amd", "libpsd.so")


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "psd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(psd_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def psd():
    if not os.path.exists(LIB):
        from paper_1607_01475_amd import build
        build.build()
    from paper_1607_01475_amd import psd as _psd
    _psd.load_library()
    return _psd


def test_exports_every_declared_symbol(psd):
    import ctypes
    lib = ctypes.CDLL(LIB)
    syms = declared_symbols()
    assert len(syms) >= 10
    for name in syms:
        assert hasattr(lib, name), name
    # the binding covers the same set
    assert set(syms) == set(psd.SIGNATURES)


@pytest.mark.parametrize("kw,status", [
    (dict(dim=2, n=64, L=12.8), 0),
    (dict(dim=3, n=256, L=12.8), 0),
    (dict(dim=2, n=1024, L=25.6, p=3.0, s=0.005, eps=0.05), 0),
    (dict(dim=2, n=192, L=12.8, order=6, lam=1.0, s=0.02), 0),
    (dict(dim=4, n=64, L=1.0), -1),
    (dict(dim=2, n=100, L=1.0), -1),
    (dict(dim=3, n=512, L=1.0), -1),
    (dict(dim=3, n=64, L=1.0, order=6, lam=1.0), 0),
    (dict(dim=2, n=64, L=-1.0), -2),
    (dict(dim=2, n=64, L=1.0, s=0.0), -2),
    (dict(dim=2, n=64, L=1.0, eps=0.0), -2),
    (dict(dim=2, n=64, L=1.0, eps=1.5), -2),
    (dict(dim=2, n=64, L=1.0, p=1.5), -2),
    (dict(dim=3, n=64, L=1.0, p=7.0), -2),
    (dict(dim=2, n=64, L=1.0, order=6, lam=-1.0), -2),
])
def test_check_problem(psd, kw, status):
    st, msg = psd.check_problem(psd.Problem(**kw))
    assert st == status, msg


def test_create_without_gpu_fails_cleanly(psd):
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    import ctypes
    lib = psd.load_library()
    P = (psd._Problem * 1)(psd.Problem(2, 64, 12.8).c())
    opt = psd._Options(1e-10, 10, 0, 0, 0, 0, 0)
    h = ctypes.c_void_p()
    st = lib.psd_create(P, 1, ctypes.byref(opt), None, ctypes.byref(h))
    assert st == psd.PSD_ERR_HIP
    assert b"device" in lib.psd_last_error(None)
