"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, validates parameters before touching the device, and sizes
its workspace consistently."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "sca.h")).read()
    return sorted(set(re.findall(r"SCA_API\s+[\w\s\*]*?\b(sca_\w+)\s*\(", txt)))


def test_header_declares_the_abi():
    syms = header_symbols()
    from paper_2311_04435_amd import _lib
    assert syms == sorted(_lib.EXPORTS)


def test_library_exports_every_header_symbol():
    from paper_2311_04435_amd import _lib
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH],
                         capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r" T (sca_\w+)", out))
    assert set(header_symbols()) <= exported
    # nothing but the C ABI is exported
    assert exported == set(header_symbols())
    for s in header_symbols():
        assert getattr(_lib.lib, s) is not None


def _params(**kw):
    from paper_2311_04435_amd import _lib
    d = dict(L=4, n_max=256, precision=0, factor=0, t=1.0, U=4.0, delta=0.0,
             T=0.1, onsite=None, tail=0, reserved=0)
    d.update(kw)
    return _lib.Params(d["L"], d["n_max"], d["precision"], d["factor"], d["t"],
                       d["U"], d["delta"], d["T"], d["onsite"], d["tail"],
                       d["reserved"])


@pytest.mark.parametrize("bad", [dict(L=3), dict(L=0), dict(L=66), dict(n_max=0),
                                 dict(U=0.0), dict(U=-1.0), dict(T=0.0),
                                 dict(T=float("nan")), dict(t=float("inf")),
                                 dict(precision=7), dict(factor=3),
                                 dict(tail=2), dict(reserved=1)])
def test_invalid_params_rejected_without_device(bad):
    from paper_2311_04435_amd import _lib
    p = _params(**bad)
    assert _lib.lib.sca_footprint_bytes(C.byref(p)) == 0
    # NULL context: rejected before any HIP call
    assert _lib.lib.sca_potential(None, C.byref(p), None, None) == _lib.SCA_EINVAL
    assert _lib.lib.sca_last_error()


def test_null_context_and_pointers():
    from paper_2311_04435_amd import _lib
    p = _params()
    assert _lib.lib.sca_grad(None, C.byref(p), None, None, None) == _lib.SCA_EINVAL
    assert b"context" in _lib.lib.sca_last_error()
    assert _lib.lib.sca_adam_solve(None, None, None, None, None, None, None) \
        == _lib.SCA_EINVAL


def test_footprint_grows_with_problem():
    from paper_2311_04435_amd import _lib
    f = lambda **kw: _lib.lib.sca_footprint_bytes(C.byref(_params(**kw)))
    a, b, c = f(L=4, n_max=64), f(L=4, n_max=256), f(L=8, n_max=256)
    assert 0 < a < b < c
    # at least the per-matrix outputs: 2M matrices x N complex diagonal
    assert b >= 2 * 256 * 16 * 16
    assert _lib.lib.sca_factor_bytes(C.byref(_params())) >= 2 * 256 * 16 * 16


def test_spectral_route_footprint():
    """SCA_FACTOR_EIGH: scratch of a few N^2 per spin instead of a factor
    per matrix; FP64 only; no factor buffer."""
    from paper_2311_04435_amd import _lib
    f = lambda **kw: _lib.lib.sca_footprint_bytes(C.byref(_params(**kw)))
    lu, eig = f(L=20, n_max=512), f(L=20, n_max=512, factor=2)
    assert 0 < eig < lu / 20
    # eigenvectors, reflectors and psi^2 of both spins at least
    assert eig >= 3 * 2 * 400 * 400 * 8
    assert f(L=20, n_max=512, factor=2, precision=1) == 0
    assert f(L=2, n_max=8, factor=2) > 0
    assert _lib.lib.sca_factor_bytes(C.byref(_params(factor=2))) == 0


def test_create_without_gpu_reports_device_error():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2311_04435_amd import _lib
    h = C.c_void_p()
    st = _lib.lib.sca_create(0, None, 0, C.byref(h))
    assert st in (_lib.SCA_EDEVICE, _lib.SCA_EINVAL)
    assert not h.value
