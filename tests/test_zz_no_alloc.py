"""GPU test of sca_grad_noalloc (the allocation-free variant of sca_grad for
callers that cannot allocate): through the C ABI, two calls in a row on one
context -- the second with a smaller problem -- and further routes, each
checked against sca_grad on the same inputs (the same kernels on the same
values: bit for bit) and the first against the FP64 oracle to 1e-10; a
problem beyond the fixed scratch is refused with SCA_ENOMEM and writes
nothing."""
import ctypes as C

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sca():
    import torch
    import paper_2311_04435_amd as sca
    assert torch.cuda.is_available()
    return sca


def cuda(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64).cuda()


def noalloc(sca, ctx, p, phi):
    """(status, grad, omega2) of sca_grad_noalloc, outputs prefilled with a
    sentinel."""
    import torch
    from paper_2311_04435_amd import _lib
    g = torch.full((p.N,), 7.25, dtype=torch.float64, device="cuda")
    o2 = torch.full((2,), 7.25, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    st = _lib.lib.sca_grad_noalloc(ctx._h, C.byref(p.c()), phi.data_ptr(),
                                   g.data_ptr(), o2.data_ptr())
    torch.cuda.synchronize()
    return st, g, o2


def test_noalloc_two_calls_then_smaller(sca):
    import torch
    from paper_2311_04435_amd import _lib
    ctx = sca.Context()
    cases = [
        (sca.Params(L=8, U=4.0, T=0.1, n_max=512, delta=0.5), 3100),
        (sca.Params(L=4, U=3.0, T=0.2, n_max=64), 3101),   # smaller
        (sca.Params(L=10, U=4.0, T=0.1, n_max=16, delta=0.4), 3102),
        (sca.Params(L=10, U=4.0, T=0.1, n_max=16, precision="fp32r"), 3103),
        (sca.Params(L=12, U=4.0, T=0.1, n_max=256, factor="eigh"), 3104),
        (sca.Params(L=8, U=4.0, T=0.1, n_max=512, tail=True), 3105),
        (sca.Params(L=4, U=4.0, T=0.1, n_max=32), 3106),
    ]
    for k, (p, seed) in enumerate(cases):
        phi = cuda(synth.uniform(seed, p.N, -0.5, 0.5))
        st, g, o2 = noalloc(sca, ctx, p, phi)
        assert st == _lib.SCA_OK, _lib.lib.sca_last_error()
        g_ref, o_ref = ctx.grad(p, phi)
        assert torch.equal(g, g_ref), k
        assert torch.equal(o2, o_ref), k
        if k == 0:
            pd = dict(L=p.L, t=p.t, U=p.U, delta=p.delta, T=p.T,
                      n_max=p.n_max)
            gr = oracle.grad(pd, phi.cpu().numpy())
            e = float(np.max(np.abs(g.cpu().numpy() - gr)) /
                      max(np.max(np.abs(gr)), 1e-300))
            assert e < 1e-10, e


def test_noalloc_refuses_beyond_scratch(sca):
    import torch
    from paper_2311_04435_amd import _lib
    ctx = sca.Context()
    p = sca.Params(L=20, U=6.0, T=0.1, n_max=512)
    phi = cuda(synth.uniform(3200, p.N, -0.5, 0.5))
    st, g, o2 = noalloc(sca, ctx, p, phi)
    assert st == _lib.SCA_ENOMEM
    assert b"scratch" in _lib.lib.sca_last_error()
    assert bool((g == 7.25).all()) and bool((o2 == 7.25).all())
    # the context and the scratch still work afterwards
    q = sca.Params(L=4, U=4.0, T=0.1, n_max=16)
    x = cuda(synth.uniform(3201, q.N, -0.5, 0.5))
    st, g, o2 = noalloc(sca, ctx, q, x)
    assert st == _lib.SCA_OK
    g_ref, o_ref = ctx.grad(q, x)
    assert torch.equal(g, g_ref) and torch.equal(o2, o_ref)
