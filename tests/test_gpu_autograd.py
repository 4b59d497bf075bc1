"""GPU tests of the differentiable potential (SCAPotential): the backward
reuses the forward's LU factors.

* forward and backward equal sca.potential / sca.grad bit for bit;
* the incoming gradients of Omega and Omega~ add, and the node composes
  with other torch terms;
* an in-place change of phi between forward and backward is refused;
* on the 32x32 ionic lattice (16 fields, U = 2, 4, 6) the gradient matches
  central finite differences of the oracle's Omega~ written by
  tests/golden/make_fd_grad.py, in both precisions: |g.d - fd| within
  10 x the quotient's rounding floor plus 1e-7 |fd|.
"""
import json
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "fd_grad_32x32.json")


@pytest.fixture(scope="module")
def sca():
    import torch
    import paper_2311_04435_amd as sca
    assert torch.cuda.is_available()
    return sca


def cuda(x, grad=False):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64).cuda()
    return t.requires_grad_(grad)


@pytest.mark.parametrize("L,precision", [(4, "fp64"), (12, "fp64"),
                                         (20, "fp32r")])
def test_autograd_equals_grad(sca, L, precision):
    import torch
    from paper_2311_04435_amd.autograd import potential
    p = sca.Params(L=L, U=4.0, T=0.1, n_max=64, delta=0.4, precision=precision)
    phi = cuda(synth.uniform(40 + L, L * L, -0.5, 0.5), grad=True)
    o2 = potential(p, phi)
    o2[1].backward()
    g_ref, o_ref = sca.grad(p, phi.detach())
    assert torch.equal(o2.detach(), o_ref)
    assert torch.equal(phi.grad, g_ref)


def test_autograd_composes(sca):
    import torch
    from paper_2311_04435_amd.autograd import potential
    p = sca.Params(L=12, U=3.0, T=0.2, n_max=32)
    phi = cuda(synth.uniform(9, 144, -0.5, 0.5), grad=True)
    o2 = potential(p, phi)
    loss = 3.0 * o2[1] + o2[0] + (phi * phi).sum()
    loss.backward(retain_graph=True)
    g, _ = sca.grad(p, phi.detach())
    want = 4.0 * g + 2.0 * phi.detach()
    diff = (phi.grad - want).abs().max().item()
    print(f"composed gradient: max |diff| {diff:.3e}, max |want| "
          f"{want.abs().max().item():.3e}")
    assert torch.allclose(phi.grad, want, rtol=1e-15, atol=1e-15)
    first = phi.grad.clone()
    phi.grad = None
    loss.backward()
    assert torch.equal(phi.grad, first)


def test_autograd_refuses_inplace_change(sca):
    import torch
    from paper_2311_04435_amd.autograd import potential
    p = sca.Params(L=4, U=4.0, T=0.1, n_max=16)
    leaf = cuda(synth.uniform(3, 16, -0.5, 0.5), grad=True)
    phi = leaf * 1.0
    o2 = potential(p, phi)
    with torch.no_grad():
        phi.add_(0.1)
    with pytest.raises(RuntimeError):
        o2[1].backward()


@pytest.mark.parametrize("precision", ["fp64", "fp32r"])
def test_autograd_vs_finite_differences_32x32(sca, precision):
    from paper_2311_04435_amd.autograd import potential
    with open(GOLDEN) as f:
        gold = json.load(f)
    N = gold["L"] ** 2
    worst = 0.0
    for case in gold["cases"]:
        pr = case["params"]
        p = sca.Params(L=pr["L"], U=pr["U"], T=pr["T"], n_max=pr["n_max"],
                       delta=pr["delta"], t=pr["t"], precision=precision)
        phi = cuda(synth.uniform(case["seed"], N, -0.5, 0.5), grad=True)
        o2 = potential(p, phi)
        o2[1].backward()
        g = phi.grad.cpu().numpy()
        om = o2[1].item()
        assert abs(om - case["omega_tilde"]) <= 1e-11 * abs(case["omega_tilde"])
        for d in case["directions"]:
            if d["kind"] == "coord":
                gd = g[d["arg"]]
            else:
                gd = float(g @ synth.rademacher(d["arg"], N))
            err = abs(gd - d["fd"])
            bound = 10.0 * case["floor"] + 1e-7 * abs(d["fd"])
            worst = max(worst, err / bound)
            assert err <= bound, (case["seed"], d, gd)
    print(f"32x32 {precision}: worst |g.d - fd| / bound = {worst:.2e}")


def test_factor_buffer_state(sca):
    import torch
    from paper_2311_04435_amd import SCAError
    ctx = sca.default_context()
    # FP64 blocked path: the backward inverts the factors in place
    p = sca.Params(L=10, U=4.0, T=0.1, n_max=16)
    phi = cuda(synth.uniform(1, 100, -0.5, 0.5))
    fac = torch.empty(ctx.factor_bytes(p), dtype=torch.uint8, device="cuda")
    ctx.factorize(p, phi, fac)
    g1 = ctx.grad_from_factors(p, phi, fac)
    with pytest.raises(SCAError, match="consumed"):
        ctx.grad_from_factors(p, phi, fac)
    ctx.factorize(p, phi, fac)
    assert torch.equal(ctx.grad_from_factors(p, phi, fac), g1)
    # other params than the factorisation's
    ctx.factorize(p, phi, fac)
    q = sca.Params(L=10, U=4.0, T=0.1, n_max=8)
    with pytest.raises(SCAError, match="do not hold"):
        ctx.grad_from_factors(q, phi, fac)
    # a buffer that never saw sca_factorize
    fresh = torch.zeros_like(fac)
    with pytest.raises(SCAError):
        ctx.grad_from_factors(p, phi, fresh)
    # fused small path: reusable
    p4 = sca.Params(L=4, U=4.0, T=0.1, n_max=16)
    phi4 = cuda(synth.uniform(2, 16, -0.5, 0.5))
    fac4 = torch.empty(ctx.factor_bytes(p4), dtype=torch.uint8, device="cuda")
    ctx.factorize(p4, phi4, fac4)
    assert torch.equal(ctx.grad_from_factors(p4, phi4, fac4),
                       ctx.grad_from_factors(p4, phi4, fac4))
