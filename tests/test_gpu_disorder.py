"""GPU parity with a random site potential (the disordered Hubbard model the
paper names as its target application): no lattice symmetry left, so every
route is checked on a general real symmetric H.

onsite_i ~ U[-W/2, W/2) with W = 2, seeded; the oracle (route S, pinned to
route D on the CPU with disorder) is the reference; bar 1e-10 (FP64) and
the refined-FP32 tolerance of its own tests.
"""
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


@pytest.mark.parametrize("L,precision,factor,tol", [
    (4, "fp64", "lu", 1e-10), (10, "fp64", "lu", 1e-10),
    (12, "fp64", "ldlt", 1e-10), (16, "fp32r", "lu", 1e-10)])
def test_disordered_grad(sca, L, precision, factor, tol):
    N = L * L
    eps = synth.uniform(700 + L, N, -1.0, 1.0)
    phi = synth.uniform(800 + L, N, -0.5, 0.5)
    p = sca.Params(L=L, U=3.0, T=0.15, n_max=64, delta=0.4,
                   precision=precision, factor=factor, onsite=cuda(eps))
    g, o2 = sca.grad(p, cuda(phi))
    g, o2 = g.cpu().numpy(), o2.cpu().numpy()
    pd = dict(L=L, t=1.0, U=3.0, delta=0.4, T=0.15, n_max=64)
    om = oracle.omega_tilde(pd, phi, onsite=eps)
    gr = oracle.grad(pd, phi, onsite=eps)
    e_om = abs(o2[1] - om) / abs(om)
    e_g = np.max(np.abs(g - gr)) / max(np.max(np.abs(gr)), 2 * np.max(np.abs(phi)) / 3.0)
    print(f"L={L} {precision} {factor} disorder: Omega~ {e_om:.1e} grad {e_g:.1e}")
    assert e_om < tol and e_g < tol


def test_disordered_adam(sca):
    L = 10
    eps = synth.uniform(900, L * L, -1.0, 1.0)
    phi0 = synth.uniform(901, L * L, -0.5, 0.5)
    p = sca.Params(L=L, U=4.0, T=0.1, n_max=64, onsite=cuda(eps))
    phi, m, v, res = sca.adam_solve(p, cuda(phi0), 30)
    pd = dict(L=L, t=1.0, U=4.0, delta=0.0, T=0.1, n_max=64)
    ref, info = oracle.adam_solve(pd, phi0, 30, onsite=eps)
    e = np.max(np.abs(phi.cpu().numpy() - ref)) / np.max(np.abs(ref))
    print(f"disordered 10x10, 30 steps: phi err {e:.1e}")
    assert e < 1e-10
