"""GPU parity of sca_hmc (Hybrid Monte Carlo of exp(-Omega/T)) against the
oracle's chain with the same momenta and uniforms: every accept decision
equal, the field after each trajectory and the Hamiltonians within 1e-10
(relative), on the fused small path (6x6), the blocked path (10x10, pivoted
and symmetric), a disordered lattice and with the Matsubara tail."""
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


CASES = [(6, "lu", False, False), (10, "lu", False, False),
         (10, "ldlt", False, False), (10, "lu", True, False),
         (8, "lu", False, True)]


@pytest.mark.parametrize("L,factor,tail,disorder", CASES)
def test_hmc_chain(sca, L, factor, tail, disorder):
    N = L * L
    n_traj, n_leap, eps = 6, 6, 0.03
    eps_i = synth.uniform(2000 + L, N, -1.0, 1.0) if disorder else None
    p = sca.Params(L=L, U=3.0, T=0.3, n_max=128 if tail else 48, delta=0.4,
                   factor=factor, tail=tail,
                   onsite=cuda(eps_i) if disorder else None)
    pd = dict(L=L, t=1.0, U=3.0, delta=0.4, T=0.3, n_max=p.n_max)
    phi0 = synth.uniform(2100 + L, N, -0.6, 0.6)
    moms = synth.normal(2200 + L, n_traj * N).reshape(n_traj, N)
    us = synth.uniform(2300 + L, n_traj, 0.0, 1.0)
    phi, acc, h0, h1 = sca.hmc(p, cuda(phi0), cuda(moms), us, eps, n_leap)
    # the oracle's chain, trajectory by trajectory
    ref = phi0.copy()
    for t in range(n_traj):
        r_phi, r_acc, r_h0, r_h1 = oracle.hmc_chain(pd, ref, moms[t:t + 1],
                                                    us[t:t + 1], eps, n_leap,
                                                    onsite=eps_i)
        assert acc[t] == r_acc[0], (t, h0[t], h1[t], r_h0, r_h1, us[t])
        assert abs(h0[t] - r_h0[0]) < 1e-10 * abs(r_h0[0])
        assert abs(h1[t] - r_h1[0]) < 1e-10 * abs(r_h1[0])
        ref = r_phi
    e = np.max(np.abs(phi.cpu().numpy() - ref)) / np.max(np.abs(ref))
    print(f"L={L} {factor} tail={tail} disorder={disorder}: accepted "
          f"{acc.sum()}/{n_traj}, dH {np.round(h1 - h0, 4)}, phi err {e:.1e}")
    assert e < 1e-10
    assert 0 < acc.sum()


def test_hmc_rejection_restores_phi(sca):
    """uniforms of 1 - 1e-15 reject every uphill trajectory: phi comes back
    bit for bit."""
    import torch
    L = 6
    p = sca.Params(L=L, U=3.0, T=0.3, n_max=48)
    phi0 = cuda(synth.uniform(2400, L * L, -0.6, 0.6))
    moms = cuda(synth.normal(2401, 3 * L * L).reshape(3, L * L))
    # a large step: energy errors of O(1), uphill
    phi, acc, h0, h1 = sca.hmc(p, phi0, moms, [1.0 - 1e-15] * 3, 0.2, 4)
    assert np.all((h1 - h0 > 0) == (acc == 0))
    if not acc.any():
        assert torch.equal(phi, phi0)
