"""GPU parity of the fused small-matrix path (N <= 64) against the oracle.

Bar (FP64): per-matrix ln|det| and diag(A^-1) within 1e-11 (relative to the
largest entry); Omega~ and the gradient within 1e-10 relative; trajectories
within 1e-10 of phi's scale.  Measured errors are printed.
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


def P(sca, L, U=4.0, delta=0.0, T=0.1, n_max=64, t=1.0):
    return sca.Params(L=L, U=U, T=T, n_max=n_max, t=t, delta=delta)


def pd(p):
    return dict(L=p.L, t=p.t, U=p.U, delta=p.delta, T=p.T, n_max=p.n_max)


def rel_inf(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("L,delta", [(2, 0.9), (4, 0.0), (6, 1.3), (8, 0.5)])
def test_shifted_terms_match_route_d(sca, L, delta):
    import torch
    p = P(sca, L, delta=delta, T=0.1)
    phi = synth.uniform(L, L * L, -0.5, 0.5)
    w = oracle.matsubara(0.1, 300)
    z = np.concatenate([1j * w[[0, 1, 7, 299]], [0.31 + 0.05j, -2.2 + 0.05j, 4.0 + 0.5j]])
    lad, dg = sca.shifted_terms(p, cuda(phi), torch.as_tensor(z).cuda())
    lad, dg = lad.cpu().numpy(), dg.cpu().numpy()
    for si, spin in enumerate((1, -1)):
        rl, rd = oracle.shifted_terms(pd(p), phi, z, spin)
        e1 = np.max(np.abs(lad[si] - rl) / np.maximum(1.0, np.abs(rl)))
        e2 = rel_inf(dg[si], rd)
        print(f"L={L} spin={spin}: logabsdet err {e1:.2e}, diag err {e2:.2e}")
        assert e1 < 1e-11 and e2 < 1e-11


def test_potential_and_gradient_hubbard_4x4(sca):
    wl = synth.WORKLOADS["hubbard_4x4"]
    p = sca.Params.from_dict(wl["params"])
    phi = synth.make_phi0(4, wl["phi0"])
    g, o2 = sca.grad(p, cuda(phi))
    g, o2 = g.cpu().numpy(), o2.cpu().numpy()
    om_t = oracle.omega_tilde(pd(p), phi)
    om = oracle.omega_full(pd(p), phi)
    gr = oracle.grad(pd(p), phi)
    e_om = abs(o2[1] - om_t) / abs(om_t)
    e_full = abs(o2[0] - om) / abs(om)
    e_g = np.max(np.abs(g - gr)) / max(np.max(np.abs(gr)), 2 * np.max(np.abs(phi)) / p.U)
    print(f"Omega~ err {e_om:.2e}  Omega err {e_full:.2e}  grad err {e_g:.2e}")
    assert e_om < 1e-10 and e_full < 1e-10 and e_g < 1e-10
    o3 = sca.potential(p, cuda(phi)).cpu().numpy()
    assert np.array_equal(o3, o2)


def test_adam_trajectory_hubbard_4x4(sca):
    """The 4x4 workload: 500 ADAM steps on the GPU vs the oracle."""
    wl = synth.WORKLOADS["hubbard_4x4"]
    p = sca.Params.from_dict(wl["params"])
    phi0 = synth.make_phi0(4, wl["phi0"])
    steps = wl["steps"]
    phi, m, v, res = sca.adam_solve(p, cuda(phi0), steps)
    ref, info = oracle.adam_solve(pd(p), phi0, steps)
    e = np.max(np.abs(phi.cpu().numpy() - ref)) / np.max(np.abs(ref))
    e_om = abs(res["omega_tilde"] - info["omega_tilde"]) / abs(info["omega_tilde"])
    e_af = abs(res["af_order"] - oracle.af_order(ref, 4)) / oracle.af_order(ref, 4)
    print(f"phi err {e:.2e}  Omega~ err {e_om:.2e}  |phi| err {e_af:.2e}  "
          f"|phi|={res['af_order']:.6f} steps={res['steps_done']}")
    assert res["steps_done"] == steps
    assert e < 1e-10 and e_om < 1e-10 and e_af < 1e-10


def test_adam_resume_is_bitwise(sca):
    import torch
    p = P(sca, 4, U=4.0, n_max=64)
    phi0 = cuda(synth.uniform(3, 16, -0.1, 0.1))
    a, ma, va, _ = sca.adam_solve(p, phi0, 60)
    b = phi0.clone()
    mb, vb = torch.zeros_like(b), torch.zeros_like(b)
    ctx = sca.default_context()
    ctx.adam_solve(p, b, mb, vb, 25)
    ctx.adam_solve(p, b, mb, vb, 35, t0=25)
    assert torch.equal(a, b) and torch.equal(ma, mb) and torch.equal(va, vb)


def test_repeat_is_bitwise(sca):
    import torch
    p = P(sca, 6, delta=0.7, n_max=128)
    phi = cuda(synth.uniform(5, 36, -0.5, 0.5))
    g1, o1 = sca.grad(p, phi)
    g2, o2 = sca.grad(p, phi)
    assert torch.equal(g1, g2) and torch.equal(o1, o2)


def test_dos_matches_oracle(sca):
    import torch
    L = 4
    p = P(sca, L, delta=0.4)
    phi = synth.uniform(9, 16, -0.6, 0.6)
    w = np.linspace(-8.0, 8.0, 1601)
    rho = sca.dos(p, cuda(phi), cuda(w), 0.05).cpu().numpy()
    ref = oracle.dos(pd(p), phi, w, 0.05)
    e = rel_inf(rho, ref)
    print(f"DOS err {e:.2e}")
    assert e < 1e-10


def test_autograd_split_equals_grad(sca):
    import torch
    p = P(sca, 8, U=3.0, delta=0.3, n_max=96)
    phi = cuda(synth.uniform(12, 64, -0.4, 0.4))
    ctx = sca.default_context()
    fac = torch.empty(ctx.factor_bytes(p), dtype=torch.uint8, device="cuda")
    o2 = ctx.factorize(p, phi, fac)
    g = ctx.grad_from_factors(p, phi, fac)
    g_ref, o_ref = sca.grad(p, phi)
    assert torch.equal(o2, o_ref) and torch.equal(g, g_ref)


def test_smallest_cases(sca):
    # 2x2 lattice (double bonds), a single Matsubara frequency
    p = P(sca, 2, U=2.5, delta=0.6, n_max=1, T=0.3)
    phi = synth.uniform(2, 4, -0.5, 0.5)
    g, o2 = sca.grad(p, cuda(phi))
    assert abs(o2[1].item() - oracle.omega_tilde(pd(p), phi)) < 1e-12
    assert np.max(np.abs(g.cpu().numpy() - oracle.grad(pd(p), phi))) < 1e-12


def test_nonfinite_field_is_reported(sca):
    p = P(sca, 4)
    phi = synth.uniform(1, 16, -0.1, 0.1)
    phi[3] = np.nan
    with pytest.raises(sca.SCAError) as ei:
        sca.grad(p, cuda(phi))
    assert ei.value.status == -4
