"""GPU parity of the blocked FP64 path (64 < N <= 1024) against the oracle.

References: route D (the oracle's own pivoted LU) for the smallest lattice,
route S (spectrum of H_s, pinned to route D on the CPU) above it, because
route D at N = 1024 takes minutes per matrix in NumPy.

Bar (FP64): per-matrix ln|det| and diag(A^-1) within 1e-11; Omega~ and the
gradient within 1e-10 relative; trajectories within 1e-10 of phi's scale.
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


def pd(p):
    return dict(L=p.L, t=p.t, U=p.U, delta=p.delta, T=p.T, n_max=p.n_max)


def rel_inf(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


# L = 10, 12, 16 use the 4-wave instance (N padded to 128/160/256), 18, 20
# the 8-wave one (352, 416), 24 and 32 the 16-wide one (576, 1024).
@pytest.mark.parametrize("L", [10, 12, 16, 18, 20, 22, 24, 32])
def test_blocked_shifted_terms(sca, L):
    import torch
    p = sca.Params(L=L, U=4.0, T=0.1, n_max=512, delta=0.8)
    phi = synth.uniform(100 + L, L * L, -0.5, 0.5)
    w = oracle.matsubara(0.1, 512)
    z = np.concatenate([1j * w[[0, 1, 511]], [0.3 + 0.05j, -2.5 + 0.02j]])
    lad, dg = sca.shifted_terms(p, cuda(phi), torch.as_tensor(z).cuda())
    lad, dg = lad.cpu().numpy(), dg.cpu().numpy()
    for si, spin in enumerate((1, -1)):
        if L <= 10:
            rl, rd = oracle.shifted_terms(pd(p), phi, z, spin)
        else:
            rl, rd = oracle.shifted_terms_s(pd(p), phi, z, spin)
        e1 = np.max(np.abs(lad[si] - rl) / np.maximum(1.0, np.abs(rl)))
        e2 = rel_inf(dg[si], rd)
        print(f"L={L} spin={spin}: logabsdet err {e1:.2e}, diag err {e2:.2e}")
        assert e1 < 1e-11 and e2 < 1e-11


@pytest.mark.parametrize("name", ["hubbard_20x20_T0.1", "hubbard_20x20_T0.6"])
def test_blocked_grad_20x20(sca, name):
    wl = synth.WORKLOADS[name]
    p = sca.Params.from_dict(wl["params"])
    phi = synth.make_phi0(20, wl["phi0"])
    g, o2 = sca.grad(p, cuda(phi))
    g, o2 = g.cpu().numpy(), o2.cpu().numpy()
    om_t = oracle.omega_tilde(pd(p), phi)
    gr = oracle.grad(pd(p), phi)
    e_om = abs(o2[1] - om_t) / abs(om_t)
    e_g = np.max(np.abs(g - gr)) / max(np.max(np.abs(gr)), 2 * np.max(np.abs(phi)) / p.U)
    print(f"{name}: Omega~ err {e_om:.2e}  grad err {e_g:.2e}")
    assert e_om < 1e-10 and e_g < 1e-10


def test_blocked_trajectory_20x20_first_steps(sca):
    wl = synth.WORKLOADS["hubbard_20x20_T0.1"]
    p = sca.Params.from_dict(wl["params"])
    phi0 = synth.make_phi0(20, wl["phi0"])
    steps = 50
    phi, m, v, res = sca.adam_solve(p, cuda(phi0), steps)
    ref, info = oracle.adam_solve(pd(p), phi0, steps)
    e = np.max(np.abs(phi.cpu().numpy() - ref)) / np.max(np.abs(ref))
    e_om = abs(res["omega_tilde"] - info["omega_tilde"]) / abs(info["omega_tilde"])
    print(f"20x20 {steps} steps: phi err {e:.2e}  Omega~ err {e_om:.2e}")
    assert e < 1e-10 and e_om < 1e-10


def test_blocked_grad_ionic_32x32(sca):
    wl = synth.WORKLOADS["ionic_32x32_U4"]
    p = sca.Params.from_dict(wl["params"], precision="fp64")
    phi = synth.make_phi0(32, wl["phi0"])
    g, o2 = sca.grad(p, cuda(phi))
    g, o2 = g.cpu().numpy(), o2.cpu().numpy()
    om_t = oracle.omega_tilde(pd(p), phi)
    gr = oracle.grad(pd(p), phi)
    e_om = abs(o2[1] - om_t) / abs(om_t)
    e_g = np.max(np.abs(g - gr)) / max(np.max(np.abs(gr)), 2 * np.max(np.abs(phi)) / p.U)
    print(f"32x32 ionic: Omega~ err {e_om:.2e}  grad err {e_g:.2e}")
    assert e_om < 1e-10 and e_g < 1e-10


def test_blocked_autograd_split_and_repeat(sca):
    import torch
    p = sca.Params(L=12, U=3.0, T=0.15, n_max=64, delta=0.3)
    phi = cuda(synth.uniform(12, 144, -0.4, 0.4))
    ctx = sca.default_context()
    fac = torch.empty(ctx.factor_bytes(p), dtype=torch.uint8, device="cuda")
    o2 = ctx.factorize(p, phi, fac)
    g = ctx.grad_from_factors(p, phi, fac)
    g_ref, o_ref = sca.grad(p, phi)
    g_2, o_2 = sca.grad(p, phi)
    assert torch.equal(o2, o_ref) and torch.equal(g, g_ref)
    assert torch.equal(g_2, g_ref) and torch.equal(o_2, o_ref)


def test_blocked_dos(sca):
    L = 10
    p = sca.Params(L=L, U=4.0, T=0.1, n_max=16, delta=0.5)
    phi = synth.uniform(77, 100, -0.6, 0.6)
    w = np.linspace(-6.0, 6.0, 121)
    rho = sca.dos(p, cuda(phi), cuda(w), 0.05).cpu().numpy()
    ref = oracle.dos(pd(p), phi, w, 0.05)
    e = rel_inf(rho, ref)
    print(f"DOS 10x10 err {e:.2e}")
    assert e < 1e-10


@pytest.mark.parametrize("name", ["hubbard_20x20_T0.1", "hubbard_20x20_T0.6"])
def test_lu_c2_trajectory_2000_steps(sca, name):
    """The headline route (pivoted LU, FP64) over the 20x20 runs of 2000
    ADAM steps against the oracle's trajectory stored by
    tests/golden/make_c2_trajectory.py: phi after 200 and 2000 steps, |phi|,
    Omega~ and the DOS of the final phi."""
    import json
    import os
    import torch
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "c2_trajectory_20x20.json")
    with open(path) as f:
        gold = json.load(f)[name]
    wl = synth.WORKLOADS[name]
    p = sca.Params.from_dict(wl["params"])
    phi0 = cuda(synth.make_phi0(20, wl["phi0"]))
    ctx = sca.default_context()
    phi = phi0.clone()
    m, v = torch.zeros_like(phi), torch.zeros_like(phi)
    ctx.adam_solve(p, phi, m, v, 200, final_eval=False)
    ref200 = np.array(gold["phi200"])
    e200 = np.max(np.abs(phi.cpu().numpy() - ref200)) / np.max(np.abs(ref200))
    res = ctx.adam_solve(p, phi, m, v, 1800, t0=200)
    ref = np.array(gold["phi2000"])
    e = np.max(np.abs(phi.cpu().numpy() - ref)) / np.max(np.abs(ref))
    e_af = abs(res["af_order"] - gold["af_order"]) / max(gold["af_order"], 1e-12)
    e_om = abs(res["omega_tilde"] - gold["omega_tilde"]) / abs(gold["omega_tilde"])
    rho = sca.dos(p, phi, cuda(gold["dos_w"]), gold["dos_eta"]).cpu().numpy()
    e_dos = rel_inf(rho, np.array(gold["dos"]))
    print(f"{name} LU 2000 steps: phi@200 {e200:.2e}  phi@2000 {e:.2e}  "
          f"|phi| {res['af_order']:.6f} ({e_af:.1e})  Omega~ {e_om:.1e}  "
          f"DOS {e_dos:.1e}")
    assert e200 < 1e-10 and e < 1e-10 and e_af < 1e-10
    assert e_om < 1e-10 and e_dos < 1e-10
