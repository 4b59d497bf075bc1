"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test names what fixes the expected value: brute force (Leibniz /
adjugate), a library routine (numpy eigvalsh/eigh/det, scipy lu_factor,
torch.optim.Adam), a closed form derived from Bloch's theorem, the textbook
infinite products over odd Matsubara frequencies, finite differences, or an
exact symmetry.  Sizes keep the whole file within a few seconds to a minute
on the CPU.
"""
import numpy as np
import pytest
import scipy.linalg

import oracle
from oracle import closed
from oracle.lu import lu_pivoted, logabsdet_lu, inverse_lu, leibniz_det, adjugate_diag
import synth
from synth import uniform


def P(L, U=4.0, delta=0.0, T=0.1, n_max=64, t=1.0):
    return dict(L=L, t=t, U=U, delta=delta, T=T, n_max=n_max)


# ---------------------------------------------------------------- lattice --

def test_kinetic_matrix_2x2_double_bonds():
    # On L = 2 the +x and -x neighbours coincide: K_ij = 2 (periodic).
    K = oracle.kinetic_matrix(2)
    assert K[0, 1] == 2.0 and K[0, 2] == 2.0 and K[0, 3] == 0.0 and K[0, 0] == 0.0
    assert np.all(K.sum(axis=1) == 4.0)


@pytest.mark.parametrize("L", [2, 4, 6])
def test_kinetic_spectrum_is_bloch(L):
    # -tK has exactly the Bloch energies -2t(cos kx + cos ky).
    ev = np.linalg.eigvalsh(-1.3 * oracle.kinetic_matrix(L))
    ref = np.sort(closed.bloch_energies(L, 1.3))
    assert np.max(np.abs(ev - ref)) < 1e-13


def test_odd_L_rejected():
    with pytest.raises(ValueError):
        oracle.neighbours(3)


def test_spin_traces_cancel():
    L = 4
    phi = uniform(3, L * L, -0.5, 0.5)
    tr = sum(np.trace(oracle.hamiltonian(L, 1.0, 0.8, phi, s)) for s in (1, -1))
    assert abs(tr) < 1e-14


# ------------------------------------------------ route D: the pivoted LU --

def test_leibniz_brute_force_itself():
    # Triangular: det = product of the diagonal; a transposition flips sign;
    # and the library determinant on a random complex matrix.
    rng = np.random.default_rng(1)
    A = np.triu(rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4)))
    assert abs(leibniz_det(A) - np.prod(np.diag(A))) < 1e-12
    B = rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4))
    assert abs(leibniz_det(B[[1, 0, 2, 3]]) + leibniz_det(B)) < 1e-12
    assert abs(leibniz_det(B) - np.linalg.det(B)) < 1e-12 * abs(np.linalg.det(B))
    assert np.max(np.abs(adjugate_diag(B) - np.diag(np.linalg.inv(B)))) < 1e-12


@pytest.mark.parametrize("spin", [1, -1])
@pytest.mark.parametrize("z", [1j * np.pi * 0.1, 1j * 37.0 * np.pi * 0.1, 0.3 + 0.05j])
def test_lu_matches_leibniz_on_2x2_lattice(spin, z):
    L = 2
    phi = uniform(7, 4, -0.6, 0.6)
    p = P(L, delta=0.9)
    A = z * np.eye(4) - oracle.hamiltonian(L, 1.0, 0.9, phi, spin)
    lad, dg = oracle.shifted_terms(p, phi, [z], spin)
    det = leibniz_det(A)
    assert abs(lad[0] - np.log(abs(det))) < 1e-13
    assert np.max(np.abs(dg[0] - adjugate_diag(A))) < 1e-13 * np.max(np.abs(dg[0]))


@pytest.mark.parametrize("N", [16, 36, 64])
def test_lu_matches_scipy(N):
    # The pivoted LU against LAPACK getrf (same pivot rule up to ties).
    rng = np.random.default_rng(N)
    A = rng.normal(size=(N, N)) + 1j * rng.normal(size=(N, N))
    LU, perm = lu_pivoted(A)
    lu2, piv2 = scipy.linalg.lu_factor(A)
    assert np.max(np.abs(np.abs(np.diag(LU)) - np.abs(np.diag(lu2)))) < 1e-10
    L_ = np.tril(LU, -1) + np.eye(N)
    U_ = np.triu(LU)
    assert np.max(np.abs(L_ @ U_ - A[perm])) < 1e-12 * np.max(np.abs(A))
    X = inverse_lu(LU, perm)
    assert np.max(np.abs(X @ A - np.eye(N))) < 1e-11


def test_lu_singular_raises():
    with pytest.raises(ZeroDivisionError):
        lu_pivoted(np.zeros((3, 3), dtype=complex))


# ------------------------------------------------ route D == route S --------

@pytest.mark.parametrize("L,delta", [(4, 0.0), (4, 1.0), (6, 0.5)])
def test_eigenvalue_identity(L, delta):
    # ln|det(iw - H)| = 1/2 sum_k ln(w^2 + e_k^2) with e_k from the library.
    phi = uniform(11, L * L, -0.5, 0.5)
    p = P(L, delta=delta)
    for spin in (1, -1):
        e = np.linalg.eigvalsh(oracle.hamiltonian(L, 1.0, delta, phi, spin))
        w = oracle.matsubara(0.1, 8)
        lad, _ = oracle.shifted_terms(p, phi, 1j * w, spin)
        ref = 0.5 * np.log(w[:, None] ** 2 + e[None, :] ** 2).sum(axis=1)
        assert np.max(np.abs(lad - ref)) < 1e-12


@pytest.mark.parametrize("L", [4, 6])
def test_shifted_terms_route_s_equals_route_d(L):
    phi = uniform(13, L * L, -0.5, 0.5)
    p = P(L, delta=0.7)
    z = np.array([0.3j, 2.9j, 0.4 + 0.05j, -3.0 + 0.2j])
    for spin in (1, -1):
        a, da = oracle.shifted_terms(p, phi, z, spin)
        b, db = oracle.shifted_terms_s(p, phi, z, spin)
        assert np.max(np.abs(a - b)) < 1e-12
        assert np.max(np.abs(da - db)) < 1e-12 * np.max(np.abs(da))


@pytest.mark.parametrize("L,delta,U", [(4, 0.0, 4.0), (4, 1.2, 6.0), (6, 0.4, 3.0)])
def test_route_d_equals_route_s(L, delta, U):
    phi = uniform(5, L * L, -0.5, 0.5)
    p = P(L, U=U, delta=delta, n_max=32)
    a, b = oracle.omega_tilde(p, phi), oracle.omega_tilde_d(p, phi)
    assert abs(a - b) < 1e-13 * abs(a)
    g1, g2 = oracle.grad(p, phi), oracle.grad_d(p, phi)
    assert np.max(np.abs(g1 - g2)) < 1e-13 * np.max(np.abs(g1))


# ------------------------------------------------ Bloch closed form ---------

@pytest.mark.parametrize("L,m,delta", [(4, 0.7, 0.6), (6, 0.3, 1.4), (8, 1.1, 0.0)])
def test_staggered_closed_form(L, m, delta):
    s = oracle.stagger_signs(L)
    p = P(L, U=3.5, delta=delta, T=0.13, n_max=48)
    phi = m * s
    om = oracle.omega_tilde(p, phi)
    ref = closed.omega_tilde_staggered(m, L, 1.0, 3.5, delta, 0.13, 48)
    assert abs(om - ref) < 1e-12 * abs(ref)
    ref_full = closed.omega_staggered(m, L, 1.0, 3.5, delta, 0.13, 48)
    assert abs(oracle.omega_full(p, phi) - ref_full) < 1e-12 * abs(ref_full)
    g = oracle.grad(p, phi)
    gref = s * closed.domega_dm_staggered(m, L, 1.0, 3.5, delta, 0.13, 48) / (L * L)
    assert np.max(np.abs(g - gref)) < 1e-12 * max(1.0, np.max(np.abs(gref)))


def test_staggered_closed_form_route_d():
    L, m, delta = 4, 0.45, 0.7
    s = oracle.stagger_signs(L)
    p = P(L, U=5.0, delta=delta, T=0.2, n_max=16)
    ref = closed.omega_tilde_staggered(m, L, 1.0, 5.0, delta, 0.2, 16)
    assert abs(oracle.omega_tilde_d(p, m * s) - ref) < 1e-12 * abs(ref)


def test_per_spin_dos_closed_form_fixes_spin_sign():
    # Spin s sees h_s = Delta/2 - s m: its gap is 2|h_s|.  This fixes the
    # sign of the field coupling, which the total potential cannot see.
    L, m, delta, eta = 6, 0.5, 0.6, 0.05
    s = oracle.stagger_signs(L)
    p = P(L, delta=delta)
    w = np.linspace(-6, 6, 241)
    rho = oracle.dos(p, m * s, w, eta, route="S")
    ref = closed.dos_staggered(w, eta, m, L, 1.0, delta)
    assert np.max(np.abs(rho - ref)) < 1e-12
    # up: h = 0.3 - 0.5 = -0.2 (small gap); down: h = 0.8 (large gap)
    i0 = np.argmin(np.abs(w))
    assert rho[0, i0] > 10 * rho[1, i0]


def test_dos_route_d_equals_route_s():
    L, eta = 4, 0.1
    phi = uniform(2, 16, -0.5, 0.5)
    p = P(L, delta=0.3)
    w = np.linspace(-5, 5, 41)
    a = oracle.dos(p, phi, w, eta, route="S")
    b = oracle.dos(p, phi, w, eta, route="D")
    assert np.max(np.abs(a - b)) < 1e-13


def test_dos_normalised():
    # Each spin's DOS integrates to 1 minus the Lorentzian tails off the grid.
    L, eta = 4, 0.05
    phi = uniform(4, 16, -0.5, 0.5)
    w = np.linspace(-8, 8, 1601)
    rho = oracle.dos(P(L), phi, w, eta)
    integ = np.trapezoid(rho, w, axis=1)
    e = [np.linalg.eigvalsh(oracle.hamiltonian(L, 1.0, 0.0, phi, s)) for s in (1, -1)]
    tails = [np.mean((np.arctan((8 - ek) / eta) - np.arctan((-8 - ek) / eta)) / np.pi)
             for ek in e]
    assert np.max(np.abs(integ - np.array(tails))) < 1e-5


# ------------------------------------------------ derivatives ---------------

@pytest.mark.parametrize("route", ["S", "D"])
def test_gradient_central_differences(route):
    L = 4
    phi = uniform(21, 16, -0.5, 0.5)
    p = P(L, U=4.0, delta=1.0, n_max=32 if route == "D" else 256)
    f = oracle.omega_tilde if route == "S" else oracle.omega_tilde_d
    g = oracle.grad(p, phi) if route == "S" else oracle.grad_d(p, phi)
    h = 1e-6
    # FD error model: h^2 |f'''| + eps64 |f| / h  ~  1e-12 + 1e-9
    tol = 1e-7
    for i in (0, 5, 11):
        e = np.zeros(16)
        e[i] = h
        fd = (f(p, phi + e) - f(p, phi - e)) / (2 * h)
        assert abs(fd - g[i]) < tol
    d = uniform(99, 16, -1.0, 1.0)
    d /= np.linalg.norm(d)
    fd = (f(p, phi + h * d) - f(p, phi - h * d)) / (2 * h)
    assert abs(fd - g @ d) < tol


def test_phi_zero_is_stationary():
    for delta in (0.0, 0.7, 2.0):
        # the two spins see the same H at phi = 0 and cancel (to round-off:
        # LAPACK may return different bases of the degenerate subspaces)
        g = oracle.grad(P(4, delta=delta), np.zeros(16))
        assert np.max(np.abs(g)) < 1e-14


# ------------------------------------------------ infinite-M limits ----------

def test_large_M_limit_is_ln_cosh():
    # prod_{n>=0}(1 + E^2/w_n^2) = cosh(E/2T): Omega~_M converges to the
    # ln cosh form from above, with an error ~ 1/M.
    L, T, U = 4, 0.2, 3.0
    phi = uniform(8, 16, -0.6, 0.6)
    e = [np.linalg.eigvalsh(oracle.hamiltonian(L, 1.0, 0.4, phi, s)) for s in (1, -1)]
    lim = closed.omega_tilde_limit(e, phi, U, T)
    errs = []
    for M in (512, 1024, 2048):
        errs.append(oracle.omega_tilde(P(L, U=U, delta=0.4, T=T, n_max=M), phi) - lim)
    assert errs[0] > errs[1] > errs[2] > 0
    assert abs(errs[0] / errs[1] - 2.0) < 0.01 and abs(errs[1] / errs[2] - 2.0) < 0.01


def test_truncated_neel_converges_to_hartree_fock():
    # 2T sum_{n>=0} 1/(w_n^2 + E^2) = tanh(E/2T)/(2E): the stationary staggered
    # amplitude at cut-off M approaches the Fermi-function Hartree-Fock
    # amplitude with an error ~ 1/M.
    mhf = closed.hf_neel_m(4, 1.0, 4.0, 0.0, 0.1)
    d = [closed.neel_m(4, 1.0, 4.0, 0.0, 0.1, M) - mhf for M in (256, 512, 1024)]
    assert d[0] < d[1] < d[2] < 0
    assert abs(d[0] / d[1] - 2.0) < 0.02 and abs(d[1] / d[2] - 2.0) < 0.02


def test_route_s_at_neel_root_is_stationary():
    L, U, T, M = 4, 4.0, 0.1, 256
    m = closed.neel_m(L, 1.0, U, 0.0, T, M)
    g = oracle.grad(P(L, U=U, T=T, n_max=M), m * oracle.stagger_signs(L))
    assert np.max(np.abs(g)) < 1e-12


# ------------------------------------------------ symmetries ----------------

def test_spin_flip_and_translation_symmetry():
    L = 6
    phi = uniform(31, 36, -0.5, 0.5)
    p0 = P(L, delta=0.0, n_max=32)
    p1 = P(L, delta=0.8, n_max=32)
    for p in (p0, p1):
        a = oracle.omega_tilde(p, phi)
        assert abs(oracle.omega_tilde(p, -phi) - a) < 1e-12 * abs(a)
    img = phi.reshape(L, L)        # [y, x]
    for p in (p0, p1):
        a = oracle.omega_tilde(p, phi)
        for shift in ((1, 0), (0, 1), (1, 1), (2, 3)):
            b = oracle.omega_tilde(p, np.roll(img, shift, axis=(0, 1)).ravel())
            assert abs(a - b) < 1e-12 * abs(a)


def test_odd_translation_mirrors_per_spin_dos():
    # A one-site shift swaps the sublattices (Delta -> -Delta); the bipartite
    # gauge S K S = -K then maps spec H_s(T phi) onto -spec H_-s(phi).  The
    # potential is even in every eigenvalue and symmetric in s, so it is
    # translation invariant, while the per-spin DOS mirrors:
    # rho_s(w; T phi) = rho_-s(-w; phi).
    L, eta = 6, 0.07
    phi = uniform(32, 36, -0.5, 0.5)
    p = P(L, delta=0.8)
    w = np.linspace(-5, 5, 101)
    shifted = np.roll(phi.reshape(L, L), (0, 1), axis=(0, 1)).ravel()
    a = oracle.dos(p, shifted, w, eta)
    b = oracle.dos(p, phi, -w, eta)[::-1]
    assert np.max(np.abs(a - b)) < 1e-12
    assert np.max(np.abs(a - oracle.dos(p, phi, w, eta))) > 1e-3


def test_half_filling_spectra_mirror_at_zero_delta():
    phi = uniform(6, 16, -0.5, 0.5)
    up = np.linalg.eigvalsh(oracle.hamiltonian(4, 1.0, 0.0, phi, 1))
    dn = np.linalg.eigvalsh(oracle.hamiltonian(4, 1.0, 0.0, phi, -1))
    assert np.max(np.abs(np.sort(up) + np.sort(dn)[::-1])) < 1e-13


# ------------------------------------------------ ADAM ----------------------

def test_adam_matches_torch():
    torch = pytest.importorskip("torch")
    p = P(4, U=4.0, n_max=256)
    phi0 = uniform(0, 16, -0.1, 0.1)
    x = phi0.copy()
    st = oracle.AdamState.zeros(16)
    tx = torch.tensor(phi0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([tx], lr=0.01, betas=(0.9, 0.999), eps=1e-8)
    for _ in range(60):
        g = oracle.grad(p, x)
        x = oracle.adam_step(x, g, st, 0.01)
        opt.zero_grad()
        tx.grad = torch.tensor(oracle.grad(p, tx.detach().numpy()), dtype=torch.float64)
        opt.step()
    assert np.max(np.abs(x - tx.detach().numpy())) < 1e-13


def test_adam_small_U_goes_paramagnetic():
    # U below the instability of phi = 0 (U_c ~ 0.93 on 4x4, T = 0.1).
    phi, info = oracle.adam_solve(P(4, U=0.5, n_max=256), uniform(0, 16, -0.1, 0.1), 500)
    assert np.max(np.abs(phi)) < 1e-4


def test_adam_reaches_neel_state():
    L, U, T, M = 4, 4.0, 0.1, 256
    s = oracle.stagger_signs(L)
    phi0 = 1.0 * s + uniform(0, 16, -0.05, 0.05)
    phi, info = oracle.adam_solve(P(L, U=U, T=T, n_max=M), phi0, 1500)
    m = closed.neel_m(L, 1.0, U, 0.0, T, M)
    assert abs(oracle.af_order(phi, L) - m) < 1e-6
    assert np.max(np.abs(phi - m * s)) < 1e-5


def test_oracle_grad_matches_stored_finite_differences():
    """The oracle's gradient (route S) against the central differences of its
    own Omega~ stored by tests/golden/make_fd_grad.py (32x32 ionic lattice,
    16 fields, 4 Rademacher + 8 coordinate directions each)."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "fd_grad_32x32.json")
    with open(path) as f:
        gold = json.load(f)
    N = gold["L"] ** 2
    for case in gold["cases"][::4]:
        phi = synth.uniform(case["seed"], N, -0.5, 0.5)
        g = oracle.grad(case["params"], phi)
        for d in case["directions"]:
            if d["kind"] == "coord":
                gd = g[d["arg"]]
            else:
                gd = float(g @ synth.rademacher(d["arg"], N))
            assert abs(gd - d["fd"]) <= 10 * case["floor"] + 1e-7 * abs(d["fd"])


def test_oracle_onsite_uniform_is_a_shift():
    """A uniform extra site potential c is the shift z -> z - c of every
    matrix: ln|det(z - H - c)| = ln|det((z - c) - H)| (the disordered model
    of the conclusions with zero disorder)."""
    p = dict(L=4, t=1.0, U=4.0, delta=0.6, T=0.1, n_max=8)
    phi = uniform(61, 16, -0.5, 0.5)
    c = 0.37
    z = np.array([0.3j, 1.1 + 0.2j, -0.4 + 0.05j])
    for spin in (1, -1):
        l1, d1 = oracle.shifted_terms(p, phi, z, spin, onsite=np.full(16, c))
        l2, d2 = oracle.shifted_terms(p, phi, z - c, spin)
        assert np.allclose(l1, l2, rtol=1e-14, atol=1e-14)
        assert np.allclose(d1, d2, rtol=1e-13, atol=1e-14)


def test_oracle_disordered_routes_agree():
    """Random site disorder breaks every lattice symmetry; route D (pivoted
    LU per matrix) and route S (spectrum) must still give the same Omega~
    and gradient."""
    p = dict(L=4, t=1.0, U=3.0, delta=0.0, T=0.2, n_max=32)
    phi = uniform(62, 16, -0.5, 0.5)
    eps = uniform(63, 16, -1.0, 1.0)
    om_s = oracle.omega_tilde(p, phi, onsite=eps)
    om_d = oracle.omega_tilde_d(p, phi, onsite=eps)
    g_s = oracle.grad(p, phi, onsite=eps)
    g_d = oracle.grad_d(p, phi, onsite=eps)
    assert abs(om_s - om_d) <= 1e-13 * abs(om_s)
    assert np.max(np.abs(g_s - g_d)) <= 1e-13 * np.max(np.abs(g_s))


# ---- Hybrid Monte Carlo of exp(-Omega/T) (oracle.hmc) ------------------------

def _hmc_case():
    p = dict(L=4, t=1.0, U=3.0, delta=0.4, T=0.3, n_max=64)
    phi = synth.uniform(31, 16, -0.6, 0.6)
    mom = synth.normal(32, 16)
    return p, phi, mom


def test_hmc_leapfrog_reversible():
    """Integrating forward, negating the momentum and integrating again
    returns to the start (a sign or half-step slip breaks this)."""
    p, phi, mom = _hmc_case()
    phi1, mom1 = oracle.leapfrog(p, phi, mom, 0.02, 12)
    phi2, mom2 = oracle.leapfrog(p, phi1, -mom1, 0.02, 12)
    assert np.max(np.abs(phi2 - phi)) < 1e-12
    assert np.max(np.abs(-mom2 - mom)) < 1e-11


def test_hmc_energy_error_second_order():
    """|H_end - H_start| falls as eps^2 at fixed trajectory length."""
    p, phi, mom = _hmc_case()
    h0 = oracle.hmc_hamiltonian(p, phi, mom)
    dh = []
    for eps, n in ((0.02, 10), (0.01, 20), (0.005, 40)):
        phi1, mom1 = oracle.leapfrog(p, phi, mom, eps, n)
        dh.append(abs(oracle.hmc_hamiltonian(p, phi1, mom1) - h0))
    r1, r2 = dh[0] / dh[1], dh[1] / dh[2]
    print("dH:", dh, "ratios", r1, r2)
    assert 3.0 < r1 < 5.0 and 3.0 < r2 < 5.0
    # the trajectory moves phi by much more than its energy error
    phi1, _ = oracle.leapfrog(p, phi, mom, 0.02, 10)
    assert np.max(np.abs(phi1 - phi)) > 1e-2


def test_hmc_acceptance_rule():
    p, phi, mom = _hmc_case()
    moms = np.stack([mom, synth.normal(33, 16)])
    # u = 1 - tiny accepts only downhill moves; u = 0 accepts everything
    _, acc0, h0, h1 = oracle.hmc_chain(p, phi, moms, [0.0, 0.0], 0.05, 6)
    assert list(acc0) == [1, 1]
    _, acc1, h0, h1 = oracle.hmc_chain(p, phi, moms, [1.0 - 1e-15] * 2, 0.05, 6)
    assert list(acc1) == [int(h1[0] <= h0[0]), int(h1[1] <= h0[1])]
