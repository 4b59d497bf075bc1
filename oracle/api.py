"""Oracle entry points used by the tests (test infrastructure).

`p` is a parameter dict {L, t, U, delta, T, n_max} (Sec. II: t hopping,
U on-site repulsion, Delta ionic potential, T temperature, n_max Matsubara
cut-off of Eq. (7)); `onsite` an optional extra site potential.
"""
from __future__ import annotations

import numpy as np

from .adam import AdamState, adam_step
from .lu import lu_pivoted, logabsdet_lu, inverse_lu
from .model import hamiltonian, matsubara, stagger_signs
from .spectral import terms_spectral, dos_spectral, shifted_terms_spectral


def _unpack(p):
    return p["L"], p["t"], p["U"], p["delta"], p["T"], p["n_max"]


def omega_tilde(p, phi, onsite=None) -> float:
    L, t, U, delta, T, M = _unpack(p)
    return terms_spectral(L, t, U, delta, T, M, phi, onsite)[0]


def omega_full(p, phi, onsite=None) -> float:
    """Omega = Omega~ - 2 N T sum_n ln w_n^2."""
    L, t, U, delta, T, M = _unpack(p)
    shift = 2.0 * L * L * T * float(np.sum(np.log(matsubara(T, M) ** 2)))
    return omega_tilde(p, phi, onsite) - shift


def grad(p, phi, onsite=None) -> np.ndarray:
    L, t, U, delta, T, M = _unpack(p)
    return terms_spectral(L, t, U, delta, T, M, phi, onsite)[1]


def shifted_terms(p, phi, z, spin, onsite=None):
    """Route D for arbitrary complex shifts z_j: (ln|det(z_j I - H_s)|,
    diag((z_j I - H_s)^-1)) for each j, by the pivoted LU."""
    L, t, U, delta, T, M = _unpack(p)
    H = hamiltonian(L, t, delta, phi, spin, onsite)
    N = H.shape[0]
    z = np.atleast_1d(np.asarray(z, dtype=np.complex128))
    lad = np.empty(z.size)
    dg = np.empty((z.size, N), dtype=np.complex128)
    for j, zj in enumerate(z):
        LU, perm = lu_pivoted(zj * np.eye(N) - H)
        lad[j] = logabsdet_lu(LU)
        dg[j] = np.diag(inverse_lu(LU, perm))
    return lad, dg


def shifted_terms_s(p, phi, z, spin, onsite=None):
    """Route S for arbitrary complex shifts (same outputs as shifted_terms)."""
    L, t, U, delta, T, M = _unpack(p)
    return shifted_terms_spectral(L, t, delta, phi, z, spin, onsite)


def omega_tilde_d(p, phi, onsite=None) -> float:
    """Omega~ by route D: sum over the 2M matrices of ln|det(A/w_n)|."""
    L, t, U, delta, T, M = _unpack(p)
    phi = np.asarray(phi, dtype=np.float64)
    w = matsubara(T, M)
    N = L * L
    tot = float(np.sum(phi * phi)) / U
    for spin in (1, -1):
        lad, _ = shifted_terms(p, phi, 1j * w, spin, onsite)
        tot -= 2.0 * T * float(np.sum(lad - N * np.log(w)))
    return tot


def grad_d(p, phi, onsite=None) -> np.ndarray:
    """Gradient by route D: 2 phi/U - 2T sum_s s sum_n Re diag(A_ns^-1)."""
    L, t, U, delta, T, M = _unpack(p)
    phi = np.asarray(phi, dtype=np.float64)
    w = matsubara(T, M)
    g = 2.0 * phi / U
    for spin in (1, -1):
        _, dg = shifted_terms(p, phi, 1j * w, spin, onsite)
        g -= 2.0 * T * spin * dg.real.sum(axis=0)
    return g


def af_order(phi, L) -> float:
    """|phi| := |N^-1 sum_i (-1)^(x+y) phi_i| (the AF order parameter)."""
    return abs(float(np.mean(stagger_signs(L) * np.asarray(phi))))


def dos(p, phi, w, eta, route: str = "S", onsite=None) -> np.ndarray:
    """rho_s(w) = -(1/(pi N)) Im tr((w + i eta) - H_s)^-1, Eq. (8), mu = 0."""
    L, t, U, delta, T, M = _unpack(p)
    if route == "S":
        return dos_spectral(L, t, delta, phi, w, eta, onsite)
    w = np.asarray(w, dtype=np.float64)
    out = np.empty((2, w.size))
    for row, spin in enumerate((1, -1)):
        _, dg = shifted_terms(p, phi, w + 1j * eta, spin, onsite)
        out[row] = -dg.imag.mean(axis=1) / np.pi
    return out


def adam_solve(p, phi0, steps, lr=0.01, b1=0.9, b2=0.999, eps=1e-8,
               record=(), onsite=None):
    """Minimise Omega~ with ADAM from phi0 for `steps` steps (route S).

    Returns (phi, info) where info holds Omega~ at the final phi, the
    gradient there, and {step: phi} for the steps listed in `record`
    (step k = phi after k updates; 0 = phi0).
    """
    L, t, U, delta, T, M = _unpack(p)
    x = np.array(phi0, dtype=np.float64, copy=True)
    st = AdamState.zeros(x.size)
    rec = {}
    if 0 in record:
        rec[0] = x.copy()
    trace = []
    for k in range(1, steps + 1):
        om, g = terms_spectral(L, t, U, delta, T, M, x, onsite)
        trace.append(om)
        x = adam_step(x, g, st, lr, b1, b2, eps)
        if k in record:
            rec[k] = x.copy()
    om, g = terms_spectral(L, t, U, delta, T, M, x, onsite)
    return x, dict(omega_tilde=om, grad=g, record=rec, trace=np.array(trace),
                   m=st.m, v=st.v)
