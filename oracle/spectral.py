"""Route S: the same quantities from the spectrum of H_s (oracle; test
infrastructure).

With H_s = sum_k e_k psi_k psi_k^T (real symmetric, numpy eigh):

  ln|det(i w - H_s)| = 1/2 sum_k ln(w^2 + e_k^2)
  (i w - H_s)^-1_ii  = sum_k psi_k(i)^2 / (i w - e_k)

so, per spin and summed over the M positive frequencies,

  Omega~ contribution   -T sum_k sum_n ln(1 + e_k^2 / w_n^2)
  gradient contribution  s sum_k psi_k(i)^2 * 2T sum_n e_k / (w_n^2 + e_k^2)
  rho_s(w)               (1/N) sum_k (eta/pi) / ((w - e_k)^2 + eta^2)

This costs one eigendecomposition per spin per step instead of M LUs, so the
long ADAM trajectories of the tests run on it.  Pinned against route D and the
Bloch closed forms.
"""
from __future__ import annotations

import numpy as np

from .model import hamiltonian, matsubara


def _eig(L, t, delta, phi, spin, onsite=None):
    return np.linalg.eigh(hamiltonian(L, t, delta, phi, spin, onsite))


def terms_spectral(L, t, U, delta, T, M, phi, onsite=None):
    """(Omega~, grad) from the spectra of both spins."""
    phi = np.asarray(phi, dtype=np.float64)
    w2 = matsubara(T, M) ** 2
    om = float(np.sum(phi * phi)) / U
    g = 2.0 * phi / U
    for spin in (1, -1):
        e, psi = _eig(L, t, delta, phi, spin, onsite)
        e2 = e * e
        # sum over n of ln(1 + e^2/w^2), per eigenvalue
        lnsum = np.log1p(e2[:, None] / w2[None, :]).sum(axis=1)
        om -= T * float(np.sum(lnsum))
        # S_M(e) = 2T sum_n e / (w_n^2 + e^2)
        s_m = 2.0 * T * (e[:, None] / (w2[None, :] + e2[:, None])).sum(axis=1)
        g += spin * (psi * psi) @ s_m
    return om, g


def omega_spectral(L, t, U, delta, T, M, phi, onsite=None) -> float:
    return terms_spectral(L, t, U, delta, T, M, phi, onsite)[0]


def grad_spectral(L, t, U, delta, T, M, phi, onsite=None) -> np.ndarray:
    return terms_spectral(L, t, U, delta, T, M, phi, onsite)[1]


def dos_spectral(L, t, delta, phi, w, eta, onsite=None) -> np.ndarray:
    """[2, n_w] Lorentzian-broadened DOS per spin (up first)."""
    w = np.asarray(w, dtype=np.float64)
    out = np.empty((2, w.size))
    for row, spin in enumerate((1, -1)):
        e, _ = _eig(L, t, delta, phi, spin, onsite)
        out[row] = (eta / np.pi / ((w[:, None] - e[None, :]) ** 2 + eta * eta)
                    ).mean(axis=1)
    return out


def shifted_terms_spectral(L, t, delta, phi, z, spin, onsite=None):
    """(ln|det(z_j I - H_s)|, diag((z_j I - H_s)^-1)) from the spectrum:
    sum_k ln|z - e_k| and sum_k psi_k(i)^2 / (z - e_k)."""
    e, psi = _eig(L, t, delta, phi, spin, onsite)
    z = np.atleast_1d(np.asarray(z, dtype=np.complex128))
    lad = np.log(np.abs(z[:, None] - e[None, :])).sum(axis=1)
    dg = (1.0 / (z[:, None] - e[None, :])) @ (psi * psi).T
    return lad, dg
