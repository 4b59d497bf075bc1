"""Closed forms that pin the oracle (oracle; test infrastructure).

Staggered field phi_i = m (-1)^(x+y).  Then H_s = -t K + h_s S with
h_s = Delta/2 - s m.  -t K is diagonal in Bloch waves with
e_k = -2t (cos kx + cos ky), k in (2 pi / L) Z_L^2, and S couples k with
k + (pi, pi), where e flips sign, so the spectrum of H_s is
+-sqrt(e_k^2 + h_s^2).  Summed over the whole Brillouin zone (each pair
counted from both of its momenta):

  Omega(m)   = N m^2/U - T sum_s sum_k sum_n ln(w_n^2 + e_k^2 + h_s^2)
  Omega~(m)  = N m^2/U - T sum_s sum_k sum_n ln(1 + (e_k^2 + h_s^2)/w_n^2)
  dOmega/dm  = 2 N m/U + 2T sum_s s h_s sum_k sum_n 1/(w_n^2 + e_k^2 + h_s^2)
  rho_s(w)   = (1/N) sum_k 1/2 [lor(w - E_ks) + lor(w + E_ks)],  E = sqrt(e^2+h^2)

and the gradient is staggered: dOmega/dphi_i = (-1)^(x+y) (dOmega/dm) / N.

Infinite-M limits (textbook products / sums over odd Matsubara frequencies):
  prod_{n>=0} (1 + E^2/w_n^2) = cosh(E/(2T))
  2T sum_{n>=0} 1/(w_n^2 + E^2) = tanh(E/(2T)) / (2E)
so Omega~ -> sum phi^2/U - T sum_s sum_k ln cosh(e_ks/(2T)), the Hartree-Fock
grand potential of the spin channel, and stationarity becomes the
Hartree-Fock equation m = (U/2) <n_A,up - n_A,down> with Fermi occupations.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import brentq


def bloch_energies(L: int, t: float) -> np.ndarray:
    k = 2.0 * np.pi * np.arange(L) / L
    return (-2.0 * t * (np.cos(k)[:, None] + np.cos(k)[None, :])).ravel()


def _w(T, M):
    return (2.0 * np.arange(M) + 1.0) * np.pi * T


def omega_tilde_staggered(m, L, t, U, delta, T, M) -> float:
    e2 = bloch_energies(L, t) ** 2
    w2 = _w(T, M) ** 2
    tot = L * L * m * m / U
    for s in (1, -1):
        h = 0.5 * delta - s * m
        tot -= T * np.log1p((e2[:, None] + h * h) / w2[None, :]).sum()
    return float(tot)


def omega_staggered(m, L, t, U, delta, T, M) -> float:
    e2 = bloch_energies(L, t) ** 2
    w2 = _w(T, M) ** 2
    tot = L * L * m * m / U
    for s in (1, -1):
        h = 0.5 * delta - s * m
        tot -= T * np.log(w2[None, :] + e2[:, None] + h * h).sum()
    return float(tot)


def domega_dm_staggered(m, L, t, U, delta, T, M) -> float:
    e2 = bloch_energies(L, t) ** 2
    w2 = _w(T, M) ** 2
    tot = 2.0 * L * L * m / U
    for s in (1, -1):
        h = 0.5 * delta - s * m
        tot += 2.0 * T * s * h * (1.0 / (w2[None, :] + e2[:, None] + h * h)).sum()
    return float(tot)


def neel_m(L, t, U, delta, T, M, hi: float = 20.0) -> float:
    """Positive root of dOmega/dm (the staggered stationary amplitude)."""
    f = lambda m: domega_dm_staggered(m, L, t, U, delta, T, M)
    lo = 1e-9
    if f(lo) >= 0.0:
        return 0.0
    return brentq(f, lo, hi, xtol=1e-15, rtol=1e-15, maxiter=500)


def dos_staggered(w, eta, m, L, t, delta) -> np.ndarray:
    """[2, n_w]; spin up first (s = +1)."""
    e2 = bloch_energies(L, t) ** 2
    w = np.asarray(w, dtype=np.float64)
    out = np.empty((2, w.size))
    lor = lambda x: eta / np.pi / (x * x + eta * eta)
    for row, s in enumerate((1, -1)):
        h = 0.5 * delta - s * m
        E = np.sqrt(e2 + h * h)
        out[row] = 0.5 * (lor(w[:, None] - E[None, :])
                          + lor(w[:, None] + E[None, :])).mean(axis=1)
    return out


def omega_tilde_limit(eig_by_spin, phi, U, T) -> float:
    """sum phi^2/U - T sum_s sum_k ln cosh(e_ks / (2T)) (infinite M)."""
    tot = float(np.sum(np.asarray(phi) ** 2)) / U
    for e in eig_by_spin:
        x = np.abs(np.asarray(e)) / (2.0 * T)
        # ln cosh x = x + log1p(exp(-2x)) - ln 2, stable for large x
        tot -= T * float(np.sum(x + np.log1p(np.exp(-2.0 * x)) - np.log(2.0)))
    return tot


def hf_neel_m(L, t, U, delta, T, hi: float = 20.0) -> float:
    """Root of m = (U/2) m_A with Fermi occupations (M -> infinity):
    m_A = -(1/N) sum_k sum_s s h_s tanh(E_ks/(2T)) / (2 E_ks)."""
    e2 = bloch_energies(L, t) ** 2
    N = L * L

    def f(m):
        acc = 0.0
        for s in (1, -1):
            h = 0.5 * delta - s * m
            E = np.sqrt(e2 + h * h)
            acc += s * h * np.sum(np.tanh(E / (2.0 * T)) / (2.0 * E))
        return m + 0.5 * U * acc / N

    lo = 1e-9
    if f(lo) >= 0.0:
        return 0.0
    return brentq(f, lo, hi, xtol=1e-15, rtol=1e-15, maxiter=500)
