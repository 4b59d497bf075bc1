"""Lattice, one-body Hamiltonian and Matsubara grid (oracle; test infrastructure).

Sec. II, Eq. (1): ionic Hubbard model on a half-filled L x L square lattice
with nearest-neighbour hopping t, staggered potential and on-site U.  After
dropping the charge channel and taking a static Hubbard-Stratonovich field
(Eqs. (4)-(6)), each spin s sees the real symmetric one-body matrix

    H_s(phi) = -t K + (Delta/2) S - s diag(phi)

(phi couples as -s phi_i with the potential sum phi_i^2 / U, the paper's
Eq. (5) form with phi rescaled by 1/2, and the ionic potential is +-Delta/2,
i.e. Delta here is twice the paper's).  Matsubara frequencies
w_n = (2n+1) pi T (text after Eq. (7)).

Pins (tests/test_oracle_pins.py): the Bloch spectrum of K and the staggered
closed form check K, S and the sign of the field term; the Leibniz brute
force checks the 2x2 lattice.
"""
from __future__ import annotations

import numpy as np


def n_sites(L: int) -> int:
    return L * L


def _check_L(L: int) -> None:
    if L < 2 or L % 2:
        raise ValueError("L must be even and >= 2 (the staggered sign must be "
                         "periodic)")


def neighbours(L: int) -> np.ndarray:
    """[N, 4] neighbour sites of i = x + L*y: +x, -x, +y, -y (periodic)."""
    _check_L(L)
    out = np.empty((L * L, 4), dtype=np.int64)
    for y in range(L):
        for x in range(L):
            i = x + L * y
            out[i, 0] = (x + 1) % L + L * y
            out[i, 1] = (x - 1) % L + L * y
            out[i, 2] = x + L * ((y + 1) % L)
            out[i, 3] = x + L * ((y - 1) % L)
    return out


def kinetic_matrix(L: int) -> np.ndarray:
    """K_ij = number of directions d in {+x,-x,+y,-y} with j = i + d (mod L)."""
    nb = neighbours(L)
    N = L * L
    K = np.zeros((N, N))
    for i in range(N):
        for d in range(4):
            K[i, nb[i, d]] += 1.0
    return K


def stagger_signs(L: int) -> np.ndarray:
    """S_ii = (-1)^(x+y)."""
    _check_L(L)
    s = np.empty(L * L)
    for y in range(L):
        for x in range(L):
            s[x + L * y] = 1.0 if (x + y) % 2 == 0 else -1.0
    return s


def hamiltonian(L: int, t: float, delta: float, phi: np.ndarray,
                spin: int, onsite: np.ndarray | None = None) -> np.ndarray:
    """Dense H_s(phi) = -t K + (Delta/2) S - s diag(phi) [+ diag(onsite)].

    `onsite` is an optional extra site potential (a disordered lattice); it is
    zero for the paper's ionic model.
    """
    if spin not in (1, -1):
        raise ValueError("spin must be +1 or -1")
    phi = np.asarray(phi, dtype=np.float64)
    H = -t * kinetic_matrix(L)
    H += np.diag(0.5 * delta * stagger_signs(L) - spin * phi)
    if onsite is not None:
        H += np.diag(np.asarray(onsite, dtype=np.float64))
    return H


def matsubara(T: float, M: int) -> np.ndarray:
    """w_n = (2n+1) pi T for n = 0 .. M-1 (the positive half of the grid)."""
    return (2.0 * np.arange(M) + 1.0) * np.pi * T
