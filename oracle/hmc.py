"""Hybrid Monte Carlo of the SCA weight exp(-Omega(phi)/T) — TEST
INFRASTRUCTURE (the oracle of sca_hmc).

The static-field partition function of the semiclassical approximation is
an integral over the auxiliary field with weight exp(-Omega(phi)/T)
(Sec. II); Omega~ differs from Omega by a phi-independent constant, so it
gives the same distribution.  Sampling it by Hybrid Monte Carlo (Duane,
Kennedy, Pendleton and Roweth, 1987) with the fictitious Hamiltonian
H(phi, p) = Omega~(phi)/T + |p|^2/2:

  leapfrog of n_leap steps of size eps:
      p <- p - (eps/2) grad Omega / T
      repeat n_leap times:  phi <- phi + eps p;  p <- p - c grad Omega / T
                            (c = eps, except eps/2 on the last step)
  accept the end point if u < exp(-(H_end - H_start)), else keep the start.

The momenta and the uniforms u are inputs (the caller draws them), so a
chain is a deterministic function of its inputs.  Omega~ and its gradient
come from route S (`api.omega_tilde`, `api.grad`).

Pins (tests/test_oracle_pins.py): the leapfrog is time-reversible (negating
the end momentum and integrating again returns to the start), its energy
error falls as eps^2, and the acceptance rule follows exp(-dH).  The
distribution itself is not pinned to values of the paper (it shows none):
parity unpinned for the sampled physics.
"""
from __future__ import annotations

import numpy as np

from .api import grad, omega_tilde


def hmc_hamiltonian(p, phi, mom, onsite=None) -> float:
    return omega_tilde(p, phi, onsite) / p["T"] + 0.5 * float(mom @ mom)


def leapfrog(p, phi, mom, eps: float, n_leap: int, onsite=None):
    """(phi, p) after n_leap leapfrog steps of size eps."""
    T = p["T"]
    phi = np.array(phi, dtype=np.float64)
    mom = np.array(mom, dtype=np.float64)
    mom = mom - 0.5 * eps * grad(p, phi, onsite) / T
    for k in range(1, n_leap + 1):
        phi = phi + eps * mom
        c = 0.5 * eps if k == n_leap else eps
        mom = mom - c * grad(p, phi, onsite) / T
    return phi, mom


def hmc_chain(p, phi0, momenta, uniforms, eps: float, n_leap: int,
              onsite=None):
    """Chain of len(uniforms) trajectories from phi0; returns (phi, accepted,
    h_start, h_end) with one entry per trajectory."""
    phi = np.array(phi0, dtype=np.float64)
    acc, h0s, h1s = [], [], []
    for t, u in enumerate(uniforms):
        mom = np.asarray(momenta[t], dtype=np.float64)
        h0 = hmc_hamiltonian(p, phi, mom, onsite)
        phin, momn = leapfrog(p, phi, mom, eps, n_leap, onsite)
        h1 = hmc_hamiltonian(p, phin, momn, onsite)
        a = (h1 - h0 <= 0.0) or (u < np.exp(-(h1 - h0)))
        if a:
            phi = phin
        acc.append(int(a))
        h0s.append(h0)
        h1s.append(h1)
    return phi, np.array(acc), np.array(h0s), np.array(h1s)
