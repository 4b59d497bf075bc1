"""Writes fd_grad_32x32.json: central finite differences of the oracle's
Omega~ on the 32x32 ionic lattice, the reference for the gradient the GPU
path returns (through its autograd backward).

Omega~ differs from Omega by a phi-independent constant (the Matsubara
normalisation of each ln|det|), so both share the gradient
dOmega/dphi_i = 2 phi_i / U - 2 T sum_s s sum_n Re (A_ns^-1)_ii (the
potential of Eq. (7) differentiated in phi).  Omega~ is used for the
differences because its magnitude, and so the rounding floor of a
difference quotient, is far smaller than Omega's.

Cases: 16 fields phi ~ U[-0.5, 0.5) (seeds 0..15) at L = 32, t = 1,
Delta = 1, T = 0.1, n_max = 256, U cycling through 2, 4, 6; per field
4 Rademacher directions and 8 coordinate directions.  h = 1e-6.
floor = 4 eps |Omega~| / h bounds the rounding part of each quotient; the
truncation part, h^2 |Omega~'''| / 6, is below 1e-10 here.

Run from the repository root:  python tests/golden/make_fd_grad.py
Only the oracle and the seeded input generators are used.
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

H = 1e-6
L = 32
N = L * L
EPS = np.finfo(np.float64).eps


def cases():
    for seed in range(16):
        U = (2.0, 4.0, 6.0)[seed % 3]
        p = dict(L=L, t=1.0, U=U, delta=1.0, T=0.1, n_max=256)
        dirs = [("rademacher", 5000 + 16 * seed + j) for j in range(4)]
        coords = [int(i) for i in synth.sample_indices(7000 + seed, N, 8)]
        yield seed, p, dirs, coords


def direction(kind, arg):
    if kind == "rademacher":
        return synth.rademacher(arg, N)
    d = np.zeros(N)
    d[arg] = 1.0
    return d


def main():
    out = dict(h=H, L=L, cases=[])
    for seed, p, dirs, coords in cases():
        phi = synth.uniform(seed, N, -0.5, 0.5)
        om = oracle.omega_tilde(p, phi)
        floor = 4.0 * EPS * abs(om) / H
        items = [(k, a) for k, a in dirs] + [("coord", c) for c in coords]
        vals = []
        for kind, arg in items:
            d = direction(kind, arg)
            fp = oracle.omega_tilde(p, phi + H * d)
            fm = oracle.omega_tilde(p, phi - H * d)
            vals.append(dict(kind=kind, arg=arg, fd=(fp - fm) / (2.0 * H)))
        out["cases"].append(dict(seed=seed, params=p, omega_tilde=om,
                                 floor=floor, directions=vals))
        print(f"seed {seed}: Omega~ {om:.6f}, floor {floor:.1e}", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                        "fd_grad_32x32.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
