"""Writes c5_trajectory_48x48.json: the oracle's ADAM trajectory on the
48x48 ionic Hubbard lattice (U = 5, Delta = 0.5, T = 0.1, n_max = 128)
from the seeded staggered start (m = 1 plus U[-0.1, 0.1) noise, seed 0),
lr = 0.01: phi after 20 and after 1000 steps, |phi|, Omega~ and the
gradient at the final phi, and the DOS of the final phi on a coarse grid
(eta = 0.05).

Run from the repository root:  python tests/golden/make_c5_trajectory.py
(about 45 minutes on 8 cores: one pair of 2304x2304 eigendecompositions per
step).  Only the oracle and the seeded input generators are used.
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

W_GRID = np.linspace(-6.0, 6.0, 25)
STEPS = 1000


def main():
    wl = synth.WORKLOADS["ionic_48x48"]
    p = dict(wl["params"])
    phi0 = synth.make_phi0(p["L"], wl["phi0"])
    phi, info = oracle.adam_solve(p, phi0, STEPS, record=(20,))
    rho = oracle.dos(p, phi, W_GRID, 0.05)
    out = dict(phi20=info["record"][20].tolist(), phi1000=phi.tolist(),
               af_order=float(oracle.af_order(phi, p["L"])),
               omega_tilde=float(info["omega_tilde"]),
               grad=info["grad"].tolist(),
               dos_w=W_GRID.tolist(), dos_eta=0.05, dos=rho.tolist())
    print("|phi| =", out["af_order"], "Omega~ =", out["omega_tilde"], flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                        "c5_trajectory_48x48.json")
    with open(path, "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
