"""Writes c2_trajectory_20x20.json: the oracle's ADAM trajectory on the
20x20 Hubbard lattice (U = 6, Delta = 0, n_max = 512) from the seeded
phi0 ~ U[-0.5, 0.5) (seed 0 at T = 0.1, seed 1 at T = 0.6), lr = 0.01,
2000 steps: phi after 200 and after 2000 steps, |phi|, Omega~, and the DOS
of the final phi on a coarse grid (eta = 0.05).

Run from the repository root:  python tests/golden/make_c2_trajectory.py
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

W_GRID = np.linspace(-6.0, 6.0, 49)


def main():
    out = {}
    for name in ("hubbard_20x20_T0.1", "hubbard_20x20_T0.6"):
        wl = synth.WORKLOADS[name]
        p = dict(wl["params"])
        phi0 = synth.make_phi0(p["L"], wl["phi0"])
        phi200, info200 = oracle.adam_solve(p, phi0, 200)
        phi, info = oracle.adam_solve(p, phi0, 2000)
        rho = oracle.dos(p, phi, W_GRID, 0.05)
        out[name] = dict(phi200=phi200.tolist(), phi2000=phi.tolist(),
                         af_order=float(oracle.af_order(phi, p["L"])),
                         omega_tilde=float(info["omega_tilde"]),
                         dos_w=W_GRID.tolist(), dos_eta=0.05,
                         dos=rho.tolist())
        print(name, "|phi| =", out[name]["af_order"], flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                        "c2_trajectory_20x20.json")
    with open(path, "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
