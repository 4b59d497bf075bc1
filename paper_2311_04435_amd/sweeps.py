"""The paper's parameter sweeps (Sec. III), run through the request server.

    E1  |phi| vs the Matsubara cut-off w_{n_max}: 20x20, U = 6, T = 0.1, 0.6
    E3  DOS of the converged field: 20x20, U = 6, T = 0.2 and 1.3
    E4  |phi| vs T: 20x20, U = 4 and 6
    E5  |phi| vs Delta: 20x20, T = 0.1, U = 3, 4, 5
    E6  DOS in the ionic model: 20x20, U = 3, T = 0.1, Delta = 0.3, 0.39, 0.4

Every point starts from a staggered field m0 (-1)^(x+y) plus seeded noise
(the antiferromagnetic basin; a random start can stop in a metastable
domain pattern) and runs a fixed number of ADAM steps.  Unless a point sets
n_max itself, the cut-off follows the paper's choice w_{n_max} ~ 100:
n_max = ceil(100 / (2 pi T)).  All points of a sweep are submitted at once;
the server batches those of equal shape.

    python -m paper_2311_04435_amd.sweeps --experiment E4 --out e4.json
"""
from __future__ import annotations

import argparse
import json
import math
from typing import Dict, List, Optional

import numpy as np
import torch

from . import Params, dos as _dos
from .serve import Server

W_MAX = 100.0   # the paper's Matsubara cut-off (Sec. III)


def n_max_for(T: float, w_max: float = W_MAX) -> int:
    """Number of positive Matsubara frequencies with w_n <= w_max."""
    return max(1, int(math.ceil(w_max / (2.0 * math.pi * T))))


def points(experiment: str, L: int = 20) -> List[dict]:
    """Parameter points of one experiment (dicts for Params)."""
    out = []
    if experiment == "E1":
        for T in (0.1, 0.6):
            for w in (2.0, 5.0, 10.0, 20.0, 50.0, 100.0, 200.0):
                out.append(dict(L=L, U=6.0, T=T, delta=0.0,
                                n_max=n_max_for(T, w), w_max=w))
    elif experiment == "E3":
        for T in (0.2, 1.3):
            out.append(dict(L=L, U=6.0, T=T, delta=0.0, n_max=n_max_for(T)))
    elif experiment == "E4":
        for U in (4.0, 6.0):
            for T in (0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.8, 1.0, 1.3, 1.6):
                out.append(dict(L=L, U=U, T=T, delta=0.0, n_max=n_max_for(T)))
    elif experiment == "E5":
        for U in (3.0, 4.0, 5.0):
            for d in (0.0, 0.2, 0.3, 0.39, 0.4, 0.5, 0.68, 0.8, 1.0, 1.19, 1.4):
                out.append(dict(L=L, U=U, T=0.1, delta=d, n_max=n_max_for(0.1)))
    elif experiment == "E6":
        for d in (0.3, 0.39, 0.4):
            out.append(dict(L=L, U=3.0, T=0.1, delta=d, n_max=n_max_for(0.1)))
    else:
        raise ValueError(f"unknown experiment {experiment!r}")
    return out


def staggered_start(L: int, seed: int, m0: float = 1.0,
                    noise: float = 0.05) -> np.ndarray:
    import synth
    return synth.phi0_staggered(L, seed, m0, noise)


def run(pts: List[dict], steps: int = 1000, factor: str = "ldlt",
        precision: str = "fp64", lr: float = 0.01, m0: float = 1.0,
        server: Optional[Server] = None, max_batch: int = 16,
        progress: bool = False, tail: bool = False) -> List[dict]:
    """Solve every point (through one server); returns per point the
    parameters, |phi|, Omega~, max|g|, and phi itself (float64 CPU array)."""
    own = server is None
    srv = server if server is not None else Server(max_batch=max_batch)
    try:
        tickets = []
        for k, pt in enumerate(pts):
            p = Params(L=pt["L"], U=pt["U"], T=pt["T"], n_max=pt["n_max"],
                       delta=pt.get("delta", 0.0), t=pt.get("t", 1.0),
                       precision=precision, factor=factor, tail=tail)
            phi0 = torch.as_tensor(staggered_start(pt["L"], 4000 + k, m0),
                                   dtype=torch.float64, device="cuda")
            tickets.append((srv.submit(p, phi0, steps, lr=lr), p))
        done = {}
        left = {t for t, _ in tickets}
        while left:
            srv.progress(0.005)
            for t in list(left):
                r = srv.poll(t)
                if r is not None:
                    done[t] = r
                    left.discard(t)
                    if progress:
                        print(f"sweep: {len(done)}/{len(tickets)} points done",
                              flush=True)
    finally:
        if own:
            srv.close()
    out = []
    for (t, p), pt in zip(tickets, pts):
        phi, _, _, res, _ = done[t]
        out.append(dict(point=pt, af_order=res["af_order"],
                        omega_tilde=res["omega_tilde"],
                        max_abs_grad=res["max_abs_grad"],
                        flags=res["flags"], params=p,
                        phi=phi.cpu().numpy()))
    return out


def dos_of(result: dict, w: np.ndarray, eta: float = 0.05) -> np.ndarray:
    """[2, n_w] DOS (spin up first) of a solved point."""
    p = result["params"]
    phi = torch.as_tensor(result["phi"], dtype=torch.float64, device="cuda")
    wt = torch.as_tensor(np.asarray(w, dtype=np.float64), device="cuda")
    return _dos(p, phi, wt, eta).cpu().numpy()


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--experiment", default="E4",
                    choices=["E1", "E3", "E4", "E5", "E6"])
    ap.add_argument("--L", type=int, default=20)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--factor", default="ldlt")
    ap.add_argument("--tail", action="store_true",
                    help="high Matsubara frequencies from the moments of H")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    pts = points(args.experiment, args.L)
    res = run(pts, args.steps, factor=args.factor, progress=True,
              tail=args.tail)
    rows: List[Dict] = []
    w = np.linspace(-6.0, 6.0, 241)
    for r in res:
        row = dict(r["point"], af_order=r["af_order"],
                   omega_tilde=r["omega_tilde"],
                   max_abs_grad=r["max_abs_grad"])
        if args.experiment in ("E3", "E6"):
            row["dos_w"] = w.tolist()
            row["dos"] = dos_of(r, w).tolist()
        rows.append(row)
        print(json.dumps({k: v for k, v in row.items() if k not in ("dos", "dos_w")}),
              flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(rows, f)


if __name__ == "__main__":
    main()
