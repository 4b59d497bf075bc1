#!/usr/bin/env python3
"""Benchmark of the SCA+ADAM hot path on one MI355X.

A step is one ADAM update: assemble every A_ns = i w_n - H_s(phi) on chip,
factor it (pivoted complex LU), take ln|det| and diag(A^-1) for all 2 n_max
matrices, reduce over frequencies and spins, and update phi, m, v.  Inputs
are synthetic and seeded (no dataset exists for this method); phi, m, v are
resident in HBM before the timed region starts.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--precision P]

Prints one JSON line.  Besides the contract fields it carries
  roofline      the dominant kernel's achieved rate against the MI355X peak,
                from HIP events on the library's stream over a second,
                profiled run of the same steps;
  cpu_baseline  the FP64 oracle timed on this host on a bounded sample;
  l32           steps/s of the 32x32 ionic lattice: FP32 refined, FP64
                pivoted LU, FP64 symmetric L D L^T, FP64 spectral;
  symmetric_ldlt the same workload on the symmetric route (unpivoted
                L D L^T, exact for these complex symmetric matrices, half
                the flops) with its own roofline;
  hmc           Hybrid Monte Carlo of exp(-Omega/T) on the workload
                (symmetric route with the tail): trajectories/s,
                acceptance;
  tail          the same workload with only the low Matsubara frequencies
                factorised and the rest from the moments of H (pivoted LU,
                then symmetric), with n_factorised and their rooflines;
  serving       served solves/s and p50/p99 latency of a Poisson stream of
                mixed requests through the request server, next to the
                one-at-a-time FIFO baseline on the same GPU;
  serving_tail  the same stream with the Matsubara tail by moments;
  serving_spectral the same stream on the spectral route;
  spectral      the spectral route (factor eigh: one eigendecomposition of
                H per spin, every frequency from the spectrum) on the
                workload with its per-class times, on the 48x48 ionic
                lattice, and the FP32-refined factorisation route on that
                lattice for comparison.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("ADAM steps/s (logdet+grad, all ω_n,σ) at L=20,32; "
          "served solves/s + p99 ms")
PEAK = {"fp64": 78.6, "fp32": 157.3}   # dense MFMA TFLOP/s, MI355X
HBM_PEAK = 8000.0                       # GB/s

# HBM bytes per launch from rocprofv3 FETCH_SIZE and WRITE_SIZE runs, scaled
# by the same counters on a copy kernel of known size (read x 2.0, write x
# 1.0); profiles/lu_f64_hubbard_20x20.md and ldlt_f64_hubbard_20x20.md
# have the runs.  Keyed by (kernel
# class, workload, precision, factorisation) with the SHA-256 of the kernel source the
# counters were taken on: a changed source reports null.
TRAFFIC = {
    ("lu", "hubbard_20x20_T0.1", "fp64", "lu"): (
        19.896e9, "k_factor.hip",
        "6ceab981287d54c76a56f45a669cdc31344a6e9317313338269fb0db00113ffa"),
    ("ldlt", "hubbard_20x20_T0.1", "fp64", "ldlt"): (
        8.093e9, "k_ldlt.hip",
        "4cf959a57de490a72fb2705cb64b0f9c8a9a37292161af1ff71b6f28f1ef2ca2"),
    # profiles/fp32r_hubbard_20x20.md, profiles/fp32r_ionic_48x48.md
    ("lu", "hubbard_20x20_T0.1", "fp32r", "lu"): (
        8.431e9, "k_factor.hip",
        "6ceab981287d54c76a56f45a669cdc31344a6e9317313338269fb0db00113ffa"),
    ("trtri", "hubbard_20x20_T0.1", "fp32r", "lu"): (
        8.994e9, "k_factor.hip",
        "6ceab981287d54c76a56f45a669cdc31344a6e9317313338269fb0db00113ffa"),
    ("wvgemm", "hubbard_20x20_T0.1", "fp32r", "lu"): (
        4.854e9, "k_refine.hip",
        "8a478518d1f480b6c3be0bc33e3b7f3901935e51e2e6a3c9061831831e5668f1"),
    ("refine", "hubbard_20x20_T0.1", "fp32r", "lu"): (
        1.483e9, "k_refine.hip",
        "8a478518d1f480b6c3be0bc33e3b7f3901935e51e2e6a3c9061831831e5668f1"),
    ("lu", "ionic_48x48", "fp32r", "lu"): (
        1376.94e9, "k_factor.hip",
        "6ceab981287d54c76a56f45a669cdc31344a6e9317313338269fb0db00113ffa"),
}


def measured_traffic(kernel: str, workload: str, prec: str, factor: str):
    import hashlib
    hit = TRAFFIC.get((kernel, workload, prec, factor))
    if hit is None:
        return None
    src = os.path.join(ROOT, "paper_2311_04435_amd", "csrc", hit[1])
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    return hit[0] if sha == hit[2] else None


def kernel_work(kind: str, N: int, B: int):
    """Algorithmic work of one launch: (amount, unit, bound)."""
    n3 = float(N) ** 3
    if kind == "lu":          # P A = L U, complex: (8/3) N^3 real flops
        return B * 8.0 / 3.0 * n3, "flop", "mfma"
    if kind == "trtri":       # U^-1 and L^-1: 2 x (4/3) N^3
        return B * 8.0 / 3.0 * n3, "flop", "mfma"
    if kind == "ldlt":        # A = L D L^T, complex symmetric: (4/3) N^3
        return B * 4.0 / 3.0 * n3, "flop", "mfma"
    if kind == "trtri_sym":   # L^-T alone: (4/3) N^3
        return B * 4.0 / 3.0 * n3, "flop", "mfma"
    if kind == "small":       # fused LU + both triangular inverses
        return B * 16.0 / 3.0 * n3, "flop", "mfma"
    if kind == "wvgemm":      # X = W V, upper x unit lower: (8/3) N^3
        return B * 8.0 / 3.0 * n3, "flop", "mfma"
    if kind == "refine":      # reads X (complex64 N x N) once
        return B * 8.0 * N * N, "byte", "hbm"
    if kind == "diagdot":     # reads the W and V triangles once
        return B * 16.0 * N * N, "byte", "hbm"
    if kind == "symdiag":     # reads the L^-T triangle once
        return B * 8.0 * N * N, "byte", "hbm"
    if kind == "reduce":      # reads diag(A^-1) of every matrix
        return B * 16.0 * N, "byte", "hbm"
    if kind == "tridiag":     # spectral route, both spins: Householder
        # reduction (4/3) N^3 and the accumulated reflectors (4/3) N^3
        return 2 * 8.0 / 3.0 * n3, "flop", "alu"
    return None


def hmc_line(sca, name, n_traj=4, n_leap=10, eps=0.02, factor="ldlt",
             tail=True):
    """Hybrid Monte Carlo of exp(-Omega/T) on a workload: trajectories/s
    (n_leap + 1 force evaluations each) from the converged antiferromagnet
    neighbourhood (staggered start), momenta and uniforms seeded."""
    import torch
    import synth
    wl = synth.WORKLOADS[name]
    p = sca.Params.from_dict(wl["params"], factor=factor, tail=tail)
    N = p.L * p.L
    phi = torch.as_tensor(synth.phi0_staggered(p.L, 7, 1.0, 0.05),
                          dtype=torch.float64).cuda()
    moms = torch.as_tensor(synth.normal(8, (n_traj + 1) * N).reshape(
        n_traj + 1, N), dtype=torch.float64).cuda()
    us = synth.uniform(9, n_traj + 1, 0.0, 1.0)
    ctx = sca.Context()
    ctx.hmc(p, phi, moms[:1], us[:1], eps, n_leap)      # warm-up trajectory
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    acc, h0, h1 = ctx.hmc(p, phi, moms[1:], us[1:], eps, n_leap)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"workload": name, "factor": factor, "tail": tail,
            "n_leap": n_leap, "eps": eps, "trajectories": n_traj,
            "trajectories_per_s": n_traj / dt,
            "force_evals_per_s": n_traj * (n_leap + 1) / dt,
            "acceptance": float(acc.mean()),
            "mean_abs_dH": float(abs(h1 - h0).mean())}


def cpu_baseline(budget_s: float):
    """The FP64 oracle on this host's cores, over whole ADAM steps only (no
    extrapolation): route D (the method's definition: a pivoted complex LU
    and inverse per Matsubara matrix, NumPy) on one whole step of the 20x20
    workload (1024 matrices of 400 x 400) and on whole steps of the 4x4
    workload; route S (one eigendecomposition per spin, algorithmically
    ~n_max times cheaper) on whole 20x20 steps for about budget_s."""
    import numpy as np
    import oracle
    from oracle.adam import AdamState, adam_step
    import synth
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        threads = 1
    nproc = os.cpu_count() or 1
    try:
        avail = len(os.sched_getaffinity(0))
    except Exception:
        avail = nproc

    def route_d_steps(name, min_s, max_steps):
        wl = synth.WORKLOADS[name]
        p = dict(wl["params"])
        hy = wl["adam"]
        x = synth.make_phi0(p["L"], wl["phi0"])
        st = AdamState.zeros(x.size)
        t0 = time.perf_counter()
        steps = 0
        while steps < max_steps and (steps == 0 or
                                     time.perf_counter() - t0 < min_s):
            g = oracle.grad_d(p, x)
            x = adam_step(x, g, st, hy["lr"], hy["beta1"], hy["beta2"], hy["eps"])
            steps += 1
        return steps, time.perf_counter() - t0

    n20, t20 = route_d_steps("hubbard_20x20_T0.1", 0.0, 1)
    n4, t4 = route_d_steps("hubbard_4x4", 3.0, 1000)
    wl = synth.WORKLOADS["hubbard_20x20_T0.1"]
    p = dict(wl["params"])
    phi = synth.make_phi0(p["L"], wl["phi0"])
    t0 = time.perf_counter()
    ns = 0
    while ns == 0 or time.perf_counter() - t0 < budget_s:
        oracle.adam_solve(p, phi, 1)
        ns += 1
    ts = time.perf_counter() - t0
    return {"value": n20 / t20, "unit": "steps/s", "cores": int(threads),
            "kind": "oracle",
            "sample": (f"route D (pivoted complex LU + inverse of each of the "
                       f"1024 Matsubara matrices of 400 x 400, NumPy FP64, "
                       f"then the ADAM update): {n20} whole step of the 20x20 "
                       f"workload in {t20:.1f} s"),
            "nproc": nproc, "cpus_available": avail, "blas_threads": int(threads),
            "route_d_4x4": {"steps": n4, "seconds": t4,
                            "steps_per_s": n4 / t4},
            "route_s_20x20": {"steps": ns, "seconds": ts,
                              "steps_per_s": ns / ts,
                              "note": "eigendecomposition of H per spin and "
                                      "closed Matsubara sums: O(N^3) per step "
                                      "instead of O(n_max N^3)"}}


def workload_rate(sca, name, prec, steps, warmup, factor="lu", tail=False):
    """Timed ADAM steps of a named workload (phi, m, v resident on the GPU)."""
    import torch
    import synth
    wl = synth.WORKLOADS[name]
    p = sca.Params.from_dict(wl["params"], precision=prec, factor=factor,
                             tail=tail)
    hy = wl["adam"]
    phi = torch.as_tensor(synth.make_phi0(p.L, wl["phi0"]),
                          dtype=torch.float64).cuda()
    m, v = torch.zeros_like(phi), torch.zeros_like(phi)
    ctx = sca.Context()
    kw = dict(lr=hy["lr"], beta1=hy["beta1"], beta2=hy["beta2"], eps=hy["eps"],
              final_eval=False)
    ctx.adam_solve(p, phi, m, v, warmup, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.adam_solve(p, phi, m, v, steps, t0=warmup, **kw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = {"workload": name, "precision": prec, "factor": factor,
           "steps": steps,
           "steps_per_s": steps / dt, "ms_per_step": 1e3 * dt / steps}
    if tail:
        out["tail"] = True
        out["n_factorised"] = sca.tail_split(p, phi)
    return out


def route_line(sca, name, prec, factor, steps, warmup, tail=False):
    """Steps/s of a workload on a given route, with the per-kernel averages
    (HIP events) and the roofline of its dominant kernel."""
    out = workload_rate(sca, name, prec, steps, warmup, factor, tail)
    import torch
    import synth
    wl = synth.WORKLOADS[name]
    p = sca.Params.from_dict(wl["params"], precision=prec, factor=factor,
                             tail=tail)
    phi = torch.as_tensor(synth.make_phi0(p.L, wl["phi0"]),
                          dtype=torch.float64).cuda()
    ctx = sca.Context()
    m, v = torch.zeros_like(phi), torch.zeros_like(phi)
    hy = wl["adam"]
    kw = dict(lr=hy["lr"], beta1=hy["beta1"], beta2=hy["beta2"], eps=hy["eps"],
              final_eval=False)
    ctx.adam_solve(p, phi, m, v, warmup, **kw)
    n_fact = sca.tail_split(p, phi)   # frequencies factorised in this call
    ctx.profile(True)
    ctx.adam_solve(p, phi, m, v, steps, t0=warmup, **kw)
    prof = ctx.profile_read()
    ctx.profile(False)
    out["kernels"] = {k: {"avg_ms": ms / n, "launches": n} for k, (ms, n) in prof.items()}
    dom = max(prof, key=lambda k: prof[k][0])
    N, B = p.L * p.L, 2 * n_fact
    work = kernel_work(dom, N, B)
    if work is not None:
        amount, unit, bound = work
        avg_s = prof[dom][0] / prof[dom][1] / 1e3
        if unit == "flop":
            peak = PEAK["fp32" if prec == "fp32r" else "fp64"]
            ach = amount / avg_s / 1e12
            out["roofline"] = {"bound": bound, "kernel": dom, "achieved": ach,
                               "peak": peak, "unit": "TFLOP/s",
                               "frac": ach / peak,
                               "traffic": None if tail else
                               measured_traffic(dom, name, prec, factor)}
        else:
            ach = amount / avg_s / 1e9
            out["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": ach,
                               "peak": HBM_PEAK, "unit": "GB/s",
                               "frac": ach / HBM_PEAK,
                               "traffic": None if tail else
                               measured_traffic(dom, name, prec, factor)}
    return out


def serving(sca, n_req, steps, n_max, Ls, max_batch, load=1.5, seed=0,
            factor="lu", tail=False):
    """Poisson stream of mixed requests: one at a time (FIFO, measured
    service times) vs the request server (real time)."""
    import numpy as np
    import torch
    import synth
    from paper_2311_04435_amd.serve import (Server, run_stream, fifo_latencies,
                                            latency_summary)
    reqs = []
    for r in synth.serving_stream(n_req, seed, n_max, Ls=Ls):
        p = sca.Params.from_dict(r["params"], factor=factor, tail=tail)
        phi0 = torch.as_tensor(synth.make_phi0(p.L, r["phi0"]),
                               dtype=torch.float64).cuda()
        reqs.append(dict(params=p, phi0=phi0, n_steps=steps))
    # warm every shape once (code objects, workspaces)
    ctx = sca.default_context()
    for L in sorted({r["params"].L for r in reqs}):
        r = next(q for q in reqs if q["params"].L == L)
        sca.adam_solve(r["params"], r["phi0"], 1)
    service, alone = [], []
    for k, r in enumerate(reqs):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = sca.adam_solve(r["params"], r["phi0"], r["n_steps"])
        torch.cuda.synchronize()
        service.append(time.perf_counter() - t0)
        alone.append(out[0])
        if (k + 1) % 32 == 0:
            print(f"bench: serving, one at a time {k + 1}/{len(reqs)} "
                  f"({sum(service):.1f} s)", file=sys.stderr, flush=True)
    service = np.array(service)
    print(f"bench: serving, one-at-a-time pass {service.sum():.1f} s",
          file=sys.stderr, flush=True)
    rate = load * len(reqs) / service.sum()
    arrivals = synth.poisson_arrivals(seed + 17, len(reqs), rate)
    fifo_lat, fifo_span = fifo_latencies(arrivals, service)
    with Server(max_batch=max_batch) as srv:
        # warm the server's groups with one short solve per shape
        warm = [srv.submit(r["params"], r["phi0"], 1)
                for r in {q["params"].L: q for q in reqs}.values()]
        srv.drain(warm)
        def done(n):
            if n % 32 == 0:
                print(f"bench: serving, served {n}/{len(reqs)}",
                      file=sys.stderr, flush=True)
        results, lat, span = run_stream(srv, reqs, arrivals, on_done=done)
    print(f"bench: serving, served pass {span:.1f} s", file=sys.stderr,
          flush=True)
    same = all(torch.equal(results[k][0], alone[k]) for k in range(len(reqs)))
    del ctx
    by_L = {}
    for r, t in zip(reqs, service):
        by_L.setdefault(r["params"].L, []).append(t)
    return {"workload": (f"{n_req} requests, L in {sorted(set(Ls))}, "
                         f"n_max={n_max}, {steps} ADAM steps each, FP64 "
                         f"({ {'lu': 'pivoted LU', 'ldlt': 'L D L^T', 'eigh': 'spectral'}[factor] }"
                         f"{', Matsubara tail by moments' if tail else ''}), "
                         f"U~U[2,8], Delta~U[0,2], T~U[0.05,0.6]"),
            "arrivals": f"Poisson, {rate:.3f}/s = {load} x FIFO capacity",
            "max_batch": max_batch,
            "served": latency_summary(lat, span),
            "fifo_one_at_a_time": latency_summary(fifo_lat, fifo_span),
            "alone_vs_mix_bitwise": bool(same),
            "service_s_by_L": {str(k): {"requests": len(v),
                                        "mean_s": float(np.mean(v))}
                               for k, v in sorted(by_L.items())}}


def c1_line(sca, steps=500, warmup=20):
    """The 4x4 workload (512 matrices of 16 x 16 per step, fused small
    kernel): microseconds per ADAM step; launch- and latency-bound, so no
    roofline fraction is claimed."""
    out = workload_rate(sca, "hubbard_4x4", "fp64", steps, warmup)
    out["us_per_step"] = 1e3 * out["ms_per_step"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="hubbard_20x20_T0.1")
    ap.add_argument("--precision", default=None, help="fp64 | fp32r")
    ap.add_argument("--factor", default="lu",
                    help="lu (pivoted, default) | ldlt (symmetric, unpivoted)")
    ap.add_argument("--cpu-seconds", type=float, default=8.0,
                    help="route S part of the CPU baseline (route D always "
                         "times one whole 20x20 step)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-l32", action="store_true",
                    help="skip the 32x32 and 48x48 lines")
    ap.add_argument("--no-tail", action="store_true",
                    help="skip the Matsubara-tail lines")
    ap.add_argument("--no-spectral", action="store_true",
                    help="skip the spectral-route lines (factor eigh)")
    ap.add_argument("--no-hmc", action="store_true",
                    help="skip the Hybrid Monte Carlo line")
    ap.add_argument("--no-symmetric", action="store_true",
                    help="skip the symmetric-route line")
    ap.add_argument("--serving-requests", type=int, default=256,
                    help="0 skips the serving measurement")
    ap.add_argument("--serving-steps", type=int, default=200)
    ap.add_argument("--serving-nmax", type=int, default=256)
    ap.add_argument("--serving-L", default="8,12,16,20,24,32")
    ap.add_argument("--serving-batch", type=int, default=16)
    ap.add_argument("--serving-factor", default="eigh",
                    help="lu | ldlt | eigh (every route computes the same "
                         "sums; eigh is the fastest on this stream)")
    ap.add_argument("--serving-tail", action="store_true",
                    help="serve with the Matsubara tail by moments")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (3 times), "
                         "the reference for the HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is "
              "not supported (the Matsubara batch would shard across GPUs "
              "with one all-reduce of the gradient per step)", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            torch.mul(a, 1.0, out=b)     # reads 4n bytes, writes 4n bytes
        torch.cuda.synchronize()
        print(json.dumps({"copy_read_bytes": 4 * n, "copy_write_bytes": 4 * n,
                          "launches": 3}), flush=True)
        return

    import paper_2311_04435_amd as sca
    import synth

    def note(msg):
        print(f"bench: {msg}", file=sys.stderr, flush=True)

    wl = synth.WORKLOADS[args.workload]
    prec = args.precision or wl.get("precision", "fp64")
    p = sca.Params.from_dict(wl["params"], precision=prec, factor=args.factor)
    L, M = p.L, p.n_max
    N, B = L * L, 2 * M
    phi0 = torch.as_tensor(synth.make_phi0(L, wl["phi0"]),
                           dtype=torch.float64).cuda()
    hy = wl["adam"]
    ctx = sca.Context()

    def run(steps, t0, phi, m, v):
        return ctx.adam_solve(p, phi, m, v, steps, lr=hy["lr"],
                              beta1=hy["beta1"], beta2=hy["beta2"],
                              eps=hy["eps"], t0=t0, final_eval=False)

    phi = phi0.clone()
    m = torch.zeros_like(phi)
    v = torch.zeros_like(phi)
    if args.warmup:
        run(args.warmup, 0, phi, m, v)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = run(args.steps, args.warmup, phi, m, v)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    steps_per_s = args.steps / dt
    note(f"{args.workload} {prec} {args.factor}: {steps_per_s:.2f} steps/s")

    # second pass of the same steps with per-kernel HIP events
    phi2, m2, v2 = phi0.clone(), torch.zeros_like(phi0), torch.zeros_like(phi0)
    if args.warmup:
        run(args.warmup, 0, phi2, m2, v2)
    ctx.profile(True)
    run(args.steps, args.warmup, phi2, m2, v2)
    prof = ctx.profile_read()
    ctx.profile(False)
    kernels = {k: {"avg_ms": ms / n, "launches": n, "total_ms": ms}
               for k, (ms, n) in prof.items()}
    dom = max(prof, key=lambda k: prof[k][0])
    roof = None
    work = kernel_work(dom, N, B)
    if work is not None:
        amount, unit, bound = work
        avg_s = prof[dom][0] / prof[dom][1] / 1e3
        if unit == "flop":
            peak = PEAK["fp32" if prec == "fp32r" else "fp64"]
            achieved = amount / avg_s / 1e12
            roof = {"bound": bound, "kernel": dom, "achieved": achieved,
                    "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                    "traffic": measured_traffic(dom, args.workload, prec,
                                                args.factor),
                    "work_per_launch": (
                        f"2 spins x (8/3) N^3 = {amount:.4g} flop in N "
                        f"dependent launches" if dom == "tridiag" else
                        f"{B} matrices x {amount / B:.4g} flop")}
        else:
            achieved = amount / avg_s / 1e9
            roof = {"bound": "hbm", "kernel": dom, "achieved": achieved,
                    "peak": HBM_PEAK, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK,
                    "traffic": measured_traffic(dom, args.workload, prec,
                                                args.factor),
                    "work_per_launch": f"{amount:.4g} bytes"}

    out = {
        "metric": METRIC, "value": steps_per_s, "unit": "steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if prec == "fp32r" else "f64",
        "data": "synthetic (seeded SplitMix64 phi0; lattice Hamiltonian generated on chip)",
        "config": {"workload": args.workload, "L": L, "N": N, "n_max": M,
                   "matrices_per_step": B, "precision": prec,
                   "factor": args.factor,
                   "U": p.U, "T": p.T, "delta": p.delta,
                   "parallelism": "single GPU, batch of (w_n, spin) matrices"},
        "roofline": roof,
        "kernels": kernels,
        "final": {"omega_tilde": res["omega_tilde"], "af_order": res["af_order"],
                  "max_abs_grad": res["max_abs_grad"],
                  "max_pivot_growth": res["max_pivot_growth"]},
    }
    if args.factor == "lu" and prec == "fp64":
        # the refined-FP32 route on the same workload, and on 32x32
        out["fp32r"] = [route_line(sca, args.workload, "fp32r", "lu",
                                   args.steps, args.warmup)]
        out["fp32r_vs_fp64"] = out["fp32r"][0]["steps_per_s"] / steps_per_s
        note(f"fp32r {out['fp32r'][0]['steps_per_s']:.2f} steps/s")
        out["c1"] = c1_line(sca)
        note(f"4x4: {out['c1']['us_per_step']:.1f} us/step")
    if not args.no_l32:
        l32 = [route_line(sca, "ionic_32x32_U4", "fp32r", "lu", 5, 1),
               route_line(sca, "ionic_32x32_U4", "fp64", "lu", 3, 1),
               route_line(sca, "ionic_32x32_U4", "fp64", "ldlt", 5, 1),
               route_line(sca, "ionic_32x32_U4", "fp64", "eigh", 20, 2)]
        out["l32"] = l32
        note("32x32 " + ", ".join(f"{r['precision']}/{r['factor']} "
                                  f"{r['steps_per_s']:.2f}" for r in l32))
        out["l48"] = [route_line(sca, "ionic_48x48", "fp32r", "lu", 3, 1),
                      route_line(sca, "ionic_48x48", "fp64", "eigh", 5, 1)]
        note("48x48 " + ", ".join(f"{r['precision']}/{r['factor']} "
                                  f"{r['steps_per_s']:.2f}" for r in out["l48"]))
    if args.factor == "lu" and prec == "fp64" and not args.no_symmetric:
        # the same workload on the symmetric route (unpivoted L D L^T)
        out["symmetric_ldlt"] = route_line(sca, args.workload, "fp64", "ldlt",
                                           max(args.steps, 10), args.warmup)
    if prec == "fp64" and not args.no_tail:
        # the same sums with the high frequencies from the moments of H
        out["tail"] = [route_line(sca, args.workload, "fp64", f,
                                  max(args.steps, 20), args.warmup, tail=True)
                       for f in ("lu", "ldlt")]
    if prec == "fp64" and not args.no_spectral:
        # one eigendecomposition per spin instead of a factorisation per
        # frequency
        out["spectral"] = [route_line(sca, args.workload, "fp64", "eigh",
                                      max(args.steps, 20), args.warmup)]
    if prec == "fp64" and not args.no_hmc:
        out["hmc"] = hmc_line(sca, args.workload)
    note("route lines done")
    if args.serving_requests > 0:
        Ls = tuple(int(x) for x in args.serving_L.split(","))
        out["serving"] = serving(sca, args.serving_requests, args.serving_steps,
                                 args.serving_nmax, Ls, args.serving_batch,
                                 factor=args.serving_factor,
                                 tail=args.serving_tail)
    if not args.no_cpu_baseline:
        note("CPU baseline (one whole 20x20 route-D step, ~1 min)")
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
