"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module holds no arithmetic of the SCA method itself: it only draws
seeded random numbers and names the workload shapes.  Both sides receive the
same initial field phi0 from here as an input array.

Generator: SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014; the finalizer constants are Vigna's
published ones).  Output k (k = 0, 1, ...) of seed s is the mix of
s + (k+1) * 0x9E3779B97F4A7C15 (mod 2**64); the top 53 bits give a double in
[0, 1).

Workloads: the lattice sizes, couplings, Matsubara cut-offs and ADAM settings
of the paper's experiments (Sec. III: 20x20 lattices, U/t up to 6, T/t in
[0.1, 1.3], an ionic potential up to Delta/t ~ 1.2) plus the small and large
lattices used to bracket them.  t = 1 sets the energy unit (Sec. II).
"""
from __future__ import annotations

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, count: int) -> np.ndarray:
    """First `count` SplitMix64 outputs for `seed`, as uint64."""
    k = np.arange(1, count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed % (1 << 64)) + k * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(seed: int, count: int, lo: float, hi: float) -> np.ndarray:
    """`count` doubles uniform in [lo, hi) from SplitMix64 (top 53 bits)."""
    u = (splitmix64(seed, count) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return lo + (hi - lo) * u


def normal(seed: int, count: int) -> np.ndarray:
    """`count` standard normal doubles (Box-Muller on pairs of uniforms from
    `uniform`; the first uniform of each pair is moved into (0, 1])."""
    m = (count + 1) // 2
    u = uniform(seed, 2 * m, 0.0, 1.0)
    u1, u2 = 1.0 - u[0::2], u[1::2]
    r = np.sqrt(-2.0 * np.log(u1))
    z = np.empty(2 * m)
    z[0::2] = r * np.cos(2.0 * np.pi * u2)
    z[1::2] = r * np.sin(2.0 * np.pi * u2)
    return z[:count]


def rademacher(seed: int, count: int) -> np.ndarray:
    """`count` independent +-1.0 values (bit 63 of each SplitMix64 output)."""
    return np.where(splitmix64(seed, count) >> np.uint64(63), -1.0, 1.0)


def sample_indices(seed: int, n: int, k: int) -> np.ndarray:
    """k distinct indices in [0, n): the first k of a seeded permutation."""
    keys = splitmix64(seed, n)
    return np.argsort(keys, kind="stable")[:k]


def stagger(L: int) -> np.ndarray:
    """(-1)^(x+y) for site i = x + L*y, as float64 (a lattice sign pattern)."""
    x = np.arange(L * L) % L
    y = np.arange(L * L) // L
    return np.where((x + y) % 2 == 0, 1.0, -1.0)


def phi0_uniform(L: int, seed: int, amp: float) -> np.ndarray:
    """phi_i i.i.d. uniform in [-amp, amp)."""
    return uniform(seed, L * L, -amp, amp)


def phi0_staggered(L: int, seed: int, m: float, noise: float) -> np.ndarray:
    """m * (-1)^(x+y) plus i.i.d. uniform noise in [-noise, noise)."""
    return m * stagger(L) + uniform(seed, L * L, -noise, noise)


# Named workloads.  `params` are the physical parameters of one SCA problem;
# `adam` the optimizer settings; `phi0` the recipe for the starting field.
WORKLOADS = {
    # 4x4 Hubbard lattice, FP64, 512 executed matrices of 16x16 per step.
    "hubbard_4x4": dict(
        params=dict(L=4, t=1.0, U=4.0, delta=0.0, T=0.1, n_max=256),
        precision="fp64", steps=500,
        adam=dict(lr=0.01, beta1=0.9, beta2=0.999, eps=1e-8),
        phi0=dict(kind="uniform", amp=0.1, seed=0)),
    # 20x20 Hubbard lattice (the paper's lattice), 1024 matrices of 400x400.
    "hubbard_20x20_T0.1": dict(
        params=dict(L=20, t=1.0, U=6.0, delta=0.0, T=0.1, n_max=512),
        precision="fp64", steps=2000,
        adam=dict(lr=0.01, beta1=0.9, beta2=0.999, eps=1e-8),
        phi0=dict(kind="uniform", amp=0.5, seed=0)),
    "hubbard_20x20_T0.6": dict(
        params=dict(L=20, t=1.0, U=6.0, delta=0.0, T=0.6, n_max=512),
        precision="fp64", steps=2000,
        adam=dict(lr=0.01, beta1=0.9, beta2=0.999, eps=1e-8),
        phi0=dict(kind="uniform", amp=0.5, seed=1)),
    # 32x32 ionic Hubbard lattice, 512 matrices of 1024x1024.
    "ionic_32x32_U4": dict(
        params=dict(L=32, t=1.0, U=4.0, delta=1.0, T=0.1, n_max=256),
        precision="fp32r", steps=100,
        adam=dict(lr=0.01, beta1=0.9, beta2=0.999, eps=1e-8),
        phi0=dict(kind="uniform", amp=0.5, seed=0)),
    # 48x48 ionic Hubbard lattice, 256 matrices of 2304x2304.
    "ionic_48x48": dict(
        params=dict(L=48, t=1.0, U=5.0, delta=0.5, T=0.1, n_max=128),
        precision="fp32r", steps=1000,
        adam=dict(lr=0.01, beta1=0.9, beta2=0.999, eps=1e-8),
        phi0=dict(kind="staggered", m=1.0, noise=0.1, seed=0)),
}


def make_phi0(L: int, recipe: dict) -> np.ndarray:
    if recipe["kind"] == "uniform":
        return phi0_uniform(L, recipe["seed"], recipe["amp"])
    if recipe["kind"] == "staggered":
        return phi0_staggered(L, recipe["seed"], recipe["m"], recipe["noise"])
    raise ValueError(f"unknown phi0 recipe {recipe['kind']!r}")


def serving_stream(n_requests: int = 256, seed: int = 0, n_max: int = 256,
                   Ls=(8, 12, 16, 20, 24, 32)):
    """A stream of SCA solve requests with mixed lattice sizes and couplings.

    L uniform over Ls (default {8,12,16,20,24,32}), U/t ~ U[2,8],
    Delta/t ~ U[0,2], T/t ~ U[0.05,0.6]; phi0 ~ U[-0.5,0.5] seeded by the
    request id.
    """
    Ls = np.asarray(Ls)
    r = uniform(seed, 4 * n_requests, 0.0, 1.0).reshape(n_requests, 4)
    out = []
    for k in range(n_requests):
        L = int(Ls[min(int(r[k, 0] * len(Ls)), len(Ls) - 1)])
        out.append(dict(id=k, params=dict(
            L=L, t=1.0, U=2.0 + 6.0 * r[k, 1], delta=2.0 * r[k, 2],
            T=0.05 + 0.55 * r[k, 3], n_max=n_max),
            phi0=dict(kind="uniform", amp=0.5, seed=1000 + k)))
    return out


def poisson_arrivals(seed: int, count: int, rate: float) -> np.ndarray:
    """Arrival times (from 0) of a Poisson process of the given rate:
    cumulative sums of exponential gaps -ln(1 - u) / rate."""
    u = uniform(seed, count, 0.0, 1.0)
    return np.cumsum(-np.log1p(-u) / rate) - (-np.log1p(-u[0]) / rate)
