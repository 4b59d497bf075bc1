"""SCA+ADAM on MI355X: the Python face of libsca.so (gfx950 HIP kernels).

Semiclassical approximation of the half-filled ionic Hubbard model (Sec. II
of the paper, Eqs. (1), (7), (8)): the potential Omega(phi), its gradient,
its ADAM minimisation and the density of states, evaluated by batched
complex LU factorisations over all Matsubara frequencies and both spins.

Every number here is computed by the HIP library; this module only moves
torch tensors' device pointers and the caller's stream across the C ABI
(include/sca.h).  Arrays are float64 CUDA (HIP) tensors.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import threading
from typing import Optional

import torch

from . import _lib
from ._lib import (SCAError, SCA_FP64, SCA_FP32_REFINED,  # noqa: F401
                   SCA_FLAG_NONFINITE, SCA_FLAG_PIVOT_GROWTH,
                   SCA_FLAG_CONVERGED, SCA_FLAG_TAIL_RANGE,
                   SCA_OPT_FP32_GROWTH_LIMIT)

PRECISIONS = {"fp64": SCA_FP64, "fp32r": SCA_FP32_REFINED}
FACTORS = {"lu": _lib.SCA_FACTOR_LU, "ldlt": _lib.SCA_FACTOR_LDLT,
           "eigh": _lib.SCA_FACTOR_EIGH}


@dataclasses.dataclass(frozen=True)
class Params:
    """One SCA problem: L x L lattice (L even), hopping t, on-site U > 0,
    ionic amplitude delta (site potential +-delta/2), temperature T > 0,
    n_max Matsubara frequencies per sign, precision 'fp64' | 'fp32r',
    factorisation 'lu' (pivoted, default) | 'ldlt' (symmetric, unpivoted,
    FP64) | 'eigh' (spectral route, FP64: one eigendecomposition of H per
    spin, every frequency from the spectrum), an optional extra site potential `onsite` (float64 CUDA tensor
    of N) and `tail`: factorise only the Matsubara frequencies below about
    4x a bound on the spectral radius of H and take the rest from the
    moments of H (the same sums, evaluated by a series whose truncation
    error the library keeps below 9^-15 of each term's scale)."""
    L: int
    U: float
    T: float
    n_max: int
    t: float = 1.0
    delta: float = 0.0
    precision: str = "fp64"
    onsite: Optional[torch.Tensor] = None
    factor: str = "lu"
    tail: bool = False

    @property
    def N(self) -> int:
        return self.L * self.L

    def c(self) -> _lib.Params:
        if self.precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {list(PRECISIONS)}")
        if self.factor not in FACTORS:
            raise ValueError(f"factor must be one of {list(FACTORS)}")
        ons = None
        if self.onsite is not None:
            ons = _dev(self.onsite, self.N, "onsite").data_ptr()
        return _lib.Params(self.L, self.n_max, PRECISIONS[self.precision],
                           FACTORS[self.factor], self.t, self.U, self.delta,
                           self.T, ons,
                           _lib.SCA_TAIL_MOMENTS if self.tail else _lib.SCA_TAIL_NONE,
                           0)

    @classmethod
    def from_dict(cls, d: dict, precision: str = "fp64", **kw) -> "Params":
        return cls(L=d["L"], U=d["U"], T=d["T"], n_max=d["n_max"],
                   t=d.get("t", 1.0), delta=d.get("delta", 0.0),
                   precision=precision, **kw)


def _dev(x, n: Optional[int], name: str) -> torch.Tensor:
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if x.dtype != torch.float64 or not x.is_contiguous():
        raise TypeError(f"{name} must be contiguous float64")
    if n is not None and x.numel() != n:
        raise ValueError(f"{name} has {x.numel()} elements, expected {n}")
    return x


class Context:
    """A library context bound to one device and one HIP stream."""

    def __init__(self, device: Optional[int] = None,
                 stream: Optional[torch.cuda.Stream] = None,
                 hbm_budget_bytes: int = 0):
        if device is None:
            device = torch.cuda.current_device()
        self.device = device
        self.stream = stream if stream is not None else \
            torch.cuda.current_stream(device)
        h = C.c_void_p()
        _lib.check(_lib.lib.sca_create(device, C.c_void_p(self.stream.cuda_stream),
                                       hbm_budget_bytes, C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib.lib.sca_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _empty(self, *shape):
        return torch.empty(*shape, dtype=torch.float64, device=self.device)

    # --- the calls of include/sca.h -----------------------------------
    def potential(self, p: Params, phi: torch.Tensor):
        o2 = self._empty(2)
        _lib.check(_lib.lib.sca_potential(self._h, C.byref(p.c()),
                                          _dev(phi, p.N, "phi").data_ptr(),
                                          o2.data_ptr()))
        return o2

    def grad(self, p: Params, phi: torch.Tensor):
        g = self._empty(p.N)
        o2 = self._empty(2)
        _lib.check(_lib.lib.sca_grad(self._h, C.byref(p.c()),
                                     _dev(phi, p.N, "phi").data_ptr(),
                                     g.data_ptr(), o2.data_ptr()))
        return g, o2

    def adam_solve(self, p: Params, phi: torch.Tensor, m: torch.Tensor,
                   v: torch.Tensor, n_steps: int, lr: float = 0.01,
                   beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
                   grad_tol: float = 0.0, check_every: int = 0, t0: int = 0,
                   final_eval: bool = True):
        """In-place ADAM on phi, m, v; returns the sca_result as a dict.
        final_eval=False skips the evaluation at the returned phi."""
        flags = 0 if final_eval else _lib.SCA_ADAM_NO_FINAL_EVAL
        opts = _lib.AdamOpts(lr, beta1, beta2, eps, grad_tol, n_steps,
                             check_every, t0, flags)
        res = _lib.Result()
        _lib.check(_lib.lib.sca_adam_solve(
            self._h, C.byref(p.c()), C.byref(opts),
            _dev(phi, p.N, "phi").data_ptr(), _dev(m, p.N, "m").data_ptr(),
            _dev(v, p.N, "v").data_ptr(), C.byref(res)))
        return {f: getattr(res, f) for f, _ in _lib.Result._fields_}

    def hmc(self, p: Params, phi: torch.Tensor, momenta: torch.Tensor,
            uniforms, eps: float, n_leap: int):
        """Hybrid Monte Carlo chain in place on phi: trajectory t starts with
        momentum momenta[t] (float64 CUDA [n_traj, N]) and is accepted if
        uniforms[t] < exp(-dH).  Returns (accepted, h_old, h_new) as NumPy
        arrays."""
        import numpy as np
        n_traj = 0 if momenta is None else momenta.shape[0]
        if n_traj:
            _dev(momenta.reshape(-1), n_traj * p.N, "momenta")
        u = np.ascontiguousarray(uniforms, dtype=np.float64)
        if u.shape != (n_traj,):
            raise ValueError("uniforms must hold one draw per trajectory")
        acc = np.zeros(n_traj, dtype=np.int32)
        h0 = np.zeros(n_traj)
        h1 = np.zeros(n_traj)
        opts = _lib.HmcOpts(eps, n_leap, n_traj)
        dbl = C.POINTER(C.c_double)
        _lib.check(_lib.lib.sca_hmc(
            self._h, C.byref(p.c()), C.byref(opts),
            _dev(phi, p.N, "phi").data_ptr(),
            momenta.data_ptr() if n_traj else None,
            u.ctypes.data_as(dbl), acc.ctypes.data_as(C.POINTER(C.c_int32)),
            h0.ctypes.data_as(dbl), h1.ctypes.data_as(dbl)))
        return acc, h0, h1

    def dos(self, p: Params, phi: torch.Tensor, w: torch.Tensor, eta: float):
        w = _dev(w, None, "w")
        rho = self._empty(2, w.numel())
        _lib.check(_lib.lib.sca_dos(self._h, C.byref(p.c()),
                                    _dev(phi, p.N, "phi").data_ptr(),
                                    w.data_ptr(), w.numel(), eta,
                                    rho.data_ptr()))
        return rho

    def shifted_terms(self, p: Params, phi: torch.Tensor, z: torch.Tensor):
        """z: complex128 or [n_z, 2] float64 CUDA tensor of shifts.
        Returns (logabsdet [2, n_z], diag [2, n_z, N] complex128)."""
        if z.is_complex():
            z = torch.view_as_real(z.to(torch.complex128)).contiguous()
        z = _dev(z, None, "z")
        n_z = z.numel() // 2
        lad = self._empty(2, n_z)
        dg = self._empty(2, n_z, p.N, 2)
        _lib.check(_lib.lib.sca_shifted_terms(
            self._h, C.byref(p.c()), _dev(phi, p.N, "phi").data_ptr(),
            z.data_ptr(), n_z, lad.data_ptr(), dg.data_ptr()))
        return lad, torch.view_as_complex(dg)

    def set_option(self, option: int, value: float):
        """sca_set_option, e.g. (SCA_OPT_FP32_GROWTH_LIMIT, 1e3)."""
        _lib.check(_lib.lib.sca_set_option(self._h, option, float(value)))

    def tail_split(self, p: Params, phi: torch.Tensor) -> int:
        """Matsubara frequencies per spin the library factorises for p at
        phi (n_max without the tail)."""
        n = C.c_int32()
        _lib.check(_lib.lib.sca_tail_split(self._h, C.byref(p.c()),
                                           _dev(phi, p.N, "phi").data_ptr(),
                                           C.byref(n)))
        return int(n.value)

    def profile(self, enable: bool = True):
        """Start (reset) or stop per-kernel HIP-event timing."""
        _lib.check(_lib.lib.sca_profile(self._h, 1 if enable else 0))

    def profile_read(self) -> dict:
        """{kernel class: (total ms, launches)} since profile(True)."""
        ms = (C.c_double * _lib.PROFILE_SLOTS)()
        n = (C.c_int64 * _lib.PROFILE_SLOTS)()
        _lib.check(_lib.lib.sca_profile_read(self._h, ms, n))
        return {k: (ms[i], n[i]) for i, k in enumerate(_lib.KERNEL_CLASSES)
                if n[i]}

    def factor_bytes(self, p: Params) -> int:
        return int(_lib.lib.sca_factor_bytes(C.byref(p.c())))

    def factorize(self, p: Params, phi: torch.Tensor, factors: torch.Tensor):
        o2 = self._empty(2)
        _lib.check(_lib.lib.sca_factorize(
            self._h, C.byref(p.c()), _dev(phi, p.N, "phi").data_ptr(),
            C.c_void_p(factors.data_ptr()), o2.data_ptr()))
        return o2

    def grad_from_factors(self, p: Params, phi: torch.Tensor,
                          factors: torch.Tensor):
        g = self._empty(p.N)
        _lib.check(_lib.lib.sca_grad_from_factors(
            self._h, C.byref(p.c()), _dev(phi, p.N, "phi").data_ptr(),
            C.c_void_p(factors.data_ptr()), g.data_ptr()))
        return g


def footprint_bytes(p: Params) -> int:
    return int(_lib.lib.sca_footprint_bytes(C.byref(p.c())))


_tls = threading.local()


def default_context() -> Context:
    """The calling thread's context for the current device and stream."""
    key = (torch.cuda.current_device(), torch.cuda.current_stream().cuda_stream)
    cache = getattr(_tls, "ctx", None)
    if cache is None:
        cache = _tls.ctx = {}
    if key not in cache:
        cache[key] = Context()
    return cache[key]


def potential(p: Params, phi: torch.Tensor):
    """(Omega, Omega~) at phi as a float64 CUDA tensor of 2."""
    return default_context().potential(p, phi)


def grad(p: Params, phi: torch.Tensor):
    """(dOmega/dphi [N], (Omega, Omega~))."""
    return default_context().grad(p, phi)


def adam_solve(p: Params, phi0: torch.Tensor, n_steps: int, **kw):
    """ADAM from phi0 (not modified); returns (phi, m, v, result dict)."""
    phi = phi0.clone()
    m = torch.zeros_like(phi)
    v = torch.zeros_like(phi)
    res = default_context().adam_solve(p, phi, m, v, n_steps, **kw)
    return phi, m, v, res


def tail_split(p: Params, phi: torch.Tensor) -> int:
    """Number of Matsubara frequencies the library factorises for p at phi
    (sca_tail_split: n_max, or the SCA_TAIL_MOMENTS split)."""
    return default_context().tail_split(p, phi)


def hmc(p: Params, phi0: torch.Tensor, momenta: torch.Tensor, uniforms,
        eps: float, n_leap: int):
    """HMC chain from phi0 (not modified); returns (phi, accepted, h_old,
    h_new)."""
    phi = phi0.clone()
    acc, h0, h1 = default_context().hmc(p, phi, momenta, uniforms, eps, n_leap)
    return phi, acc, h0, h1


def dos(p: Params, phi: torch.Tensor, w: torch.Tensor, eta: float = 0.05):
    """rho[2, n_w] per spin (up first)."""
    return default_context().dos(p, phi, w, eta)


def shifted_terms(p: Params, phi: torch.Tensor, z: torch.Tensor):
    return default_context().shifted_terms(p, phi, z)
