"""GPU tests of the guards of a solve and of non-finite detection.

* FP32-refined pivot growth: with the context's limit lowered
  (SCA_OPT_FP32_GROWTH_LIMIT) the evaluation calls return exactly the FP64
  route's numbers, sca_adam_solve switches to FP64 at the step whose growth
  first exceeds the limit and ends bit for bit on the trajectory that runs
  FP32 up to that step and FP64 after it, whatever check_every is, and the
  autograd split keeps FP64 factors;
* the Matsubara tail's guard: a solve thrown out of the planned range
  follows the oracle's all-frequency trajectory (the pass that saw the
  bound applies no update), independently of check_every, alone and in a
  server mix;
* a NaN in phi is reported (SCA_ENUMERIC, SCA_FLAG_NONFINITE) on every
  route: fused small, blocked FP64 LU, FP32 refined, L D L^T, spectral,
  and the tail's planning.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sca():
    import torch
    import paper_2311_04435_amd as sca
    assert torch.cuda.is_available()
    return sca


def cuda(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64).cuda()


def pd(p):
    return dict(L=p.L, t=p.t, U=p.U, delta=p.delta, T=p.T, n_max=p.n_max)


def fresh(phi0):
    import torch
    phi = phi0.clone()
    return phi, torch.zeros_like(phi), torch.zeros_like(phi)


def params32(sca, L, **kw):
    return sca.Params(L=L, U=4.0, T=0.1, n_max=64, delta=0.6,
                      precision="fp32r", **kw)


# --- FP32 pivot growth -------------------------------------------------------

@pytest.mark.parametrize("L", [12, 20])
def test_growth_fallback_grad_potential(sca, L):
    """Limit 1: every complex64 factorisation is refused and sca_grad /
    sca_potential return the FP64 route's results bit for bit."""
    import torch
    p32 = params32(sca, L)
    p64 = sca.Params(L=L, U=4.0, T=0.1, n_max=64, delta=0.6)
    phi = cuda(synth.uniform(2100 + L, L * L, -0.5, 0.5))
    ctx = sca.Context()
    g_hi, o_hi = ctx.grad(p32, phi)         # default limit: FP32 kept
    ctx.set_option(sca.SCA_OPT_FP32_GROWTH_LIMIT, 1.0)
    g32, o32 = ctx.grad(p32, phi)
    g64, o64 = ctx.grad(p64, phi)
    assert torch.equal(g32, g64) and torch.equal(o32, o64)
    assert torch.equal(ctx.potential(p32, phi), ctx.potential(p64, phi))
    # the FP32 result it replaced differs (in the last digits)
    assert not torch.equal(g_hi, g64)
    rel = float((g_hi - g64).abs().max() / g64.abs().max())
    print(f"L={L}: FP32-refined vs FP64 gradient {rel:.1e}")
    assert rel < 1e-10


def test_growth_option_validation(sca):
    from paper_2311_04435_amd import SCAError
    ctx = sca.Context()
    for bad in (0.5, float("nan"), float("inf")):
        with pytest.raises(SCAError, match="EINVAL"):
            ctx.set_option(sca.SCA_OPT_FP32_GROWTH_LIMIT, bad)
    with pytest.raises(SCAError, match="EINVAL"):
        ctx.set_option(99, 1.0)


def growth_per_step(sca, p, phi0, steps, lr):
    """Pivot growth of the evaluation behind each of the first `steps`
    updates (one update per call, resumed)."""
    ctx = sca.Context()
    phi, m, v = fresh(phi0)
    out = []
    for k in range(steps):
        r = ctx.adam_solve(p, phi, m, v, 1, lr=lr, t0=k, final_eval=False)
        out.append(r["max_pivot_growth"])
    return np.array(out)


def test_growth_switch_mid_run(sca):
    """The limit is set between the growth before step k* and at k*: the
    solve runs FP32 up to k*, the pass at k* applies no update, and the rest
    runs in FP64 -- bitwise the concatenation of an FP32 run of k* steps and
    an FP64 run resumed from it, for any check_every."""
    import torch
    L, steps, lr = 12, 24, 0.05
    p32 = params32(sca, L)
    p64 = sca.Params(L=L, U=4.0, T=0.1, n_max=64, delta=0.6)
    phi0 = cuda(synth.uniform(2200, L * L, -0.5, 0.5))
    gr = growth_per_step(sca, p32, phi0, steps, lr)
    run_max = np.maximum.accumulate(gr)
    ks = [k for k in range(1, steps - 2) if gr[k] > run_max[k - 1]]
    print("growth per step:", np.array2string(gr, precision=4))
    if not ks:
        pytest.skip("growth never sets a new maximum after step 0")
    k = ks[0]
    limit = 0.5 * (run_max[k - 1] + gr[k])
    # expected: FP32 for k updates, then FP64
    ctx = sca.Context()
    phi_e, m_e, v_e = fresh(phi0)
    ctx.adam_solve(p32, phi_e, m_e, v_e, k, lr=lr, final_eval=False)
    res_e = ctx.adam_solve(p64, phi_e, m_e, v_e, steps - k, lr=lr, t0=k)
    for ce in (0, 1, 5):
        ctx = sca.Context()
        ctx.set_option(sca.SCA_OPT_FP32_GROWTH_LIMIT, limit)
        phi, m, v = fresh(phi0)
        res = ctx.adam_solve(p32, phi, m, v, steps, lr=lr, check_every=ce)
        assert res["flags"] & sca.SCA_FLAG_PIVOT_GROWTH, ce
        assert res["steps_done"] == steps, ce
        assert torch.equal(phi, phi_e) and torch.equal(m, m_e), ce
        assert torch.equal(v, v_e), ce
        assert res["omega_tilde"] == res_e["omega_tilde"], ce
        assert res["max_pivot_growth"] >= gr[k]
    print(f"switch at step {k} (limit {limit:.4f}): bitwise for "
          "check_every 0, 1, 5")


def test_growth_fallback_from_start_matches_fp64(sca):
    import torch
    L = 20
    p32 = params32(sca, L)
    p64 = sca.Params(L=L, U=4.0, T=0.1, n_max=64, delta=0.6)
    phi0 = cuda(synth.uniform(2300, L * L, -0.5, 0.5))
    ctx = sca.Context()
    ctx.set_option(sca.SCA_OPT_FP32_GROWTH_LIMIT, 1.0)
    phi, m, v = fresh(phi0)
    res = ctx.adam_solve(p32, phi, m, v, 12, lr=0.02)
    phi_e, m_e, v_e = fresh(phi0)
    res_e = ctx.adam_solve(p64, phi_e, m_e, v_e, 12, lr=0.02)
    assert res["flags"] & sca.SCA_FLAG_PIVOT_GROWTH
    assert torch.equal(phi, phi_e) and torch.equal(v, v_e)
    assert res["omega_tilde"] == res_e["omega_tilde"]


def test_growth_fallback_autograd_split(sca):
    """sca_factorize under a lowered limit keeps FP64 factors; the backward
    then gives the FP64 gradient bit for bit."""
    import torch
    L = 12
    p32 = params32(sca, L)
    p64 = sca.Params(L=L, U=4.0, T=0.1, n_max=64, delta=0.6)
    phi = cuda(synth.uniform(2400, L * L, -0.5, 0.5))
    ctx = sca.Context()
    assert ctx.factor_bytes(p32) >= ctx.factor_bytes(p64)
    ctx.set_option(sca.SCA_OPT_FP32_GROWTH_LIMIT, 1.0)
    buf = torch.empty(ctx.factor_bytes(p32), dtype=torch.uint8, device="cuda")
    o2 = ctx.factorize(p32, phi, buf)
    g = ctx.grad_from_factors(p32, phi, buf)
    g64, o64 = ctx.grad(p64, phi)
    assert torch.equal(o2, o64) and torch.equal(g, g64)


# --- the tail's guard ----------------------------------------------------------

def tail_case(sca, L):
    p = sca.Params(L=L, U=0.5, T=0.1, n_max=256, tail=True)
    phi0 = synth.uniform(1800 + L, L * L, -0.1, 0.1)
    return p, phi0


@pytest.mark.parametrize("L", [8, 12])
def test_tail_guard_trajectory_matches_oracle(sca, L):
    """lr = 8 throws phi beyond the bound the split was planned for: the pass
    that sees it applies no update and the solve continues with every
    frequency, so the trajectory is the oracle's (every frequency, Eq. (7))
    to the FP64 bar, and the same bit for bit for any check_every."""
    import torch
    p, phi0 = tail_case(sca, L)
    steps, lr = 6, 8.0
    ref, info = oracle.adam_solve(pd(p), phi0, steps, lr=lr)
    first = None
    for ce in (0, 1, 4):
        ctx = sca.Context()
        phi, m, v = fresh(cuda(phi0))
        res = ctx.adam_solve(p, phi, m, v, steps, lr=lr, check_every=ce)
        assert res["flags"] & sca.SCA_FLAG_TAIL_RANGE, ce
        assert res["steps_done"] == steps
        e = np.max(np.abs(phi.cpu().numpy() - ref)) / np.max(np.abs(ref))
        e_om = abs(res["omega_tilde"] - info["omega_tilde"]) / abs(info["omega_tilde"])
        print(f"L={L} check_every={ce}: phi err {e:.1e} Omega~ err {e_om:.1e}")
        assert e < 1e-10 and e_om < 1e-10
        if first is None:
            first = (phi, m, v)
        else:
            assert torch.equal(phi, first[0]) and torch.equal(v, first[2])


def test_tail_guard_served_alone_vs_mix_and_oracle(sca):
    """A tail request whose guard fires, served together with others of its
    shape: bitwise its own sca_adam_solve, and the oracle's trajectory."""
    import torch
    from paper_2311_04435_amd.serve import Server
    p, phi0 = tail_case(sca, 12)
    steps, lr = 6, 8.0
    others = []
    for k in range(3):
        r = synth.uniform(2500 + k, 3, 0.0, 1.0)
        q = sca.Params(L=12, U=0.5, T=0.1, n_max=256, tail=bool(k % 2),
                       delta=0.5 * r[0])
        others.append((q, cuda(synth.uniform(2510 + k, 144, -0.3, 0.3)),
                       5 + k, 0.02))
    reqs = [(p, cuda(phi0), steps, lr)] + others
    with Server(max_batch=4) as srv:
        tickets = [srv.submit(q, x, n, lr=l) for q, x, n, l in reqs]
        done = srv.drain(tickets)
    for (q, x, n, l), t in zip(reqs, tickets):
        phi_s, m_s, v_s, res_s, _ = done[t]
        phi_a, m_a, v_a, res_a = sca.adam_solve(q, x, n, lr=l)
        assert torch.equal(phi_s, phi_a) and torch.equal(v_s, v_a)
        assert res_s["flags"] == res_a["flags"]
        assert res_s["omega_tilde"] == res_a["omega_tilde"]
    phi_s, _, _, res_s, _ = done[tickets[0]]
    assert res_s["flags"] & sca.SCA_FLAG_TAIL_RANGE
    ref, info = oracle.adam_solve(pd(p), phi0, steps, lr=lr)
    e = np.max(np.abs(phi_s.cpu().numpy() - ref)) / np.max(np.abs(ref))
    print(f"served tail request after its guard fired: phi err {e:.1e}")
    assert e < 1e-10


# --- non-finite values ----------------------------------------------------------

ROUTES = [(4, "fp64", "lu", False), (10, "fp64", "lu", False),
          (20, "fp64", "lu", False), (10, "fp32r", "lu", False),
          (20, "fp32r", "lu", False), (10, "fp64", "ldlt", False),
          (20, "fp64", "ldlt", False), (10, "fp64", "eigh", False),
          (20, "fp64", "eigh", False), (10, "fp64", "lu", True),
          (20, "fp64", "ldlt", True)]


@pytest.mark.parametrize("L,prec,factor,tail", ROUTES)
def test_nan_phi_reported(sca, L, prec, factor, tail):
    from paper_2311_04435_amd import SCAError
    p = sca.Params(L=L, U=4.0, T=0.1, n_max=32, delta=0.4, precision=prec,
                   factor=factor, tail=tail)
    x = synth.uniform(2600 + L, L * L, -0.5, 0.5)
    x[L + 1] = np.nan
    phi = cuda(x)
    with pytest.raises(SCAError, match="ENUMERIC"):
        sca.grad(p, phi)
    with pytest.raises(SCAError, match="ENUMERIC"):
        sca.potential(p, phi)
    ctx = sca.Context()
    ph, m, v = fresh(phi)
    with pytest.raises(SCAError, match="ENUMERIC"):
        ctx.adam_solve(p, ph, m, v, 3)
    # the same context still works on a finite field
    g, o2 = ctx.grad(p, cuda(np.nan_to_num(x)))
    assert bool(g.isfinite().all()) and bool(o2.isfinite().all())


def test_nan_in_adam_result_flags(sca):
    """The result struct of a failing solve carries SCA_FLAG_NONFINITE (read
    through the raw C call, which fills it before returning)."""
    import ctypes as C
    from paper_2311_04435_amd import _lib
    p = sca.Params(L=10, U=4.0, T=0.1, n_max=32)
    x = synth.uniform(2700, 100, -0.5, 0.5)
    x[3] = np.nan
    phi, m, v = fresh(cuda(x))
    ctx = sca.Context()
    opts = _lib.AdamOpts(0.01, 0.9, 0.999, 1e-8, 0.0, 3, 0, 0, 0)
    res = _lib.Result()
    st = _lib.lib.sca_adam_solve(ctx._h, C.byref(p.c()), C.byref(opts),
                                 phi.data_ptr(), m.data_ptr(), v.data_ptr(),
                                 C.byref(res))
    assert st == _lib.SCA_ENUMERIC
    assert res.flags & sca.SCA_FLAG_NONFINITE
