"""Cases of the C ABI (include/sca.h) on the emulated library: every route of
the library, from sca_create to the server, run on the CPU against the
oracle (tests/test_kernel_emu.py starts one process per case, with the
AddressSanitizer runtime preloaded).

    python tests/emu/lib_cases.py <libsca_emu.so> <case>

prints one JSON line {"case": ..., "errors": {...}, "bitwise": {...},
"digest": ...} and exits 0, or raises; the digest is a SHA-256 of every
output the case read back.  EMU_ORDER in the environment sets the
emulator's scheduling order (0 forward, 1 reverse, 2 random).  The ctypes
signatures are the product binding's own (paper_2311_04435_amd/_lib.py,
executed with its library path replaced).
"""
import ctypes as C
import hashlib
import json
import os
import sys
import types

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle  # noqa: E402


def bind(path):
    src_path = os.path.join(ROOT, "paper_2311_04435_amd", "_lib.py")
    with open(src_path) as f:
        src = f.read()
    marker = "\nlib = _load()\n"
    assert src.count(marker) == 1
    mod = types.ModuleType("sca_lib_emu")
    mod.__file__ = src_path
    exec(compile(src.replace(marker, "\nlib = None\n"), src_path, "exec"),
         mod.__dict__)
    mod.LIB_PATH = path
    mod.lib = mod._load()
    emu = C.CDLL(path)
    emu.emu_device_alloc.restype = C.c_void_p
    emu.emu_device_alloc.argtypes = [C.c_size_t]
    emu.emu_device_free.argtypes = [C.c_void_p]
    return mod, emu


S, E = bind(sys.argv[1])
E.emu_set_order(int(os.environ.get("EMU_ORDER", "0")))
DIGEST = hashlib.sha256()


def dev(a, dtype=np.float64):
    a = np.ascontiguousarray(a, dtype=dtype)
    p = E.emu_device_alloc(max(a.nbytes, 1))
    if a.nbytes:
        C.memmove(p, a.ctypes.data, a.nbytes)
    return p


def zeros(n, dtype=np.float64):
    return dev(np.zeros(n, dtype))


def host(p, n, dtype=np.float64):
    out = np.empty(n, dtype)
    C.memmove(out.ctypes.data, p, out.nbytes)
    DIGEST.update(out.tobytes())
    return out


def params(L, M, precision=0, factor=0, tail=0, U=4.0, delta=0.8, T=0.1,
           t=1.0):
    return S.Params(L=L, n_max=M, precision=precision, factor=factor, t=t,
                    U=U, delta=delta, T=T, onsite=None, tail=tail,
                    reserved=0)


def pd(p):
    return dict(L=p.L, t=p.t, U=p.U, delta=p.delta, T=p.T, n_max=p.n_max)


def field(L, seed):
    rng = np.random.default_rng(seed)
    sg = oracle.stagger_signs(L)
    return 0.6 * sg + rng.uniform(-0.3, 0.3, L * L)


def context():
    ctx = C.c_void_p()
    S.check(S.lib.sca_create(0, None, 0, C.byref(ctx)))
    return ctx


def rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) /
                 max(np.max(np.abs(np.asarray(b))), 1e-300))


def grad_case(p, seed=1):
    ctx = context()
    N = p.L * p.L
    phi = field(p.L, seed)
    g, o2 = zeros(N), zeros(2)
    S.check(S.lib.sca_grad(ctx, C.byref(p), dev(phi), g, o2))
    gr = oracle.grad(pd(p), phi)
    om = oracle.omega_tilde(pd(p), phi)
    o = host(o2, 2)
    return {"grad": rel(host(g, N), gr), "omega_tilde": abs(o[1] - om) / abs(om)}


def case_adam():
    p = params(4, 8)
    ctx = context()
    N = 16
    phi0 = field(4, 3)
    ph, m, v = dev(phi0), zeros(N), zeros(N)
    o = S.AdamOpts(lr=0.01, beta1=0.9, beta2=0.999, eps=1e-8, grad_tol=0.0,
                   n_steps=5, check_every=2, t0=0, flags=0)
    res = S.Result()
    S.check(S.lib.sca_adam_solve(ctx, C.byref(p), C.byref(o), ph, m, v,
                                 C.byref(res)))
    ref, info = oracle.adam_solve(pd(p), phi0, 5)
    return {"phi": rel(host(ph, N), ref),
            "omega_tilde": abs(res.omega_tilde - info["omega_tilde"]) /
            abs(info["omega_tilde"]),
            "m": rel(host(m, N), info["m"]), "v": rel(host(v, N), info["v"])}, \
        {"steps_done": res.steps_done == 5}


def case_dos():
    p = params(4, 8)
    ctx = context()
    phi = field(4, 5)
    w = np.linspace(-4.0, 4.0, 11)
    rho = zeros(22)
    S.check(S.lib.sca_dos(ctx, C.byref(p), dev(phi), dev(w), 11, 0.1, rho))
    ref = oracle.dos(pd(p), phi, w, 0.1)
    return {"dos": rel(host(rho, 22).reshape(2, 11), ref)}, {}


def case_factors():
    p = params(10, 4)
    ctx = context()
    N = 100
    phi = dev(field(10, 7))
    g1, o1 = zeros(N), zeros(2)
    S.check(S.lib.sca_grad(ctx, C.byref(p), phi, g1, o1))
    nb = S.lib.sca_factor_bytes(C.byref(p))
    fac = E.emu_device_alloc(nb)
    g2, o2 = zeros(N), zeros(2)
    S.check(S.lib.sca_factorize(ctx, C.byref(p), phi, fac, o2))
    S.check(S.lib.sca_grad_from_factors(ctx, C.byref(p), phi, fac, g2))
    return {"grad": rel(host(g2, N), host(g1, N))}, \
        {"omega": bool(np.array_equal(host(o1, 2), host(o2, 2))),
         "grad": bool(np.array_equal(host(g1, N), host(g2, N)))}


def case_noalloc():
    p = params(4, 16)
    ctx = context()
    phi = dev(field(4, 9))
    g1, o1, g2, o2 = zeros(16), zeros(2), zeros(16), zeros(2)
    S.check(S.lib.sca_grad(ctx, C.byref(p), phi, g1, o1))
    S.check(S.lib.sca_grad_noalloc(ctx, C.byref(p), phi, g2, o2))
    return {}, {"grad": bool(np.array_equal(host(g1, 16), host(g2, 16))),
                "omega": bool(np.array_equal(host(o1, 2), host(o2, 2)))}


def case_server():
    p = params(4, 8)
    N = 16
    o = S.AdamOpts(lr=0.01, beta1=0.9, beta2=0.999, eps=1e-8, grad_tol=0.0,
                   n_steps=4, check_every=0, t0=0, flags=0)
    alone = []
    ctx = context()
    for seed in (11, 12):
        ph, m, v = dev(field(4, seed)), zeros(N), zeros(N)
        res = S.Result()
        S.check(S.lib.sca_adam_solve(ctx, C.byref(p), C.byref(o), ph, m, v,
                                     C.byref(res)))
        alone.append(host(ph, N))
    srv = C.c_void_p()
    S.check(S.lib.sca_server_create(0, 0, 8, C.byref(srv)))
    tickets, bufs = [], []
    for seed in (11, 12):
        ph, m, v = dev(field(4, seed)), zeros(N), zeros(N)
        t = C.c_int64()
        S.check(S.lib.sca_server_submit(srv, C.byref(p), C.byref(o), ph, m, v,
                                        C.byref(t)))
        tickets.append(t.value)
        bufs.append(ph)
    done = [0, 0]
    for _ in range(1000):
        a, q = C.c_int32(), C.c_int32()
        S.check(S.lib.sca_server_progress(srv, 0.0, C.byref(a), C.byref(q)))
        for k, t in enumerate(tickets):
            if not done[k]:
                d, res, td = C.c_int32(), S.Result(), C.c_double()
                S.check(S.lib.sca_server_poll(srv, t, C.byref(d), C.byref(res),
                                              C.byref(td)))
                done[k] = d.value
        if all(done):
            break
    S.lib.sca_server_destroy(srv)
    return {}, {"done": all(done),
                "phi0": bool(np.array_equal(host(bufs[0], N), alone[0])),
                "phi1": bool(np.array_equal(host(bufs[1], N), alone[1]))}


def case_hmc():
    p = params(4, 8)
    ctx = context()
    N = 16
    phi0 = field(4, 13)
    rng = np.random.default_rng(14)
    mom = rng.standard_normal((2, N))
    uni = np.array([0.3, 0.7])
    ph = dev(phi0)
    acc = (C.c_int32 * 2)()
    h0 = (C.c_double * 2)()
    h1 = (C.c_double * 2)()
    u = (C.c_double * 2)(*uni)
    ho = S.HmcOpts(eps=0.02, n_leap=3, n_traj=2)
    S.check(S.lib.sca_hmc(ctx, C.byref(p), C.byref(ho), ph, dev(mom), u, acc,
                          h0, h1))
    ref, racc, rh0, rh1 = oracle.hmc_chain(pd(p), phi0, mom, uni, 0.02, 3)
    return {"phi": rel(host(ph, N), ref), "h_old": rel(np.array(h0[:]), rh0),
            "h_new": rel(np.array(h1[:]), rh1)}, \
        {"accepted": list(acc[:]) == [int(x) for x in racc]}


CASES = {
    "grad_small": lambda: (grad_case(params(4, 16)), {}),
    "grad_blocked": lambda: (grad_case(params(10, 4)), {}),
    # L = 18 (Np = 352): the row-panel LU instances of the 20x20 runs, and
    # the complex64 inverse two workgroups per CU
    "grad_rowpanel": lambda: (grad_case(params(18, 1)), {}),
    "grad_rowpanel_fp32r": lambda: (grad_case(params(18, 1, precision=1)), {}),
    "grad_fp32r": lambda: (grad_case(params(10, 4, precision=1)), {}),
    "grad_ldlt": lambda: (grad_case(params(10, 4, factor=1)), {}),
    "grad_eigh": lambda: (grad_case(params(6, 8, factor=2)), {}),
    # L = 14 (N = 196): Householder launches for the first columns, then the
    # one-workgroup kernel for the last 160
    "grad_eigh_chain": lambda: (grad_case(params(14, 1, factor=2)), {}),
    "grad_tail": lambda: (grad_case(params(6, 64, tail=1)), {}),
    "adam": case_adam,
    "dos": case_dos,
    "factors": case_factors,
    "noalloc": case_noalloc,
    "server": case_server,
    "hmc": case_hmc,
}

if __name__ == "__main__":
    name = sys.argv[2]
    errs, bits = CASES[name]()
    print(json.dumps({"case": name, "errors": errs, "bitwise": bits,
                      "digest": DIGEST.hexdigest()}))
