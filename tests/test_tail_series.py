"""The moment expansion behind Params(tail=True), restated in NumPy and
checked against the oracle (CPU): for frequencies w_n above 3x the spectral
radius of H,

  ln|det(i w - H)|      = N ln w + 1/2 sum_m (-1)^(m+1)/m tr(H^2m) w^-2m,
  Re (i w - H)^-1_ii    = -sum_m (-1)^m (H^(2m+1))_ii w^-(2m+2),

cut after 14 terms.  Replacing the oracle's terms for n >= n_c by these
series must reproduce Omega~ and the gradient to rounding; a wrong sign,
factor or power fails by many orders of magnitude."""
import numpy as np
import pytest

import oracle
from oracle import model
import synth

K = 14


def series_terms(H, w):
    """(sum_n ln|det| - N ln w_n, sum_n Re diag G) over the frequencies w."""
    N = H.shape[0]
    pw = [np.eye(N)]
    for _ in range(2 * K + 1):
        pw.append(pw[-1] @ H)
    red = 0.0
    g = np.zeros(N)
    for wn in w:
        red += 0.5 * sum((-1) ** (m + 1) / m * np.trace(pw[2 * m]) * wn ** (-2 * m)
                         for m in range(1, K + 1))
        g -= sum((-1) ** m * np.diag(pw[2 * m + 1]) * wn ** (-(2 * m + 2))
                 for m in range(K + 1))
    return red, g


@pytest.mark.parametrize("L,U,delta,T,M,seed", [(6, 4.0, 0.0, 0.1, 256, 1),
                                               (6, 3.0, 1.0, 0.3, 128, 2),
                                               (4, 6.0, 0.4, 0.05, 512, 3)])
def test_tail_series_matches_oracle(L, U, delta, T, M, seed):
    N = L * L
    phi = synth.uniform(seed, N, -0.8, 0.8)
    p = dict(L=L, t=1.0, U=U, delta=delta, T=T, n_max=M)
    w = model.matsubara(T, M)
    # split as the library does: rho bound from Gershgorin, w_c = 4 rho_b
    rho_b = 4.0 + 0.5 * abs(delta) + max(np.max(np.abs(phi)), U / 2) + 0.5
    nc = max(1, int(np.ceil((4 * rho_b / (np.pi * T) - 1) / 2)))
    assert nc < M
    pe = dict(p, n_max=nc)
    # exact part: the oracle over n < n_c; tail by the series
    om_e = oracle.omega_tilde(pe, phi)
    g_e = oracle.grad(pe, phi)
    red_t, gsum = 0.0, np.zeros(N)
    for s in (1, -1):
        H = model.hamiltonian(L, 1.0, delta, phi, s)
        assert np.max(np.abs(np.linalg.eigvalsh(H))) < w[nc] / 3
        r, g = series_terms(H, w[nc:])
        red_t += r
        gsum += s * g
    om = om_e - 2 * T * red_t
    gr = g_e - 2 * T * gsum
    om_ref = oracle.omega_tilde(p, phi)
    g_ref = oracle.grad(p, phi)
    e_om = abs(om - om_ref) / abs(om_ref)
    e_g = np.max(np.abs(gr - g_ref)) / np.max(np.abs(g_ref))
    print(f"L={L} T={T} M={M} n_c={nc}: Omega~ {e_om:.1e} grad {e_g:.1e}")
    assert e_om < 1e-12 and e_g < 1e-11
