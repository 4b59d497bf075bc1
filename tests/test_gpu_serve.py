"""GPU tests of the request server (continuous batching of ADAM solves).

* alone vs mix: requests of mixed shapes (fused small path, blocked FP64,
  FP32-refined, symmetric L D L^T), submitted together and batched with
  each other, give bit-for-bit the phi, moments and statistics that sca.adam_solve gives
  for each alone;
* the same under an HBM budget that holds one group at a time (requests
  wait in the queue, groups give their memory back);
* staggered arrivals join running groups between chunks, with the same
  bitwise result;
* argument errors.
"""
import numpy as np
import pytest

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


def mix(sca):
    out = []
    shapes = [(4, 32, "fp64", "lu"), (8, 32, "fp64", "lu"),
              (4, 32, "fp64", "lu"), (10, 16, "fp64", "lu"),
              (8, 32, "fp64", "lu"), (12, 16, "fp32r", "lu"),
              (10, 16, "fp64", "lu"), (12, 16, "fp32r", "lu"),
              (4, 16, "fp64", "lu"), (12, 16, "fp64", "ldlt"),
              (12, 16, "fp64", "ldlt")]
    for k, (L, M, prec, fac) in enumerate(shapes):
        r = synth.uniform(900 + k, 4, 0.0, 1.0)
        p = sca.Params(L=L, U=2.0 + 4.0 * r[0], delta=1.5 * r[1],
                       T=0.1 + 0.3 * r[2], n_max=M, precision=prec,
                       factor=fac)
        steps = 5 + int(10 * r[3])
        out.append(dict(params=p, phi0=cuda(synth.uniform(k, L * L, -0.5, 0.5)),
                        n_steps=steps, lr=0.02, final_eval=(k % 3 != 2)))
    return out


def alone(sca, r):
    kw = {k: v for k, v in r.items() if k not in ("params", "phi0", "n_steps")}
    return sca.adam_solve(r["params"], r["phi0"], r["n_steps"], **kw)


def check_same(sca, reqs, results):
    import torch
    for k, r in enumerate(reqs):
        phi, m, v, res, _ = results[k]
        phi_a, m_a, v_a, res_a = alone(sca, r)
        assert torch.equal(phi, phi_a), k
        assert torch.equal(m, m_a) and torch.equal(v, v_a), k
        for f in ("omega", "omega_tilde", "af_order", "max_abs_grad",
                  "max_pivot_growth", "steps_done"):
            assert res[f] == res_a[f], (k, f, res[f], res_a[f])


def test_alone_vs_mix_bitwise(sca):
    from paper_2311_04435_amd.serve import Server
    reqs = mix(sca)
    with Server(max_batch=4) as srv:
        tickets = [srv.submit(r["params"], r["phi0"], r["n_steps"], lr=r["lr"],
                              final_eval=r["final_eval"]) for r in reqs]
        done = srv.drain(tickets)
    check_same(sca, reqs, [done[t] for t in tickets])


def test_budget_one_group_at_a_time(sca):
    from paper_2311_04435_amd.serve import Server
    reqs = mix(sca)
    biggest = max(sca.footprint_bytes(r["params"]) for r in reqs)
    with Server(hbm_budget_bytes=int(1.5 * biggest), max_batch=2) as srv:
        tickets = [srv.submit(r["params"], r["phi0"], r["n_steps"], lr=r["lr"],
                              final_eval=r["final_eval"]) for r in reqs]
        a, q = srv.progress()
        assert q > 0          # not everything fits at once
        done = srv.drain(tickets)
    check_same(sca, reqs, [done[t] for t in tickets])


def test_staggered_arrivals(sca):
    from paper_2311_04435_amd.serve import Server, run_stream
    reqs = mix(sca)
    arrivals = np.linspace(0.0, 0.05, len(reqs))
    with Server(max_batch=8) as srv:
        results, lat, makespan = run_stream(srv, reqs, arrivals)
    assert np.all(lat > 0) and makespan > 0
    check_same(sca, reqs, results)


def test_server_argument_errors(sca):
    from paper_2311_04435_amd import SCAError
    from paper_2311_04435_amd.serve import Server
    p = sca.Params(L=4, U=4.0, T=0.1, n_max=16)
    with Server(max_batch=2) as srv:
        with pytest.raises(SCAError):
            srv.submit(sca.Params(L=5, U=4.0, T=0.1, n_max=16),
                       cuda(np.zeros(25)), 3)
        with pytest.raises(SCAError):
            srv.submit(p, cuda(np.zeros(16)), -1)
        with pytest.raises(SCAError):
            srv.poll(12345)
    with pytest.raises(SCAError):
        Server(max_batch=0)
    with Server(hbm_budget_bytes=1024) as srv:
        with pytest.raises(SCAError, match="ENOMEM"):
            srv.submit(p, cuda(np.zeros(16)), 3)


def test_tail_requests_bitwise(sca):
    """Requests with the Matsubara tail (fewer matrices each) share groups
    with ordinary ones of the same shape; each still matches its own
    sca.adam_solve bit for bit."""
    from paper_2311_04435_amd.serve import Server
    reqs = []
    for k in range(6):
        r = synth.uniform(1200 + k, 3, 0.0, 1.0)
        p = sca.Params(L=12, U=3.0 + 2.0 * r[0], delta=r[1], T=0.1 + 0.1 * r[2],
                       n_max=128, factor="ldlt" if k % 3 == 2 else "lu",
                       tail=(k % 2 == 0))
        reqs.append(dict(params=p, phi0=cuda(synth.uniform(40 + k, 144, -0.5, 0.5)),
                         n_steps=6 + k, lr=0.02, final_eval=True))
    with Server(max_batch=4) as srv:
        tickets = [srv.submit(r["params"], r["phi0"], r["n_steps"], lr=r["lr"])
                   for r in reqs]
        done = srv.drain(tickets)
    for t in tickets:
        assert not (done[t][3]["flags"] & sca.SCA_FLAG_TAIL_RANGE)
    check_same(sca, reqs, [done[t] for t in tickets])
