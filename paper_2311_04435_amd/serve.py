"""Serving: many SCA+ADAM solves at once on one GPU (sca_server_* calls).

Server wraps the library's request loop: submit() hands over a parameter
point and a starting field, progress() lets the library retire, admit and
launch, poll() returns finished solves.  phi, m and v live in device tensors
this object keeps alive until the request is polled.

run_stream() replays a list of requests with given arrival times in real
time and measures per-request latency (finish - arrival);
fifo_latencies() gives the one-at-a-time baseline from measured service
times (each request solved alone with sca.adam_solve, in arrival order).
"""
from __future__ import annotations

import ctypes as C
import time
from typing import Optional

import numpy as np
import torch

from . import _lib, Params, _dev

__all__ = ["Server", "run_stream", "fifo_latencies", "latency_summary"]


class Server:
    def __init__(self, device: Optional[int] = None, hbm_budget_bytes: int = 0,
                 max_batch: int = 16):
        if device is None:
            device = torch.cuda.current_device()
        self.device = device
        h = C.c_void_p()
        _lib.check(_lib.lib.sca_server_create(device, hbm_budget_bytes,
                                              max_batch, C.byref(h)))
        self._h = h
        self._live = {}

    def close(self):
        if getattr(self, "_h", None):
            _lib.lib.sca_server_destroy(self._h)
            self._h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def clock(self) -> float:
        """Seconds since the server was created (the clock of finish times)."""
        return float(_lib.lib.sca_server_clock(self._h))

    def submit(self, p: Params, phi0: torch.Tensor, n_steps: int,
               lr: float = 0.01, beta1: float = 0.9, beta2: float = 0.999,
               eps: float = 1e-8, t0: int = 0, final_eval: bool = True,
               m: Optional[torch.Tensor] = None,
               v: Optional[torch.Tensor] = None) -> int:
        """Queue an ADAM solve from phi0 (copied); returns its ticket."""
        phi = _dev(phi0, p.N, "phi0").clone()
        m = torch.zeros_like(phi) if m is None else _dev(m, p.N, "m").clone()
        v = torch.zeros_like(phi) if v is None else _dev(v, p.N, "v").clone()
        flags = 0 if final_eval else _lib.SCA_ADAM_NO_FINAL_EVAL
        opts = _lib.AdamOpts(lr, beta1, beta2, eps, 0.0, n_steps, 0, t0, flags)
        ticket = C.c_int64()
        # the tensors must be ready before the server's streams read them
        torch.cuda.current_stream(self.device).synchronize()
        _lib.check(_lib.lib.sca_server_submit(
            self._h, C.byref(p.c()), C.byref(opts), phi.data_ptr(),
            m.data_ptr(), v.data_ptr(), C.byref(ticket)))
        self._live[ticket.value] = (phi, m, v, p)
        return ticket.value

    def progress(self, wait_s: float = 0.0):
        """One scheduling round; returns (running, queued) request counts."""
        a, q = C.c_int32(), C.c_int32()
        _lib.check(_lib.lib.sca_server_progress(self._h, wait_s, C.byref(a),
                                                C.byref(q)))
        return a.value, q.value

    def poll(self, ticket: int):
        """None while running; else (phi, m, v, result dict, t_done)."""
        done = C.c_int32()
        res = _lib.Result()
        t_done = C.c_double()
        _lib.check(_lib.lib.sca_server_poll(self._h, ticket, C.byref(done),
                                            C.byref(res), C.byref(t_done)))
        if not done.value:
            return None
        phi, m, v, _ = self._live.pop(ticket)
        out = {f: getattr(res, f) for f, _ in _lib.Result._fields_}
        return phi, m, v, out, t_done.value

    def drain(self, tickets, wait_s: float = 0.002):
        """Run until every ticket finished; returns {ticket: poll result}."""
        left = set(tickets)
        out = {}
        while left:
            self.progress(wait_s)
            for t in list(left):
                r = self.poll(t)
                if r is not None:
                    out[t] = r
                    left.discard(t)
        return out


def run_stream(server: Server, requests, arrivals, wait_s: float = 0.0005,
               on_done=None):
    """Submit request k at server time arrivals[k] (seconds from now) and run
    until all finish.  requests: list of dict(params=Params, phi0=tensor,
    n_steps=int, **adam kwargs).  Returns (results, latencies, makespan):
    results[k] the poll result, latencies[k] = finish - arrival.  on_done,
    if given, is called with the number of finished requests each time one
    finishes."""
    order = np.argsort(arrivals, kind="stable")
    base = server.clock()
    arr = base + np.asarray(arrivals, dtype=np.float64)
    tickets = {}
    results = [None] * len(requests)
    lat = np.zeros(len(requests))
    nxt = 0
    pending = set()
    while nxt < len(order) or pending:
        now = server.clock()
        while nxt < len(order) and arr[order[nxt]] <= now:
            k = int(order[nxt])
            r = dict(requests[k])
            t = server.submit(r.pop("params"), r.pop("phi0"), r.pop("n_steps"),
                              **r)
            tickets[t] = k
            pending.add(t)
            nxt += 1
        wait = wait_s
        if nxt < len(order):
            wait = min(wait, max(0.0, arr[order[nxt]] - server.clock()))
        server.progress(wait)
        for t in list(pending):
            out = server.poll(t)
            if out is not None:
                k = tickets[t]
                results[k] = out
                lat[k] = out[4] - arr[k]
                pending.discard(t)
                if on_done is not None:
                    on_done(sum(r is not None for r in results))
        if not pending and nxt < len(order):
            time.sleep(max(0.0, min(0.001, arr[order[nxt]] - server.clock())))
    makespan = server.clock() - base
    return results, lat, makespan


def fifo_latencies(arrivals, service):
    """Latencies of one-at-a-time service in arrival order (Lindley)."""
    order = np.argsort(arrivals, kind="stable")
    lat = np.zeros(len(arrivals))
    free = 0.0
    for k in order:
        start = max(arrivals[k], free)
        free = start + service[k]
        lat[k] = free - arrivals[k]
    makespan = free - float(np.min(arrivals)) if len(arrivals) else 0.0
    return lat, makespan


def latency_summary(lat, makespan):
    n = len(lat)
    return {"solves": n, "solves_per_s": n / makespan if makespan > 0 else 0.0,
            "p50_ms": 1e3 * float(np.percentile(lat, 50)),
            "p99_ms": 1e3 * float(np.percentile(lat, 99)),
            "mean_ms": 1e3 * float(np.mean(lat))}
