"""Serving loop over the continuous-batching engine (marshalling and timing).

Queries arrive at given wall-clock offsets; each is submitted when it
arrives, the engine advances all admitted work a few launches at a time, and
completion is detected with device events.  Latency = completion - arrival.
"""
from __future__ import annotations

import collections
import time

import numpy as np
import torch

from . import eigseis


class Query:
    def __init__(self, grid, medium, theta, receivers, lo, hi, weights, sigma,
                 sigma_mode=eigseis.SIGMA_GIVEN, arrival=0.0, device="cuda"):
        S = len(theta)
        self.grid, self.medium, self.theta = grid, medium, np.asarray(theta)
        self.receivers, self.lo, self.hi = receivers, lo, hi
        self.weights, self.sigma, self.sigma_mode = weights, sigma, sigma_mode
        self.arrival = arrival
        self.H1 = torch.empty((S, 7, 7), dtype=torch.float64, device=device)
        self.dkl = torch.empty(S, dtype=torch.float64, device=device)
        self.eig = torch.empty(1, dtype=torch.float64, device=device)
        self.status = torch.empty(S, dtype=torch.int32, device=device)
        self.chol_status = torch.empty(S, dtype=torch.int32, device=device)
        self.qid = None
        self.t_submit = None
        self.t_done = None

    def submit(self, server: eigseis.Server):
        self.qid = server.submit(self.grid, self.medium, self.theta, self.receivers,
                                 eigseis.make_prior(self.lo, self.hi), self.weights, self.H1,
                                 self.dkl, self.eig, self.sigma, self.sigma_mode,
                                 status=self.status, chol_status=self.chol_status)


def serve(server: eigseis.Server, queries, launches_per_step: int = 40,
          max_inflight_steps: int = 2, overlap: bool = True, on_event=None):
    """Runs the arrival process in real time.  Returns the queries with
    t_submit / t_done filled in (seconds from the start).  overlap=False is
    the queue-only discipline: a query is submitted only once the previous
    one has completed (no continuous batching).  on_event(kind, query, t),
    if given, is called as each query is submitted ("submit") and done
    ("done")."""
    pending = sorted(queries, key=lambda q: q.arrival)
    active = []
    inflight = collections.deque()
    t0 = time.perf_counter()
    i = 0
    while i < len(pending) or active:
        now = time.perf_counter() - t0
        while i < len(pending) and pending[i].arrival <= now and (overlap or not active):
            q = pending[i]
            q.submit(server)
            q.t_submit = now
            active.append(q)
            i += 1
            if on_event:
                on_event("submit", q, now)
        queued, running = server.pending()
        if queued or running:
            server.step(launches_per_step)
            ev = torch.cuda.Event()
            ev.record()
            inflight.append(ev)
            while len(inflight) > max_inflight_steps:
                inflight.popleft().synchronize()
        elif i < len(pending) and (overlap or not active):
            time.sleep(min(0.01, max(0.0, pending[i].arrival - now)))
        else:
            torch.cuda.synchronize()
        for q in list(active):
            if server.poll(q.qid):
                q.t_done = time.perf_counter() - t0
                active.remove(q)
                if on_event:
                    on_event("done", q, q.t_done)
    torch.cuda.synchronize()
    return queries


def latency_stats(queries):
    lat = np.array([q.t_done - q.arrival for q in queries])
    return {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "n": int(lat.size)}
