"""Request loop over continuous-batching servers (one per resident database).

Requests arrive over time (seeded Poisson arrivals in the benchmark), each
routed to one database. The loop admits waiting requests into free solver
columns as soon as columns free up (hd_serve_submit), queues one CG
iteration on every server that has work (hd_serve_step, asynchronous, so the
servers' GPU work overlaps), and collects finished requests
(hd_serve_poll) when it knows some have finished. Latency is measured from
arrival to collection.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    arrival: float            # seconds after the start of the run
    db: str
    y_ids: np.ndarray = None  # k_y ids, or None with q_desc
    y_val: np.ndarray = None
    q_desc: np.ndarray = None
    max_iter: int = 20
    admitted: float = -1.0
    finished: float = -1.0
    result: dict = field(default_factory=dict)


def poisson_arrivals(rate_per_s: float, count: int, seed: int) -> np.ndarray:
    """Arrival times of a Poisson process (exponential gaps), seeded."""
    gaps = np.random.default_rng(seed).exponential(1.0 / rate_per_s, size=count)
    return np.cumsum(gaps)


def run(servers: dict, requests: list, iters_per_step: int = 1, max_admit: int = 1024,
        poll_every: int = 8):
    """Serve `requests` (sorted by arrival) on `servers` ({db: hd.Server}).
    Returns (requests with timings and results, wall seconds).

    A server without a tolerance (tol <= 0: every request runs to its cap)
    is polled (a stream synchronisation, and for the finished columns one
    pass over U1 to combine and one top-K) only when a request on it has
    certainly finished - the loop counts each request's iterations against
    its cap - or every `poll_every` turns (columns that stop at once, with
    y = 0 or a breakdown); between polls the loop queues the next iterations
    without waiting for the device. A server with tol > 0, whose columns may
    converge at any iteration, is polled every turn."""
    pending = deque(sorted(requests, key=lambda r: r.arrival))
    waiting = {db: deque() for db in servers}
    by_ticket = {db: {} for db in servers}
    iters_done = {db: {} for db in servers}    # ticket -> iterations queued since admission
    t0 = time.perf_counter()
    done = 0
    turn = 0
    while done < len(requests):
        turn += 1
        now = time.perf_counter() - t0
        while pending and pending[0].arrival <= now:
            r = pending.popleft()
            waiting[r.db].append(r)
        busy = False
        for db, srv in servers.items():
            q = waiting[db]
            if q:
                batch = list(q)[:max_admit]
                if batch[0].q_desc is not None:
                    tk = srv.submit(q_desc=np.stack([r.q_desc for r in batch]),
                                    max_iter=np.array([r.max_iter for r in batch]))
                else:
                    tk = srv.submit(np.stack([r.y_ids for r in batch]), np.stack([r.y_val for r in batch]),
                                    max_iter=np.array([r.max_iter for r in batch]))
                t_adm = time.perf_counter() - t0
                for t, r in zip(tk, batch):
                    r.admitted = t_adm
                    by_ticket[db][int(t)] = r
                    iters_done[db][int(t)] = 0
                    q.popleft()
            if srv.in_use:
                srv.step(iters_per_step)
                for t in iters_done[db]:
                    iters_done[db][t] += iters_per_step
                busy = True
        for db, srv in servers.items():
            if not by_ticket[db]:
                continue
            # each request's own cap is passed at submission (it overrides
            # the server's default)
            capped = getattr(srv, "tol", 1.0) <= 0.0
            known = any(iters_done[db][t] >= r.max_iter for t, r in by_ticket[db].items())
            if capped and not known and turn % poll_every != 0:
                continue
            res = srv.poll()
            t_fin = time.perf_counter() - t0
            for k, t in enumerate(res["tickets"]):
                r = by_ticket[db].pop(int(t))
                iters_done[db].pop(int(t))
                r.finished = t_fin
                r.result = {key: res[key][k] for key in ("ids", "scores", "iters", "relres", "status")}
                done += 1
        if not busy and pending and not any(waiting.values()):
            gap = pending[0].arrival - (time.perf_counter() - t0)
            if gap > 0:
                time.sleep(min(gap, 0.001))
    return requests, time.perf_counter() - t0


def latency_stats(requests) -> dict:
    lat = np.array([r.finished - r.arrival for r in requests])
    return {"p50_ms": float(1e3 * np.percentile(lat, 50)), "p99_ms": float(1e3 * np.percentile(lat, 99)),
            "mean_ms": float(1e3 * lat.mean()), "count": int(lat.size)}
