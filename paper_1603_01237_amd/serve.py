"""Trace replay on the libism server: requests are submitted at their arrival times
(relative to the start of the replay) and the server is polled until every one has
finished.  Latency = completion - arrival, queueing included."""
from __future__ import annotations

import time

import numpy as np

from ._lib import REQ_DONE, REQ_FAILED, Server


def replay(server: Server, items, idle_sleep: float = 2e-4, timeout: float = 600.0,
           report_every: float = 0.0, log=print):
    """items: list of (arrival_s, problem, submit-kwargs) sorted by arrival.  Returns
    (records, wall_s) with one record per item: ticket, state, status, iters, J, F,
    latency_s, queue_s, u (final controls or None).  With report_every > 0 a progress
    line (submitted / finished / queued / running) is logged at that interval."""
    t0 = Server.clock()
    t_rep = 0.0
    pending = {}
    records = [None] * len(items)
    i = 0
    done_seen = -1
    while i < len(items) or pending:
        now = Server.clock() - t0
        if now > timeout:
            raise TimeoutError(f"replay exceeded {timeout} s with {len(pending)} requests open")
        while i < len(items) and items[i][0] <= now:
            arr, prob, kw = items[i]
            pending[server.submit(prob, t_arrival=t0 + arr, **kw)] = i
            i += 1
        nq, nr = server.progress()
        st = server.stats()
        if report_every > 0 and now - t_rep >= report_every:
            t_rep = now
            log(f"replay t={now:.1f}s submitted={i} finished={st['completed'] + st['failed']} "
                f"queued={nq} running={nr}")
        finished = st["completed"] + st["failed"]
        if finished != done_seen:
            done_seen = finished
            for t in list(pending):
                if server.poll(t)["state"] in (REQ_DONE, REQ_FAILED):
                    res, u = server.take(t)
                    k = pending.pop(t)
                    records[k] = dict(ticket=t, state=res["state"], status=res["status"],
                                      iters=res["iters"], J=res["J"], F=res["F"],
                                      latency_s=res["t_done"] - res["t_arrival"],
                                      queue_s=max(res["t_admit"] - res["t_arrival"], 0.0),
                                      u=u)
        nxt = items[i][0] - (Server.clock() - t0) if i < len(items) else idle_sleep
        time.sleep(min(max(nxt, 0.0), idle_sleep))
    return records, Server.clock() - t0


def latency_summary(records, wall_s: float) -> dict:
    lat = np.array([r["latency_s"] for r in records if r["state"] == REQ_DONE])
    return {"requests": len(records), "completed": int(lat.size),
            "failed": sum(r["state"] == REQ_FAILED for r in records),
            "p50_s": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_s": float(np.percentile(lat, 99)) if lat.size else None,
            "solves_per_s": float(lat.size / wall_s) if wall_s > 0 else None,
            "wall_s": wall_s}
