"""Request drivers for the continuous-batching server.

A request is the next load step of one resident problem's strain ramp.  The
drivers only submit requests and collect results; admission, batching and
the solve run in the library (spff_server_progress)."""

import time

import numpy as np


def _collect(server, inflight, lat, done_at):
    finished = []
    for t, (pid, t_arr) in list(inflight.items()):
        st = server.poll(t)
        if st is not None:
            lat.append(st["wall_ms"])
            finished.append((t, pid, st))
            del inflight[t]
            done_at.append(time.perf_counter())
    return finished


def run_closed(server, ramps, steps_per_problem):
    """Saturation run: every problem's next `steps_per_problem` load steps are
    submitted at once (in ramp order per problem); returns (requests/s,
    latencies ms, wall s, per-request stats)."""
    nxt = {pid: 0 for pid in ramps}
    inflight, lat, done_at, results = {}, [], [], []
    t0 = time.perf_counter()
    for pid, ramp in ramps.items():
        for _ in range(steps_per_problem):
            t = server.submit(pid, ramp[nxt[pid]])
            nxt[pid] += 1
            inflight[t] = (pid, t0)
    while inflight:
        server.progress(1)
        results += _collect(server, inflight, lat, done_at)
    wall = time.perf_counter() - t0
    return len(lat) / wall, lat, wall, results


def run_poisson(server, ramps, start_step, rate, n_requests, seed=0, warmup=0):
    """Open-loop run: requests arrive as a Poisson process of `rate` per
    second; each picks a problem uniformly and asks for its next load step
    (a problem's requests queue behind each other).  Returns (throughput
    requests/s over the measured requests, latencies ms, offered rate)."""
    rng = np.random.default_rng(seed)
    pids = sorted(ramps)
    nxt = {pid: start_step for pid in pids}
    total = n_requests + warmup
    gaps = rng.exponential(1.0 / rate, size=total)
    arrivals = np.cumsum(gaps)
    who = rng.integers(0, len(pids), size=total)
    inflight, lat, done_at = {}, [], []
    order = {}
    t0 = time.perf_counter()
    k = 0
    while k < total or inflight:
        now = time.perf_counter() - t0
        while k < total and arrivals[k] <= now:
            pid = pids[who[k]]
            if nxt[pid] >= len(ramps[pid]):
                nxt[pid] = start_step
            t = server.submit(pid, ramps[pid][nxt[pid]])
            nxt[pid] += 1
            inflight[t] = (pid, arrivals[k])
            order[t] = k
            k += 1
        if inflight:
            server.progress(1)
            fin = []
            for t in list(inflight):
                st = server.poll(t)
                if st is not None:
                    fin.append((order[t], st["wall_ms"], time.perf_counter() - t0))
                    del inflight[t]
            for idx, ms, tdone in fin:
                if idx >= warmup:
                    lat.append(ms)
                    done_at.append(tdone)
        elif k < total:
            time.sleep(max(0.0, min(arrivals[k] - (time.perf_counter() - t0), 0.002)))
    span = (max(done_at) - arrivals[warmup]) if done_at else float("nan")
    return len(lat) / span, lat, rate
