"""Request drivers for the continuous-batching server.

A request is the next load step of one resident problem's strain ramp.  The
drivers only submit requests and collect results; admission, batching and
the solve run in the library (spff_server_progress).

Each problem walks its own ramp: ``cursor[pid]`` is the index of its next
load step and is advanced by every driver call, so successive calls continue
the ramps (through crack nucleation) instead of replaying their start.  A
problem whose ramp is exhausted receives no further requests.

Latency of a request is measured from its arrival (the scheduled arrival
time of an open-loop run, the start of a closed-loop run) to the moment the
host observes its completion: the wait before ``submit`` (the host was busy
driving the device) plus the server's submit-to-completion time."""

import time

import numpy as np


def _has_next(ramps, cursor, pid):
    return cursor[pid] < len(ramps[pid])


def run_closed(server, ramps, cursor, steps_per_problem, deadline=None):
    """Saturation run: the next `steps_per_problem` load steps of every
    problem (fewer where its ramp ends) are submitted at once, in ramp order
    per problem.  `deadline` (a time.perf_counter() value) stops the run;
    requests still running then stay queued in the server.  Returns
    (completed requests/s, latencies ms, wall s, per-request stats dicts,
    tickets still running)."""
    inflight, lat, results = {}, [], []
    t0 = time.perf_counter()
    for pid in ramps:
        for _ in range(steps_per_problem):
            if not _has_next(ramps, cursor, pid):
                break
            t = server.submit(pid, ramps[pid][cursor[pid]])
            cursor[pid] += 1
            inflight[t] = (pid, (time.perf_counter() - t0) * 1e3)
    while inflight and (deadline is None or time.perf_counter() < deadline):
        server.progress(1)
        for t, (pid, wait_ms) in list(inflight.items()):
            st = server.poll(t)
            if st is not None:
                lat.append(wait_ms + st["wall_ms"])
                results.append(dict(st, pid=pid, ticket=t))
                del inflight[t]
    wall = time.perf_counter() - t0
    return len(lat) / wall, lat, wall, results, sorted(inflight)


def run_poisson(server, ramps, cursor, rate, n_requests, seed=0, warmup=0, arrivals=None, deadline=None):
    """Open-loop run: requests arrive as a Poisson process of `rate` per
    second (or at the given `arrivals`, seconds from the start, one per
    request); each picks uniformly one problem that still has load steps
    left and asks for its next one (a problem's requests queue behind each
    other).  `deadline` (a time.perf_counter() value) ends the run early:
    no request is submitted after it and the host stops driving the device;
    requests still in flight then are "censored" and enter the latency list
    with their age at the deadline (a lower bound of their latency).
    Returns (throughput requests/s over the measured completed requests,
    latencies ms from arrival, offered rate, per-request stats dicts of the
    measured completed requests, number of censored measured requests)."""
    rng = np.random.default_rng(seed)
    pids = sorted(ramps)
    total = n_requests + warmup
    if arrivals is None:
        arrivals = np.cumsum(rng.exponential(1.0 / rate, size=total))
    else:
        arrivals = np.asarray(arrivals, dtype=np.float64)
        assert arrivals.shape == (total,)
    picks = rng.random(size=total)
    inflight, lat, done_at, results = {}, [], [], []
    t0 = time.perf_counter()
    k = 0
    while k < total or inflight:
        if deadline is not None and time.perf_counter() >= deadline:
            break
        now = time.perf_counter() - t0
        while k < total and arrivals[k] <= now:
            live = [pid for pid in pids if _has_next(ramps, cursor, pid)]
            if not live:
                total = k
                break
            pid = live[int(picks[k] * len(live))]
            t = server.submit(pid, ramps[pid][cursor[pid]])
            cursor[pid] += 1
            wait_ms = (time.perf_counter() - t0 - arrivals[k]) * 1e3
            inflight[t] = (k, pid, wait_ms)
            k += 1
        if inflight:
            server.progress(1)
            for t, (idx, pid, wait_ms) in list(inflight.items()):
                st = server.poll(t)
                if st is not None:
                    del inflight[t]
                    if idx >= warmup:
                        lat.append(wait_ms + st["wall_ms"])
                        done_at.append(time.perf_counter() - t0)
                        results.append(dict(st, pid=pid, ticket=t, arrival_s=float(arrivals[idx])))
        elif k < total:
            time.sleep(max(0.0, min(arrivals[k] - (time.perf_counter() - t0), 0.002)))
    end = time.perf_counter() - t0
    censored = 0
    for t, (idx, pid, wait_ms) in inflight.items():
        if idx >= warmup:
            lat.append((end - arrivals[idx]) * 1e3)
            censored += 1
    span = (max(done_at) - arrivals[warmup]) if done_at and total > warmup else float("nan")
    return (len(done_at) / span if span > 0 else float("nan")), lat, rate, results, censored
