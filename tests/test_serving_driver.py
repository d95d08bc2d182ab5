"""Request drivers of the server (host logic only, no GPU): latency is
counted from a request's arrival, not from the moment the driver got round
to submitting it, and problems walk their ramps across driver calls."""

import numpy as np

from paper_2203_16467_amd import serving


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def perf_counter(self):
        return self.t

    def sleep(self, dt):
        # a real sleep always lets some time pass
        self.t += max(dt, 1e-6)


class FakeServer:
    """Every progress() call blocks for `block` seconds of the fake clock and
    completes the requests that were submitted before it started; wall_ms is
    submit-to-completion, as the library reports it."""

    def __init__(self, clock, block):
        self.clock, self.block = clock, block
        self.next, self.pending, self.done = 0, [], {}
        self.submitted = {}   # ticket -> (pid, eps_bar, submit time)
        self.completed = {}   # ticket -> completion time

    def submit(self, pid, eps_bar):
        t = self.next
        self.next += 1
        self.submitted[t] = (pid, tuple(eps_bar), self.clock.t)
        self.pending.append(t)
        return t

    def progress(self, max_rounds=1):
        batch, self.pending = self.pending, []
        self.clock.t += self.block
        for t in batch:
            self.completed[t] = self.clock.t
            self.done[t] = {"wall_ms": (self.clock.t - self.submitted[t][2]) * 1e3, "am_iters": 1}
        return len(batch), len(self.pending)

    def poll(self, ticket):
        return self.done.pop(ticket, None)


def _ramps(nprob, steps):
    return {pid: np.arange(steps * 3, dtype=float).reshape(steps, 3) + 100 * pid for pid in range(nprob)}


def test_poisson_latency_counts_from_arrival(monkeypatch):
    clock = FakeClock()
    monkeypatch.setattr(serving, "time", clock)
    sv = FakeServer(clock, block=0.05)
    ramps = _ramps(4, 50)
    cursor = {pid: 0 for pid in ramps}
    arrivals = np.arange(40) * 0.007  # several requests arrive while progress() blocks
    thr, lat, _, res, cens = serving.run_poisson(sv, ramps, cursor, rate=1.0, n_requests=40, arrivals=arrivals)
    assert cens == 0
    assert len(lat) == 40 and len(res) == 40
    # tickets are handed out in arrival order
    order = sorted(range(40), key=lambda i: res[i]["ticket"])
    assert [res[i]["ticket"] for i in order] == list(range(40))
    want = np.array([(sv.completed[t] - arrivals[t]) * 1e3 for t in range(40)])
    np.testing.assert_allclose(np.array(lat)[order], want, atol=1e-9)
    # the submit-to-completion time alone would hide the wait before submit
    wall = np.array([r["wall_ms"] for r in res])[order]
    assert (want - wall).max() > 20.0


def test_closed_and_poisson_walk_the_ramps(monkeypatch):
    clock = FakeClock()
    monkeypatch.setattr(serving, "time", clock)
    sv = FakeServer(clock, block=0.01)
    ramps = _ramps(3, 5)
    cursor = {pid: 0 for pid in ramps}
    assert serving.run_closed(sv, ramps, cursor, 2)[4] == []
    assert cursor == {0: 2, 1: 2, 2: 2}
    serving.run_poisson(sv, ramps, cursor, rate=100.0, n_requests=9, seed=1)
    assert sum(cursor.values()) == 15 and all(c == 5 for c in cursor.values())
    # every load step of every ramp was requested exactly once, in order
    seen = {}
    for t in sorted(sv.submitted):
        pid, eb, _ = sv.submitted[t]
        seen.setdefault(pid, []).append(eb)
    for pid, ramp in ramps.items():
        assert seen[pid] == [tuple(r) for r in ramp]


def test_poisson_deadline_censors_requests_in_flight(monkeypatch):
    """At the deadline the driver stops; requests still running count with
    their age (a lower bound of their latency)."""
    clock = FakeClock()
    monkeypatch.setattr(serving, "time", clock)

    class Slow(FakeServer):
        def progress(self, max_rounds=1):
            self.clock.t += self.block  # never completes anything
            return 0, len(self.pending)

    sv = Slow(clock, block=0.05)
    ramps = _ramps(2, 20)
    cursor = {pid: 0 for pid in ramps}
    arrivals = np.arange(10) * 0.01
    _, lat, _, res, cens = serving.run_poisson(sv, ramps, cursor, rate=1.0, n_requests=10, arrivals=arrivals,
                                               deadline=0.3)
    assert res == [] and cens == len(lat) and cens >= 5
    assert all(l > 0 for l in lat)
