"""The serving loop's bookkeeping (arrivals, admission, latency) against a
mock fleet with a simulated clock; no GPU."""
import numpy as np

from paper_2606_30620_amd import serve, synth


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)


class MockFleet:
    """Advances every admitted fit one step per round; FIFO admission with at
    most max_fits at once; a round takes round_s seconds of the clock."""

    def __init__(self, clock, max_fits=2, round_s=0.001):
        self.clock, self.max_fits, self.round_s = clock, max_fits, round_s
        self.queue, self.active, self.done, self.next = [], {}, [], 1
        self.max_active_seen = 0

    def submit(self, geom, image, sigma, psf, mask, mu, rho, samples, steps, n_sub, lr, seed, log_params=None):
        t = self.next
        self.next += 1
        self.queue.append((t, steps))
        return t

    def _admit(self):
        while self.queue and len(self.active) < self.max_fits:
            t, steps = self.queue.pop(0)
            self.active[t] = steps

    def run(self, rounds):
        for _ in range(rounds):
            self._admit()
            if not self.active:
                return
            self.max_active_seen = max(self.max_active_seen, len(self.active))
            self.clock.t += self.round_s
            for t in list(self.active):
                self.active[t] -= 1
                if self.active[t] == 0:
                    del self.active[t]
                    self.done.append(t)

    def sync(self):
        self._admit()

    def poll(self):
        out, self.done = self.done, []
        return out

    def result(self, t):
        return (np.zeros(1), np.zeros(1), np.zeros(1), 0)

    def stats(self):
        return {"active": len(self.active), "queued": len(self.queue), "bytes_in_use": 0, "rounds": 0}


def test_serve_loop_accounting_with_mock_fleet():
    clock = Clock()
    fleet = MockFleet(clock, max_fits=2, round_s=0.001)
    geom = synth.CONFIGS["C1"]
    prob = synth.make_problem("C1")
    # 5 requests of 10 steps; arrivals at 0, 0, 0, 0.05, 0.2 s
    arr = [0.0, 0.0, 0.0, 0.05, 0.2]
    reqs = [serve.Request(i, a, prob, 10) for i, a in enumerate(arr)]
    res = serve.serve_fleet(reqs, fleet=fleet, clock=clock, sleep=clock.sleep, sync_every=5)
    assert fleet.max_active_seen == 2
    # first two run together (10 rounds = 10 ms), the third waits for a slot
    assert np.isclose(res.latency[0], 0.010) and np.isclose(res.latency[1], 0.010)
    assert np.isclose(res.latency[2], 0.020)
    # idle gap until 0.05 s, then alone
    assert np.isclose(res.latency[3], 0.010) and np.isclose(res.latency[4], 0.010)
    assert np.isclose(res.makespan, 0.21)
    s = res.summary()
    assert s["n"] == 5 and s["p99_ms"] >= s["p50_ms"]
