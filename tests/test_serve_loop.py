"""Host logic of the continuous-batching driver, against a scripted stand-in
for the GPU batch (no GPU, no oracle)."""
from paper_2302_12519_amd import serve


class FakeBatch:
    """Admits up to `slots` requests FIFO; each advance moves every resident
    request by K steps; a request finishes after its step count."""

    def __init__(self, slots=2, K=10):
        self.slots, self.K = slots, K
        self.queue, self.res, self.done = [], {}, []
        self.next, self.steps, self.launches = 1, 0.0, 0
        self.t = 0.0

    def submit(self, nsteps):
        bid = self.next
        self.next += 1
        self.queue.append((bid, nsteps))
        return bid

    def advance(self):
        while self.queue and len(self.res) < self.slots:
            bid, n = self.queue.pop(0)
            self.res[bid] = [0, n]
        self.launches += 1
        self.t += 1.0
        for bid, st in list(self.res.items()):
            adv = min(self.K, st[1] - st[0])
            st[0] += adv
            self.steps += adv
            if st[0] >= st[1]:
                self.done.append(bid)
                del self.res[bid]

    def finished(self):
        out, self.done = self.done, []
        return out

    def read(self, bid, field):
        return bid

    def release(self, bid):
        pass

    def stats(self):
        return {"voxel_steps": self.steps, "graph_launches": self.launches, "arena_peak": 0}


class Req:
    def __init__(self, rid, arrival, n):
        self.rid, self.arrival, self.n = rid, arrival, n

    def submit(self, batch):
        return batch.submit(self.n)


def test_all_requests_complete_with_latency():
    fb = FakeBatch(slots=2, K=10)
    clock = lambda: fb.t
    reqs = [Req(k, 0.0, 10 * (k + 1)) for k in range(5)]
    out = serve.serve(fb, reqs, clock=clock, sleep=lambda s: None, submit_per_advance=5)
    assert sorted(out["latency"]) == list(range(5))
    # with 2 slots: r0 (1 launch), r1 (2) run first; r2 enters after r0 ...
    assert out["latency"][0] == 1.0
    assert out["latency"][1] == 2.0
    assert all(out["latency"][k] > 0 for k in range(5))
    assert out["voxel_steps"] == sum(10 * (k + 1) for k in range(5))
    assert out["p50"] <= out["p99"]


def test_idle_until_next_arrival():
    fb = FakeBatch(slots=4, K=5)
    waits = []

    def sleep(s):
        waits.append(s)
        fb.t += s

    reqs = [Req(0, 0.0, 5), Req(1, 10.0, 5)]
    out = serve.serve(fb, reqs, clock=lambda: fb.t, sleep=sleep)
    assert waits and abs(sum(waits) - 9.0) < 1e-12
    assert out["latency"][1] == 1.0


def test_percentile_interpolates():
    assert serve.percentile([1, 2, 3, 4], 50) == 2.5
    assert serve.percentile([5], 99) == 5


def test_one_submission_per_advance():
    """A burst is fed one request per advance: every request still
    completes, the first starts after one launch, and no launch is idle."""
    fb = FakeBatch(slots=8, K=10)
    clock = lambda: fb.t
    reqs = [Req(k, 0.0, 20) for k in range(4)]
    out = serve.serve(fb, reqs, clock=clock, sleep=lambda s: None, submit_per_advance=1)
    assert sorted(out["latency"]) == list(range(4))
    assert out["latency"][0] == 2.0
    assert out["latency"][3] == 5.0
    assert out["voxel_steps"] == 80
