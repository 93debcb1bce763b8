"""The serving loop's scheduling on the CPU, with a simulated executor and
clock (no GPU): every request completes once; a step only holds requests of
one (N, op) group (at any levels), in arrival order within the group; admission never
exceeds the output slots of an N; steps run on at most `lanes` lanes at once;
and under load, continuous batching serves the same arrivals with lower
latency than one request at a time."""
import pytest

from paper_2112_06396_amd import serving


class VirtualClock:
    def __init__(self):
        self.t = 0.0

    def now(self):
        return self.t

    def idle(self, dt):
        self.t += dt


class FakeExecutor:
    """A step of n requests takes a + b n seconds of simulated time."""

    def __init__(self, clock, slots, a=6e-4, b=1e-4):
        self.clock, self.n_slots, self.a, self.b = clock, slots, a, b
        self.steps, self.running = [], set()
        self.max_running = 0
        self.held_slots = {}

    def slots(self, log_n):
        return self.n_slots

    def submit(self, lane, batch):
        assert lane not in self.running
        self.running.add(lane)
        self.max_running = max(self.max_running, len(self.running))
        for r in batch:
            key = (r.log_n, r.slot)
            assert key not in self.held_slots, "output slot handed out twice"
            self.held_slots[key] = r.rid
        self.steps.append([r.rid for r in batch])
        return (lane, self.clock.now() + self.a + self.b * len(batch), batch)

    def done(self, h):
        lane, t_end, batch = h
        if self.clock.now() >= t_end:
            self.running.discard(lane)
            for r in batch:
                del self.held_slots[(r.log_n, r.slot)]
            return True
        return False


def _serve(reqs, lanes, max_batch, slots, one=False):
    clk = VirtualClock()
    ex = FakeExecutor(clk, slots)
    eng = serving.Engine(ex, lanes=lanes, max_batch=max_batch, clock=clk.now, idle=clk.idle)
    st = eng.run(reqs, one_at_a_time=one)
    return st, ex


def test_every_request_served_once_in_groups_and_order():
    reqs = serving.poisson_requests(3000, rate=8000.0, n_clients=64, levels=(3, 6), seed=1)
    st, ex = _serve(reqs, lanes=2, max_batch=16, slots=24)
    seen = [rid for step in ex.steps for rid in step]
    assert sorted(seen) == list(range(len(reqs)))
    by_id = {r.rid: r for r in reqs}
    for step in ex.steps:
        groups = {by_id[i].group for i in step}
        assert len(groups) == 1
        arr = [by_id[i].arrival for i in step]
        assert arr == sorted(arr)
        assert len(step) <= 16
    assert ex.max_running <= 2
    for r in reqs:
        assert r.arrival <= r.start <= r.done


def test_continuous_batching_beats_one_at_a_time_under_load():
    # one request at a time serves 1 / (a + b) = 1430 requests/s; arrivals at 1200/s
    mk = lambda: serving.poisson_requests(2000, rate=1200.0, n_clients=8, levels=(3, 4), seed=2)
    plain, _ = _serve(mk(), lanes=1, max_batch=1, slots=64, one=True)
    batched, ex = _serve(mk(), lanes=2, max_batch=16, slots=64)
    assert batched["p99_ms"] < plain["p99_ms"]
    assert batched["p50_ms"] < plain["p50_ms"]
    assert max(len(s) for s in ex.steps) > 1


def test_admission_is_bounded_by_slots():
    reqs = serving.poisson_requests(500, rate=1e6, n_clients=4, levels=(3, 3), seed=3)
    st, ex = _serve(reqs, lanes=2, max_batch=16, slots=5)
    assert max(len(s) for s in ex.steps) <= 5
    assert sorted(rid for s in ex.steps for rid in s) == list(range(500))
