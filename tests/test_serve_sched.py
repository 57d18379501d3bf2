"""Scheduling logic of the serving loop with a simulated executor (CPU only).

The fake executor computes nothing: it models each batch's service time as
cell-steps / rate on a virtual clock, so admission, batching, lane concurrency
and latency accounting can be checked deterministically.
"""
import pytest

from paper_1101_3615_amd.serve import Request, Server, poisson_requests, summarize


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-5)


class FakeExecutor:
    def __init__(self, clock, lanes, rate=1e10, budget=None, per_shot=1.0):
        self.clock = clock
        self._lanes = lanes
        self.rate = rate
        self.budget = budget
        self.per_shot = per_shot
        self.launched = []

    def lane_keys(self):
        return list(self._lanes)

    def footprint(self, lane, op, nshots, nreq):
        return nshots * nreq * self.per_shot

    def lane_budget(self, lane):
        return self.budget if self.budget is not None else float("inf")

    def cell_steps(self, shape, nshots):
        return 1e8 * nshots

    def launch(self, lane, reqs):
        busy_until = max([self.clock()] + [h for (l, h, _) in self.launched if l == lane])
        t_end = busy_until + sum(r.cell_steps for r in reqs) / self.rate
        self.launched.append((lane, t_end, [r.rid for r in reqs]))
        return t_end

    def done(self, handle):
        return self.clock() >= handle


def _reqs(arrivals, shape="a", nshots=4, op="H", rid0=0):
    return [Request(rid=rid0 + i, arrival=t, shape=shape, shots=list(range(nshots)), op=op)
            for i, t in enumerate(arrivals)]


def test_requests_waiting_together_are_batched_in_arrival_order():
    clk = Clock()
    ex = FakeExecutor(clk, [("a", 0)], rate=4e8)          # 1 s per 4-shot request
    srv = Server(ex, max_batch=2, clock=clk, sleep=clk.sleep)
    done = srv.run(_reqs([0.0, 0.1, 0.2, 0.3]))
    assert len(done) == 4
    batches = [b for (_, _, b) in ex.launched]
    assert batches[0] == [0]                 # alone: nothing else had arrived
    assert batches[1] == [1, 2]              # the next two, capped at 2 requests
    assert batches[2] == [3]
    for r in done:
        assert r.finished >= r.started >= r.arrival


def test_footprint_admission_limits_batch_size():
    clk = Clock()
    ex = FakeExecutor(clk, [("a", 0)], rate=4e8, budget=10.0, per_shot=1.0)  # 10 shots fit
    srv = Server(ex, max_batch=1000, clock=clk, sleep=clk.sleep)
    srv.run(_reqs([0.0, 0.01, 0.02, 0.03, 0.04], nshots=4))
    sizes = [len(b) for (_, _, b) in ex.launched]
    assert max(sizes) * 4 <= 10 and srv.rejected_waits > 0


def test_lanes_run_concurrently_and_shapes_do_not_mix():
    clk = Clock()
    ex = FakeExecutor(clk, [("a", 0), ("a", 1), ("b", 0)], rate=4e8)
    srv = Server(ex, max_batch=1, clock=clk, sleep=clk.sleep)
    reqs = _reqs([0.0, 0.0, 0.0], "a") + [Request(rid=10, arrival=0.0, shape="b", shots=[0, 1, 2, 3])]
    done = srv.run(reqs)
    starts = {r.rid: r.started for r in done}
    assert starts[0] == starts[1] == starts[10]           # two lanes of "a" and the lane of "b"
    for lane, _, rids in ex.launched:
        shapes = {("b" if rid == 10 else "a") for rid in rids}
        assert shapes == {lane[0]}


def test_only_requests_of_one_operator_and_shot_set_share_a_batch():
    """A batch shares one background sweep: same shape, operator and shot set."""
    clk = Clock()
    ex = FakeExecutor(clk, [("a", 0)], rate=4e8)
    reqs = (_reqs([0.0], op="H") + _reqs([0.01], op="F", rid0=1) + _reqs([0.02], op="H", nshots=8, rid0=2)
            + _reqs([0.03, 0.04], op="H", rid0=3) + _reqs([0.05], op="Fadj", rid0=5))
    srv = Server(ex, max_batch=16, clock=clk, sleep=clk.sleep)
    done = srv.run(reqs)
    assert len(done) == 6
    batches = [b for (_, _, b) in ex.launched]
    assert batches[0] == [0]                 # alone: nothing else had arrived
    assert batches[1] == [1]                 # the oldest waiting request leads (F)
    assert batches[2] == [2]                 # H over 8 shots: another shot set
    assert batches[3] == [3, 4]              # H over the 4-shot set, together
    assert batches[4] == [5]
    for b in batches:
        assert len({(reqs[i].op, tuple(reqs[i].shots)) for i in b}) == 1


def test_poisson_stream_is_seeded_and_summary_percentiles():
    shapes = {"s": {16: list(range(16)), 32: list(range(16, 48))}}
    a = poisson_requests(20.0, 5.0, shapes, (16, 32), seed=13)
    b = poisson_requests(20.0, 5.0, shapes, (16, 32), seed=13)
    assert [r.arrival for r in a] == [r.arrival for r in b]
    assert 60 <= len(a) <= 140                            # ~100 expected
    assert all(len(r.shots) in (16, 32) for r in a)
    m = poisson_requests(20.0, 5.0, shapes, (16, 32), seed=13, ops=("H", "F", "Fadj"))
    assert {r.op for r in m} == {"H", "F", "Fadj"}
    for i, r in enumerate(a):
        r.finished = r.arrival + 0.01 * (i % 10 + 1)
        r.cell_steps = 1e9
    s = summarize(a)
    assert s["p50_s"] <= s["p99_s"] <= 0.1 + 1e-12
    assert s["requests"] == len(a)
