"""Continuous batching of F, F* and H requests on one GPU.

Requests (apply F, F* or H = F*F on one of several grid shapes, over one of the
shape's shot sets) arrive over time.  The server keeps one resident context per
(shape, lane): the background model, its damping tables and the wavefield,
checkpoint and image stores stay on the device between requests.  A lane runs
one batch at a time on its own HIP stream; lanes of different shapes (and
several lanes of one shape) run concurrently, so work of requests that arrive
while others are on the GPU overlaps on the device.

Scheduling loop (event driven, one host thread):
  * arrivals enter a FIFO queue;
  * finished batches are retired (completion time = when the host sees the
    batch's event complete) and their lanes freed;
  * each idle lane takes the oldest queued request of its shape and every
    other queued request of the same operator and shot set, in arrival order,
    while the batch's device footprint (mp_footprint_batch: the shared
    background's fields, slots and checkpoints plus each request's wavefields,
    data and images) fits the lane's share of the HBM budget and the batch
    stays under max_batch -- admission by footprint;
  * the batch is one mp_apply_batch call: the background of each shot is
    propagated (and recomputed from its checkpoints) once for the whole batch,
    the requests' Born and adjoint fields run in the same launches, and every
    request's result is bit-identical alone and in any batch.

The executor is pluggable so that the scheduling logic can be exercised on
the CPU with simulated service times (tests); the GPU executor is the only
one that computes.
"""
import collections
import math
import time
from dataclasses import dataclass
from typing import Any, List, Optional


@dataclass
class Request:
    rid: int
    arrival: float                  # seconds since the start of the run
    shape: Any                      # key of the server's shapes
    shots: List[int]                # acquisition shot indices of the shape
    op: str = "H"                   # "F", "Fadj" or "H"
    x: Any = None                   # input (device tensor): model for F / H, data for Fadj
    cell_steps: float = 0.0
    admitted: Optional[float] = None
    started: Optional[float] = None
    finished: Optional[float] = None
    result: Any = None
    batch: int = -1

    @property
    def latency(self):
        return None if self.finished is None else self.finished - self.arrival

    @property
    def key(self):
        """Requests with equal keys share a background sweep."""
        return (self.shape, self.op, tuple(self.shots))


class GpuExecutor:
    """Runs batches with mp_apply_batch on per-lane contexts and streams."""

    def __init__(self, shapes, lanes_per_shape=2, budget_bytes=0, device="cuda:0"):
        import torch

        from .problem import Problem
        self.torch = torch
        self.lanes = {}
        self.specs = {}
        nlanes = lanes_per_shape * len(shapes)
        per_lane = (budget_bytes // nlanes) if budget_bytes else 0
        for key, (spec, c) in shapes.items():
            self.specs[key] = spec
            for j in range(lanes_per_shape):
                P = Problem.from_spec(spec, budget_bytes=per_lane, device=device)
                st = torch.cuda.Stream(device=device)
                with torch.cuda.stream(st):
                    P.set_background(torch.as_tensor(c).to(device), stream=st)
                self.lanes[(key, j)] = dict(problem=P, stream=st, budget=per_lane)

    def lane_keys(self):
        return list(self.lanes.keys())

    def footprint(self, lane, op, nshots, nreq):
        return self.lanes[lane]["problem"].footprint_batch(op, nshots, nreq)

    def lane_budget(self, lane):
        b = self.lanes[lane]["budget"]
        return b if b else float("inf")

    def cell_steps(self, shape, nshots):
        s = self.specs[shape]
        return s.prop_cells * s.nt * nshots

    def launch(self, lane, reqs):
        torch = self.torch
        L = self.lanes[lane]
        st = L["stream"]
        r0 = reqs[0]
        with torch.cuda.stream(st):
            outs = L["problem"].apply_batch(r0.op, [r.x for r in reqs], r0.shots, stream=st)
            ev = torch.cuda.Event()
            ev.record(st)
        for r, o in zip(reqs, outs):
            r.result = o
        return ev

    def done(self, handle):
        return handle.query()

    def wait(self, handle):
        handle.synchronize()


class Server:
    def __init__(self, executor, max_batch=16, clock=time.perf_counter, sleep=time.sleep):
        self.ex = executor
        self.max_batch = max_batch
        self.clock = clock
        self.sleep = sleep
        self.queue = collections.OrderedDict()       # rid -> Request
        self.busy = {}                               # lane -> (handle, reqs)
        self.done: List[Request] = []
        self.nbatches = 0
        self.rejected_waits = 0

    def _form_batch(self, lane, now):
        shape = lane[0]
        budget = self.ex.lane_budget(lane)
        head = next((r for r in self.queue.values() if r.shape == shape), None)
        if head is None:
            return []
        batch = [head]
        for r in self.queue.values():
            if r is head or r.key != head.key:
                continue
            if len(batch) >= self.max_batch:
                break
            if self.ex.footprint(lane, r.op, len(r.shots), len(batch) + 1) > budget:
                self.rejected_waits += 1
                break
            batch.append(r)
        for r in batch:
            del self.queue[r.rid]
            r.admitted = now
        return batch

    def run(self, requests, t_end=None):
        """Serve requests (sorted by arrival) in real time; returns the finished requests."""
        pending = sorted(requests, key=lambda r: r.arrival)
        i = 0
        t0 = self.clock()
        while i < len(pending) or self.queue or self.busy:
            now = self.clock() - t0
            while i < len(pending) and pending[i].arrival <= now:
                r = pending[i]
                r.cell_steps = self.ex.cell_steps(r.shape, len(r.shots))
                self.queue[r.rid] = r
                i += 1
            for lane, (h, reqs) in list(self.busy.items()):
                if self.ex.done(h):
                    tf = self.clock() - t0
                    for r in reqs:
                        r.finished = tf
                        self.done.append(r)
                    del self.busy[lane]
            progressed = False
            for lane in self.ex.lane_keys():
                if lane in self.busy or not self.queue:
                    continue
                batch = self._form_batch(lane, now)
                if not batch:
                    continue
                for r in batch:
                    r.started = now
                    r.batch = self.nbatches
                self.busy[lane] = (self.ex.launch(lane, batch), batch)
                self.nbatches += 1
                progressed = True
            if not progressed:
                nxt = pending[i].arrival - (self.clock() - t0) if i < len(pending) else 0.0
                self.sleep(min(max(nxt, 0.0), 2e-4) if (self.busy or i < len(pending)) else 0.0)
        return self.done


def poisson_requests(rate, duration, shapes, shot_choices, seed, make_x=None, ops=("H",)):
    """Seeded open-loop Poisson arrivals: shape uniform over `shapes`, shot set
    uniform over `shot_choices` (shapes[shape][n]: the shape's set of n shots),
    operator uniform over `ops`; make_x(request) builds the request's input."""
    from fixtures.rng import Stream  # input generator, not method arithmetic
    st = Stream(seed)
    t, rid, out = 0.0, 0, []
    keys = list(shapes)
    while True:
        t += -math.log1p(-float(st.uniform(1)[0])) / rate
        if t > duration:
            break
        shape = keys[int(st.uniform(1)[0] * len(keys)) % len(keys)]
        ns = shot_choices[int(st.uniform(1)[0] * len(shot_choices)) % len(shot_choices)]
        op = ops[int(st.uniform(1)[0] * len(ops)) % len(ops)] if len(ops) > 1 else ops[0]
        r = Request(rid=rid, arrival=t, shape=shape, shots=list(shapes[shape][ns]), op=op)
        if make_x is not None:
            r.x = make_x(r)
        out.append(r)
        rid += 1
    return out


def summarize(reqs, warmup=0.0, wall=None):
    lat = sorted(r.latency for r in reqs if r.finished is not None and r.arrival >= warmup)
    if not lat:
        return {}
    def pct(p):
        k = min(len(lat) - 1, max(0, int(math.ceil(p / 100.0 * len(lat))) - 1))
        return lat[k]
    span = wall if wall is not None else max(r.finished for r in reqs) - min(r.arrival for r in reqs)
    cs = sum(r.cell_steps for r in reqs if r.finished is not None)
    return {"requests": len(reqs), "p50_s": pct(50), "p99_s": pct(99), "mean_s": sum(lat) / len(lat),
            "gcell_steps_per_s": cs / span / 1e9 if span > 0 else None, "span_s": span}
