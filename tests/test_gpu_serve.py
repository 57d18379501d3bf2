"""Serving on the GPU: shared-background batches of F, F* and H (mp_apply_batch) and the
continuous-batching loop over the three serving grid shapes (FP32 fields, BF16
checkpoints every 4 steps).  Every request's result must be the same alone, in a batch
and in the served mix (bitwise here; the stated tolerance is 1e-6 relative), and
batched results must match the FP64 oracle: F within 1e-5 (it reads no checkpoint),
F* and H within the BF16 bound 1e-2."""
import numpy as np
import pytest

import fixtures as F
from oracle import Problem as Oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1101_3615_amd as M
    return M


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def _inputs(op, w, c, shots, seeds):
    if op == "Fadj":
        return [torch.from_numpy(F.bandlimited_data((len(shots), w.nt, w.nr), s, w.dt, w.f_peak)) for s in seeds]
    if w.ndim == 3:   # the ragged cube is too small for wavepackets
        return [torch.from_numpy(F.normal_field(w.model_shape, s)) for s in seeds]
    return [torch.from_numpy(F.wavepackets(w, c, s, 8)) for s in seeds]


def _oracle(op, O, x):
    x = x.double().numpy()
    return O.apply_F(x) if op == "F" else O.apply_Fadj(x) if op == "Fadj" else O.apply_H(x)


@pytest.mark.parametrize("op", ["F", "Fadj", "H"])
def test_apply_batch_2d_alone_mix_and_oracle(op):
    """Three requests over four shots of the 256 x 128 serving shape, 400 steps (the
    wavefield crosses the grid): batched == alone bit for bit, and the oracle."""
    M = _gpu()
    w, groups = F.c4_union(256, 128, 10)
    w = w.with_(nt=400)
    c = F.medium(w)
    P = M.Problem.from_spec(w)
    P.set_background(torch.from_numpy(c))
    shots = list(groups[16][::4])
    xs = _inputs(op, w, c, shots, (201, 202, 203))
    mixed = [o.cpu() for o in P.apply_batch(op, xs, shots)]
    for x, m in zip(xs, mixed):
        alone = P.apply_batch(op, [x], shots)[0].cpu()
        assert torch.equal(alone, m)
    O = Oracle(w.with_(src=w.src[shots]), c)
    err = rel(mixed[1].numpy(), _oracle(op, O, xs[1]))
    print(f"256x128, 400 steps, 4 shots, BF16 ckpt/4, batched {op}: rel L2 vs FP64 oracle {err:.3e}")
    assert err <= (1e-5 if op == "F" else 1e-2)


@pytest.mark.parametrize("snap,k", [("full", 0), ("ckpt_bf16", 8)])
@pytest.mark.parametrize("op", ["F", "Fadj", "H"])
def test_apply_batch_3d_alone_mix_and_oracle(op, snap, k):
    """The same on the ragged 3D cube (shot pairs, separate background and Born launches)."""
    M = _gpu()
    import sys, os
    sys.path.insert(0, os.path.dirname(__file__))
    from test_gpu_wave3d import cube
    w = cube("f32", nt=60, snap=snap, k=k)
    c = F.medium(w)
    P = M.Problem.from_spec(w)
    P.set_background(torch.from_numpy(c))
    shots = [1, 0, 1]
    xs = _inputs(op, w, c, shots, (211, 212))
    mixed = [o.cpu() for o in P.apply_batch(op, xs, shots)]
    for x, m in zip(xs, mixed):
        assert torch.equal(P.apply_batch(op, [x], shots)[0].cpu(), m)
    O = Oracle(w.with_(src=w.src[shots]), c)
    err = rel(mixed[0].numpy(), _oracle(op, O, xs[0]))
    print(f"3D cube, {snap}, batched {op}: rel L2 vs FP64 oracle {err:.3e}")
    assert err <= (1e-5 if (op == "F" or snap == "full") else 1e-2)


def test_apply_batch_refuses_what_does_not_fit():
    """A budget that holds the shared background and one request's fields refuses four."""
    M = _gpu()
    w, groups = F.c4_union(256, 128, 10)
    c = F.medium(w)
    shots = list(groups[16])
    Q = M.Problem.from_spec(w)
    one, four = Q.footprint_batch("H", len(shots), 1), Q.footprint_batch("H", len(shots), 4)
    assert four > one
    P = M.Problem.from_spec(w, budget_bytes=(one + four) // 2)
    P.set_background(torch.from_numpy(c))
    xs = _inputs("H", w, c, shots, (1, 2, 3, 4))
    with pytest.raises(M.MatprobeError):
        P.apply_batch("H", xs, shots)
    out = P.apply_batch("H", xs[:1], shots)[0].cpu()   # one request still fits
    Q.set_background(torch.from_numpy(c))
    assert torch.equal(out, Q.apply_batch("H", xs[:1], shots)[0].cpu())


def test_served_mix_matches_alone():
    """A Poisson stream of F, F* and H requests on the three serving shapes: every
    request's result equals the same request submitted alone, bit for bit."""
    M = _gpu()
    from paper_1101_3615_amd.serve import GpuExecutor, Server, poisson_requests, summarize
    shapes, groups = {}, {}
    for (nx, nz), seed in zip(F.SERVE_SHAPES, (10, 11, 12)):
        w, g = F.c4_union(nx, nz, seed)
        shapes[(nx, nz)] = (w, F.medium(w))
        groups[(nx, nz)] = g
    ex = GpuExecutor(shapes, lanes_per_shape=2)

    def make_x(r):
        w, c = shapes[r.shape]
        if r.op == "Fadj":
            return torch.from_numpy(F.bandlimited_data((len(r.shots), w.nt, w.nr), 1000 + r.rid, w.dt,
                                                       w.f_peak)).cuda()
        return torch.from_numpy(F.wavepackets(w, c, 1000 + r.rid, max(1, w.model_cells // 4096))).cuda()

    reqs = poisson_requests(200.0, 0.4, groups, F.SERVE_SHOTS, seed=13, make_x=make_x, ops=("H", "F", "Fadj"))
    srv = Server(ex, max_batch=16)
    done = srv.run(reqs)
    torch.cuda.synchronize()
    st = summarize(done)
    print(f"{len(done)} requests in {srv.nbatches} batches: p50 {st['p50_s']*1e3:.1f} ms, "
          f"p99 {st['p99_s']*1e3:.1f} ms, {st['gcell_steps_per_s']:.1f} Gcell-steps/s")
    assert len(done) == len(reqs)
    assert srv.nbatches < len(reqs)                 # some requests shared a sweep
    assert {r.op for r in done} == {"H", "F", "Fadj"}
    mixed = {r.rid: r.result.clone() for r in done}
    checked = {}
    for r in sorted(done, key=lambda r: r.rid):
        if checked.get(r.op, 0) >= 5:
            continue
        P = ex.lanes[(r.shape, 0)]["problem"]
        alone = P.apply_batch(r.op, [r.x], r.shots)[0]
        torch.cuda.synchronize()
        assert torch.equal(alone, mixed[r.rid]), f"request {r.rid} ({r.op}) differs alone vs in the mix"
        checked[r.op] = checked.get(r.op, 0) + 1
    assert checked == {"H": 5, "F": 5, "Fadj": 5}
