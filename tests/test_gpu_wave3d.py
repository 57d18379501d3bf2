"""Parity of the 3D HIP sweeps (through the C ABI) against the FP64 oracle."""
import numpy as np
import pytest

import fixtures as F
from fixtures.configs import Workload
from oracle import Problem as Oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1101_3615_amd as M
    return M


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return 0.0 if np.linalg.norm(a) == 0.0 else float("inf")
    return float(np.linalg.norm(a - b) / nb)


class _env:
    """Set environment knobs of the engine for one block (read at create / plan time)."""

    def __init__(self, **kw):
        self.kw = {k: str(v) for k, v in kw.items()}

    def __enter__(self):
        import os
        self.old = {k: os.environ.get(k) for k in self.kw}
        os.environ.update(self.kw)

    def __exit__(self, *a):
        import os
        for k, v in self.old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def cube(dtype="f64", nx=100, ny=22, nz=18, nb=8, nt=60, ns=2, snap="full", k=0):
    """Two 64-cell x tiles, two 16-row y tiles and several z chunks, all ragged."""
    src = np.array([[3, 5, 0], [nx - 2, ny // 2, 2]], np.int32)[:ns]
    rx, ry = np.meshgrid(np.arange(0, nx, 7), np.arange(1, ny, 5))
    rec = np.stack([rx.ravel(), ry.ravel(), np.zeros(rx.size, int)], 1).astype(np.int32)
    rec = np.concatenate([rec, np.array([[nx - 1, ny - 1, nz - 1]], np.int32)])
    return Workload(name="cube", ndim=3, nx=nx, ny=ny, nz=nz, h=12.5, nb=nb, dt=1.0e-3, nt=nt,
                    f_peak=15.0, src=src, rec=rec, dtype=dtype, snap=snap, ckpt_every=k,
                    medium=dict(kind="smooth_random", cmin=1500.0, cmax=3500.0, corr=60.0, seed=41))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_3d_operators_match_oracle(dtype):
    M = _gpu()
    w = cube(dtype)
    c = F.medium(w)
    P = M.Problem.from_spec(w)
    P.set_background(torch.from_numpy(c))
    O = Oracle(w, c)
    tol = 1e-10 if dtype == "f64" else 1e-5
    dm = F.normal_field(w.model_shape, 51)
    d = F.normal_field((w.ns, w.nt, w.nr), 52)
    assert rel(P.apply_F(torch.from_numpy(dm)).cpu().numpy(), O.apply_F(dm)) <= tol
    assert rel(P.apply_Fadj(torch.from_numpy(d)).cpu().numpy(), O.apply_Fadj(d)) <= tol
    assert rel(P.apply_H(torch.from_numpy(dm)).cpu().numpy(), O.apply_H(dm)) <= tol
    # resident background reused by the second call, bit for bit
    again = P.apply_H(torch.from_numpy(dm)).cpu().numpy()
    assert P.stats()["background_cached"]
    assert np.array_equal(again, P.apply_H(torch.from_numpy(dm)).cpu().numpy())


def test_3d_dot_product_f32():
    M = _gpu()
    w = cube("f32", nt=50)
    c = F.medium(w)
    P = M.Problem.from_spec(w)
    P.set_background(torch.from_numpy(c))
    m = F.normal_field(w.model_shape, 53)
    d = F.normal_field((w.ns, w.nt, w.nr), 54)
    lhs = np.sum(P.apply_F(torch.from_numpy(m)).double().cpu().numpy() * d)
    rhs = np.sum(m * P.apply_Fadj(torch.from_numpy(d)).double().cpu().numpy())
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


@pytest.mark.parametrize("snap,tol", [("ckpt_bf16", 1e-2), ("ckpt_f32", 1e-5)])
def test_3d_checkpoints(snap, tol):
    """Checkpoints every 8 steps on the ragged cube (70 steps): apply_H and apply_Fadj
    against the FP64 oracle, BF16 at the stated 1e-2 bound (measured 7.1e-3 for H), FP32
    at 1e-5."""
    M = _gpu()
    w = cube("f32", nt=70, snap=snap, k=8)
    c = F.medium(w)
    P = M.Problem.from_spec(w)
    P.set_background(torch.from_numpy(c))
    O = Oracle(w, c)
    dm = F.normal_field(w.model_shape, 55)
    err = rel(P.apply_H(torch.from_numpy(dm)).cpu().numpy(), O.apply_H(dm))
    d = F.bandlimited_data((w.ns, w.nt, w.nr), 56, w.dt, w.f_peak)
    errA = rel(P.apply_Fadj(torch.from_numpy(d)).cpu().numpy(), O.apply_Fadj(d))
    print(f"3D {snap} every 8, 70 steps: apply_H {err:.3e}, apply_Fadj {errA:.3e} vs FP64 oracle")
    assert err <= tol and errA <= tol


def test_3d_odd_shot_count_and_batches():
    """Three shots: the device images shots in pairs, so the job is padded with a null shot
    (no source, no data); apply_F / Fadj / H still match the oracle, and apply_H_batch gives
    each request (one and two shots) the same bits alone and in the mix."""
    M = _gpu()
    w = cube("f32", nt=50)
    w = w.with_(src=np.array([[3, 5, 0], [w.nx - 2, w.ny // 2, 2], [50, 11, 9]], np.int32))
    c = F.medium(w)
    P = M.Problem.from_spec(w)
    P.set_background(torch.from_numpy(c))
    O = Oracle(w, c)
    dm = F.normal_field(w.model_shape, 61)
    d = F.normal_field((w.ns, w.nt, w.nr), 62)
    assert rel(P.apply_F(torch.from_numpy(dm)).cpu().numpy(), O.apply_F(dm)) <= 1e-5
    assert rel(P.apply_Fadj(torch.from_numpy(d)).cpu().numpy(), O.apply_Fadj(d)) <= 1e-5
    assert rel(P.apply_H(torch.from_numpy(dm)).cpu().numpy(), O.apply_H(dm)) <= 1e-5
    lists = [[2], [0, 1]]
    dms = [F.normal_field(w.model_shape, 63 + i) for i in range(2)]
    mixed = [o.cpu().numpy() for o in P.apply_H_batch([torch.from_numpy(x) for x in dms], lists)]
    for i, (sl, x) in enumerate(zip(lists, dms)):
        alone = P.apply_H_batch([torch.from_numpy(x)], [sl])[0].cpu().numpy()
        assert np.array_equal(alone, mixed[i])
        assert rel(mixed[i], Oracle(w.with_(src=w.src[sl]), c).apply_H(x)) <= 1e-5


@pytest.mark.parametrize("zc", [None, 34])
@pytest.mark.parametrize("snap,k", [("full", 0), ("ckpt_bf16", 8), ("ckpt_bf16", 1), ("ckpt_f32", 8),
                                    ("ckpt_f32", 1)])
def test_3d_repeatable(snap, k, zc):
    """Repeated calls give the same bits (ten calls of F, two of H), with the engine's
    z chunking and with one chunk per tile: a regression test for the 16-byte field stores,
    which took later register values (the odd shot of a pair differed between calls)
    while their uniform offset sat in SOFFSET."""
    M = _gpu()
    w = cube("f32", nt=40, snap=snap, k=k)
    c = F.medium(w)
    with _env(**({"MP_ZC": zc} if zc else {})):
        P = M.Problem.from_spec(w)
    P.set_background(torch.from_numpy(c))
    dm = torch.from_numpy(F.normal_field(w.model_shape, 57))
    first = P.apply_F(dm).cpu().numpy()
    for _ in range(9):
        assert np.array_equal(P.apply_F(dm).cpu().numpy(), first)
    h = P.apply_H(dm).cpu().numpy()
    assert np.array_equal(P.apply_H(dm).cpu().numpy(), h)


def test_c5_reduced_parity():
    """The 256^3 workload's configuration (FP32 fields, BF16 checkpoints every 8 steps, nb 20,
    its medium and surface acquisition) on a 48^3 model, 200 steps, two shots: apply_H
    against the FP64 oracle within the BF16 bound (1e-2)."""
    M = _gpu()
    w5 = F.c5()
    r = np.arange(2, 48, 4)
    rx, ry = np.meshgrid(r, r)
    w = w5.with_(nx=48, ny=48, nz=48, nt=200,
                 src=np.array([[12, 12, 0], [36, 30, 0]], np.int32),
                 rec=np.stack([rx.ravel(), ry.ravel(), np.zeros(rx.size, int)], 1).astype(np.int32))
    c = F.medium(w)
    P = M.Problem.from_spec(w)
    P.set_background(torch.from_numpy(c))
    y = F.normal_field(w.model_shape, 57)
    got = P.apply_H(torch.from_numpy(y)).cpu().numpy()
    err = rel(got, Oracle(w, c).apply_H(y))
    print(f"48^3 BF16 ckpt/8: apply_H rel L2 vs FP64 oracle = {err:.3e}")
    assert err <= 1e-2


def test_c5_full_size_dot_product():
    """At the full 256^3 spatial size (296^3 propagation grid), two shots and 40 steps with
    FP32 fields: <F m, d> = <m, F* d> to FP32 rounding."""
    M = _gpu()
    w = F.c5()
    w = w.with_(nt=40, snap="full", ckpt_every=0, src=np.asarray(w.src)[:2])
    c = F.medium(w)
    P = M.Problem.from_spec(w)
    P.set_background(torch.from_numpy(c))
    m = torch.from_numpy(F.normal_field(w.model_shape, 55))
    d = torch.from_numpy(F.normal_field((w.ns, w.nt, w.nr), 56))
    Fm = P.apply_F(m).double()
    lhs = float((Fm * d.to(Fm.device).double()).sum())
    Fd = P.apply_Fadj(d).double()
    rhs = float((m.to(Fd.device).double() * Fd).sum())
    print(f"256^3 dot product: {abs(lhs - rhs) / abs(lhs):.3e}")
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


@pytest.mark.parametrize("snap,k", [("full", 0), ("ckpt_bf16", 4)])
def test_3d_zero_inputs_give_exact_zeros(snap, k):
    """Linear operators: zero in, exactly zero out, after a nonzero call on the same context."""
    M = _gpu()
    w = cube("f32", nt=40, snap=snap, k=k)
    P = M.Problem.from_spec(w)
    P.set_background(torch.from_numpy(F.medium(w)))
    P.apply_H(torch.from_numpy(F.normal_field(w.model_shape, 53)))
    zm = torch.zeros(w.model_shape)
    assert not torch.any(P.apply_H(zm).cpu())
    assert not torch.any(P.apply_F(zm).cpu())
    assert not torch.any(P.apply_Fadj(torch.zeros((w.ns, w.nt, w.nr))).cpu())


def _many_shot_cube(dtype, snap, k, nt=40):
    """64 shots on an 8 x 8 lattice over a 64 x 64 x 48 model (nb 8): 32 pairs x 10 tiles.

    With one z chunk per tile that is 320 workgroup items, more than the 256
    workgroups resident at once, so every persistent workgroup walks more than one
    item, as in the full-size launches.
    """
    sx, sy = np.meshgrid(4 + 8 * np.arange(8), 4 + 8 * np.arange(8))
    src = np.stack([sx.ravel(), sy.ravel(), np.zeros(64, int)], 1).astype(np.int32)
    rx, ry = np.meshgrid(np.arange(1, 64, 3), np.arange(2, 64, 3))
    rec = np.stack([rx.ravel(), ry.ravel(), np.zeros(rx.size, int)], 1).astype(np.int32)
    return Workload(name="lattice", ndim=3, nx=64, ny=64, nz=48, h=12.5, nb=8, dt=1.0e-3, nt=nt,
                    f_peak=15.0, src=src, rec=rec, dtype=dtype, snap=snap, ckpt_every=k,
                    medium=dict(kind="smooth_random", cmin=1500.0, cmax=3500.0, corr=60.0, seed=43))


SAMPLED = [0, 1, 33, 62, 63]


@pytest.mark.parametrize("snap,k", [("full", 0), ("ckpt_bf16", 8)])
def test_3d_one_chunk_persistent_rounds_against_oracle(snap, k):
    """One z chunk per tile and several items per persistent workgroup (the launch
    shape of the full-size workload): apply_F on sampled shots of both halves of
    pairs, first and last pair, against the oracle; apply_Fadj of data that is
    nonzero on those shots only; and the default z chunking gives the same bits."""
    M = _gpu()
    w = _many_shot_cube("f32", snap, k)
    c = F.medium(w)
    O = Oracle(w, c)
    dm = F.normal_field(w.model_shape, 57)
    d = np.zeros((w.ns, w.nt, w.nr), np.float32)
    d[SAMPLED] = F.bandlimited_data((len(SAMPLED), w.nt, w.nr), 58, w.dt, w.f_peak)
    outs = {}
    for zc in (w.nz + 2 * w.nb, None):
        kw = {"MP_ZC": zc} if zc else {}
        with _env(**kw):
            P = M.Problem.from_spec(w)
        P.set_background(torch.from_numpy(c))
        outs[zc] = (P.apply_F(torch.from_numpy(dm)).cpu().numpy(), P.apply_Fadj(torch.from_numpy(d)).cpu().numpy())
    one, dflt = outs[w.nz + 2 * w.nb], outs[None]
    assert np.array_equal(one[0], dflt[0]) and np.array_equal(one[1], dflt[1])
    ref_F = np.stack([O.born(s, dm, O.background(s)[0]) for s in SAMPLED])
    err_F = rel(one[0][SAMPLED], ref_F)
    ref_A = None
    for s in SAMPLED:
        g, _ = O.background(s)
        part = O.adjoint(s, d[s].astype(np.float64), g)
        ref_A = part if ref_A is None else ref_A + part
    err_A = rel(one[1], ref_A)
    print(f"64 shots, one chunk per tile, {snap}: apply_F (5 shots) {err_F:.3e}, apply_Fadj {err_A:.3e}")
    assert err_F <= 1e-5                     # F never reads a checkpoint
    if snap == "full":
        assert err_A <= 1e-5


def test_c5_full_shape_sampled_shot_against_oracle():
    """The 256^3 workload's own launch shape: all 32 shots in waves of 8 (what the
    2000-step checkpoint footprint allows), the engine's z chunking, at the full 296^3
    propagation grid; 16 steps (two checkpoint segments).  Shot 31 (odd half of the last pair of the last wave): its Born
    traces against the oracle, and F* of data nonzero on that shot only, with the
    workload's BF16 checkpoints (1e-2) and with the full FP32 history (1e-5)."""
    M = _gpu()
    w = F.c5().with_(nt=16)
    c = F.medium(w)
    dm = F.normal_field(w.model_shape, 61)
    s = 31
    d = np.zeros((w.ns, w.nt, w.nr), np.float32)
    d[s] = F.bandlimited_data((1, w.nt, w.nr), 62, w.dt, w.f_peak)[0]
    got = {}
    with _env(MP_MAX_WAVE=8):
        for snap in ("ckpt_bf16", "full"):
            P = M.Problem.from_spec(w, snap=snap, ckpt_every=(8 if snap == "ckpt_bf16" else 0))
            P.set_background(torch.from_numpy(c))
            got[snap] = (P.apply_F(torch.from_numpy(dm))[s].cpu().numpy(),
                         P.apply_Fadj(torch.from_numpy(d)).cpu().numpy())
            assert P.stats()["waves"] == 4
            P.close()
            del P
    O = Oracle(w, c)
    g, _ = O.background(s)
    ref_F = O.born(s, dm, g)
    ref_A = O.adjoint(s, d[s].astype(np.float64), g)
    for snap, tol in (("ckpt_bf16", 1e-2), ("full", 1e-5)):
        err_F, err_A = rel(got[snap][0], ref_F), rel(got[snap][1], ref_A)
        print(f"256^3 workload, waves of 8, shot {s}, {snap}: apply_F {err_F:.3e}, apply_Fadj {err_A:.3e}")
        assert err_F <= 1e-5
        assert err_A <= tol


@pytest.mark.parametrize("snap,k", [("full", 0), ("ckpt_bf16", 8), ("ckpt_f32", 1)])
def test_3d_z_chunk_heights_give_the_same_bits(snap, k):
    """Forced z-chunk heights on the 34-plane propagation grid of the cube: 4 planes (9
    chunks, the last two planes), 6 (6 chunks, the last one, with z decreasing, four planes)
    and 9 (4 chunks, the last with z decreasing) against one chunk per tile: odd chunks
    march with z decreasing and even ones with z increasing, and no bit of F, F* or H may depend on it."""
    M = _gpu()
    w = cube("f32", nt=40, snap=snap, k=k)
    c = F.medium(w)
    dm = torch.from_numpy(F.normal_field(w.model_shape, 57))
    d = torch.from_numpy(F.normal_field((w.ns, w.nt, w.nr), 58))
    outs = {}
    for zc in (4, 6, 9, 34):
        with _env(MP_ZC=zc):
            P = M.Problem.from_spec(w)
        P.set_background(torch.from_numpy(c))
        outs[zc] = [P.apply_F(dm).cpu().numpy(), P.apply_Fadj(d).cpu().numpy(), P.apply_H(dm).cpu().numpy()]
        P.close()
    for zc in (4, 6, 9):
        for name, a, b in zip(("F", "F*", "H"), outs[zc], outs[34]):
            assert np.array_equal(a, b), f"{name} with chunk height {zc} differs from one chunk"


@pytest.mark.parametrize("snap,k", [("full", 0), ("ckpt_bf16", 8)])
def test_3d_wave_sizes_give_the_same_bits(snap, k):
    """Six shots in waves of 2, 4 (4 + 2) and 6: the job's images are stacked per pair
    of shots and summed in one fixed order, so no bit of F, F* or H may depend on how
    the shots are split into waves; the three-wave F* matches the oracle."""
    M = _gpu()
    w = cube("f32", nt=40, snap=snap, k=k)
    w = w.with_(src=np.array([[3, 5, 0], [w.nx - 2, w.ny // 2, 2], [50, 11, 9], [20, 3, 4], [70, 18, 1],
                              [90, 7, 12]], np.int32))
    c = F.medium(w)
    dm = torch.from_numpy(F.normal_field(w.model_shape, 71))
    d = torch.from_numpy(F.normal_field((w.ns, w.nt, w.nr), 72))
    outs = {}
    for wave in (2, 4, 6):
        with _env(MP_MAX_WAVE=wave):
            P = M.Problem.from_spec(w)
            P.set_background(torch.from_numpy(c))
            outs[wave] = [P.apply_F(dm).cpu().numpy(), P.apply_Fadj(d).cpu().numpy(), P.apply_H(dm).cpu().numpy()]
            assert P.stats()["waves"] == 6 // wave + (6 % wave > 0)
            P.close()
    for wave in (2, 4):
        for name, a, b in zip(("F", "F*", "H"), outs[wave], outs[6]):
            assert np.array_equal(a, b), f"{name} in waves of {wave} differs from one wave"
    tol = 1e-5 if snap == "full" else 1e-2
    assert rel(outs[2][1], Oracle(w, c).apply_Fadj(d.numpy())) <= tol


def test_3d_long_record_fp32_against_oracle():
    """FP32 fields over a 400-step record on the ragged cube (the waves cross the grid
    and return through the layers): F, F* and H stay within the FP32 bound of the FP64
    oracle (measured 5.4e-6, 5.1e-6 and 2.4e-6; the error grows with the record)."""
    M = _gpu()
    w = cube("f32", nt=400)
    c = F.medium(w)
    P = M.Problem.from_spec(w)
    P.set_background(torch.from_numpy(c))
    O = Oracle(w, c)
    dm = F.normal_field(w.model_shape, 51)
    d = F.normal_field((w.ns, w.nt, w.nr), 52)
    eF = rel(P.apply_F(torch.from_numpy(dm)).cpu().numpy(), O.apply_F(dm))
    eA = rel(P.apply_Fadj(torch.from_numpy(d)).cpu().numpy(), O.apply_Fadj(d))
    eH = rel(P.apply_H(torch.from_numpy(dm)).cpu().numpy(), O.apply_H(dm))
    print(f"3D FP32, 400 steps: apply_F {eF:.3e}, apply_Fadj {eA:.3e}, apply_H {eH:.3e} vs FP64 oracle")
    assert max(eF, eA, eH) <= 1e-5
