#!/usr/bin/env python3
"""Throughput of the matrix-probing pass on one MI355X.

Workload (default): the 256^3 configuration -- propagation grid 296^3 (20
absorbing cells per side, 12.5 m), 32 surface sources on an 8 x 4 lattice,
64 x 64 receivers, 10 Hz Ricker, dt = 1 ms, FP32 stencils, BF16 checkpoints of
the background every 8 steps with recomputation, FP64 imaging; 4 wavepacket
trial functions of 4096 packets; p = 40 basis terms (Legendre polynomials of
total degree <= 2 in (z, y, x) times rho^0..3); the FP64 least-squares fit on
the GPU; the fitted inverse applied by 3D FFT multipliers.

The record is 2000 steps.  Its checkpoints (25.9 GB per shot) limit a shot wave
to what the device holds: the benchmark computes that wave size from the
library's footprint of the 2000-step job (8 shots on one MI355X, four waves) and
runs every application of H with it.  A step applies H over the first
--record-steps steps of the record (default 40: five checkpoint segments), so
every launch has the shape of the full application; value = apply_H
propagation cell-steps of the step / step time, i.e. the rate of a full
application extrapolated over the record length (--full-record times one
2000-step application to check it).

One step, with every input resident in HBM: set the background; x_t = H y_t for
the 4 trials; the least-squares fit over the 4 x 256^3 stacked rows; the fitted
inverse applied to x_0.

Extra legs on the same line: the 512 x 256 FP32 workload (full 3000-step
record) and the 1024 x 512 BF16-checkpointed workload (400 of its 4000 steps,
waves of 64 shots as at full length), each with its dominant kernel's roofline
fraction; the serving run; the FP64 oracle on a bounded sample of the 256^3
workload as the CPU baseline.

Prints one JSON line (see the keys below).  --gpus must be 1.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


_CPU_INPUT = {}


def _cpu_shot(args):
    """Oracle apply_H of one shot over the first `nsteps` steps (CPU baseline leg)."""
    shot, nsteps = args
    from oracle import Problem
    w, c, y = _CPU_INPUT["w"].with_(nt=nsteps), _CPU_INPUT["c"], _CPU_INPUT["y"]
    P = Problem(w, c)
    t = time.perf_counter()
    P.apply_H(y, shots=[shot])
    return time.perf_counter() - t


def cpu_baseline(w, c, y, nsteps, workers):
    """The FP64 oracle on a bounded sample of workload w (inputs c, y built by the
    caller), one shot per forked process.  Run before anything initialises the GPU."""
    import multiprocessing as mp
    _CPU_INPUT.update(w=w, c=c, y=y)
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        times = pool.map(_cpu_shot, [(s, nsteps) for s in range(workers)])
    wall = max(times)                      # the workers run concurrently
    cell_steps = w.prop_cells * nsteps * workers
    return {"value": cell_steps / wall / 1e9, "unit": "Gcell-steps/s", "cores": workers,
            "kind": "oracle",
            "sample": f"{w.name}: {workers} shots x {nsteps} of {w.nt} steps of apply_H (background, Born and "
                      f"adjoint sweeps), FP64 numpy, one process per shot, slowest worker {wall:.1f} s"}


def kernel_bytes3d(kind, w, nsh):
    """Algorithmic HBM bytes of one launch (one time step) of a 3D sweep kernel over
    nsh shots (FP32 fields, FP64 image), P = propagation cells, M = model cells:
      fused:      per shot reads u, D, du, du^{n-1} and writes u, D, du^{n+1}
                  (28 B per cell); kappa and the perturbation once (8 B per cell);
      background: per shot reads u, D and writes u, D (16 B per cell), writes its slot
                  (the level u^{n+1} while recomputing from checkpoints; 4 B per model
                  cell); kappa once;
      adjoint:    per shot reads nu, nu^{k+2} and writes nu^k (12 B per cell), reads the
                  slot (4 B per model cell), one FP64 image read-modify-write per pair of
                  shots (8 B per model cell and shot); kappa once.
    The BF16 checkpoint writes (4 B per cell every 8th step) and the receiver traffic
    are left out."""
    P, M = w.prop_cells, w.model_cells
    per = {"fused": 28 * P, "background": 16 * P + 4 * M, "adjoint": 12 * P + 4 * M + 8 * M}[kind]
    shared = 8 * P if kind == "fused" else 4 * P
    return per * nsh + shared


def kernel_bytes(kind, w, s=2):
    """Algorithmic HBM bytes of one launch of a 2D sweep kernel that takes s time
    steps (1 or 2) for every shot of the workload (FP32 fields, FP64 image).

    Per shot, a launch reads its two input levels and writes its outputs once on
    the propagation grid, and touches the g store and image on the model grid:
      background: reads u, D and writes u, D (16 B per cell); writes g of each
                  step (4 B per model cell and step);
      Born:       reads du^n, du^{n-1} (8 B per cell), writes s levels (4 B
                  each); reads g of each step (4 B per model cell and step);
      adjoint:    as Born for the field and g, plus one read-modify-write of the
                  FP64 image per group of four shots (16 B per model cell and
                  group, 4 B per shot).
    Shared by all shots and counted once per launch: kappa (4 B per cell) and,
    for the Born kernel, the extended perturbation (4 B per cell).
    """
    e = 4
    prop, model, ns = w.prop_cells, w.model_cells, w.ns
    per = {"background": 4 * e * prop + s * e * model,
           "born": 2 * e * prop + s * e * prop + s * e * model,
           "adjoint": 2 * e * prop + s * e * prop + s * e * model + 4 * model}[kind]
    shared = e * prop * (2 if kind == "born" else 1)
    return per * ns + shared


def _sha(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


TRAFFIC = {"2d": ("traffic.json", "wave2d.hip"), "3d": ("traffic_c5.json", "wave3d.hip"),
           "c3": ("traffic_c3.json", "wave2d.hip")}


# shots per launch of the runs the counter summaries are taken on: the 512 x 256 leg (one
# wave of 64), the 1024 x 512 leg (waves of 64) and the 256^3 benchmark (waves of 8)
LAUNCH_SHOTS = {"2d": 64, "c3": 64, "3d": 8}


def traffic_for(kind, w, nsh):
    """Measured HBM bytes per launch from the committed counter summary, if it was taken
    on this workload, with launches of nsh shots and with the kernel source as it is now
    (else None)."""
    rec_name, src_name = TRAFFIC["3d" if w.ndim == 3 else "c3" if w.name.startswith("c3_") else "2d"]
    try:
        with open(os.path.join(ROOT, "profiles", rec_name)) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    digest = _sha(os.path.join(ROOT, "paper_1101_3615_amd", "csrc", src_name))
    k = rec.get("kernels", {}).get(kind)
    if (not k or rec.get("source_sha256", rec.get("wave2d_sha256")) != digest or rec.get("workload") != w.name
            or rec.get("launch_shots") != nsh):
        return None
    return k.get("bytes_per_launch")


KIND_OF_MODE = {"0": "fused", "1": "born", "2": "background", "3": "adjoint"}


def serve_leg(seconds, rate=20.0, seed=13):
    """Serving workload: seeded Poisson arrivals (rate req/s) of apply_H requests
    on the grids {256x128, 512x256, 1024x512} (records of 104/208/416 steps) with
    16/32/64 shots, FP32 fields and BF16 checkpoints every 4 steps.  Reports
    latency percentiles under the offered load; then the throughput of the same
    requests, and of a stream of F, F* and H requests, submitted at once through
    the continuous-batching server ("served": requests of one operator and shot
    set share a background sweep) versus one request at a time on one stream
    ("plain")."""
    import torch

    import fixtures as F
    from paper_1101_3615_amd.serve import GpuExecutor, Server, poisson_requests, summarize

    shapes, groups = {}, {}
    for (nx, nz), sd in zip(F.SERVE_SHAPES, (10, 11, 12)):
        w, g = F.c4_union(nx, nz, sd)
        shapes[(nx, nz)] = (w, F.medium(w))
        groups[(nx, nz)] = g
    ex = GpuExecutor(shapes, lanes_per_shape=2)

    def make_x(r):
        w, c = shapes[r.shape]
        if r.op == "Fadj":
            return torch.from_numpy(F.bandlimited_data((len(r.shots), w.nt, w.nr), 1000 + r.rid, w.dt,
                                                       w.f_peak)).cuda()
        return torch.from_numpy(F.wavepackets(w, c, 1000 + r.rid, max(1, w.model_cells // 4096))).cuda()

    # warm every lane once per operator (allocations, code objects)
    for lane in ex.lane_keys():
        w, c = shapes[lane[0]]
        for op in ("H", "F", "Fadj"):
            r0 = type("R", (), {"op": op, "shots": [0], "shape": lane[0], "rid": -1})()
            ex.lanes[lane]["problem"].apply_batch(op, [make_x(r0)], [0])
    torch.cuda.synchronize()

    def capacity(reqs):
        for r in reqs:
            r.arrival, r.finished = 0.0, None
        srv = Server(ex, max_batch=16)
        t0 = time.perf_counter()
        srv.run(reqs)
        torch.cuda.synchronize()
        t_served = time.perf_counter() - t0
        t0 = time.perf_counter()
        for r in reqs:
            ex.lanes[(r.shape, 0)]["problem"].apply_batch(r.op, [r.x], r.shots)
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        cs = sum(r.cell_steps for r in reqs)
        return {"requests": len(reqs), "batches": srv.nbatches,
                "served_gcell_steps_per_s": round(cs / t_served / 1e9, 3),
                "plain_gcell_steps_per_s": round(cs / t_plain / 1e9, 3),
                "served_vs_plain": round(t_plain / t_served, 3)}

    reqs = poisson_requests(rate, seconds, groups, F.SERVE_SHOTS, seed=seed, make_x=make_x)
    srv = Server(ex, max_batch=16)
    done = srv.run(reqs)
    torch.cuda.synchronize()
    load = summarize(done, warmup=min(1.0, 0.1 * seconds))
    out = {"requests": len(reqs), "rate_per_s": rate, "seconds": seconds, "ops": "H",
           "steps": {f"{nx}x{nz}": shapes[(nx, nz)][0].nt for (nx, nz) in F.SERVE_SHAPES},
           "batches": srv.nbatches,
           "p50_ms": round(1e3 * load["p50_s"], 3), "p99_ms": round(1e3 * load["p99_s"], 3),
           "offered_gcell_steps_per_s": round(load["gcell_steps_per_s"], 3)}
    out["admission_waits"] = srv.rejected_waits
    out["capacity_H"] = capacity(reqs)
    # offered load over the served capacity of the same requests
    out["rho"] = round(out["offered_gcell_steps_per_s"] / out["capacity_H"]["served_gcell_steps_per_s"], 3)
    mix = poisson_requests(rate, seconds, groups, F.SERVE_SHOTS, seed=seed + 1, make_x=make_x,
                           ops=("H", "F", "Fadj"))
    out["capacity_F_Fadj_H"] = capacity(mix)
    out["served_vs_plain"] = out["capacity_H"]["served_vs_plain"]
    return out


def ingest_counters(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, copy_mib, dims):
    """profiles/traffic.json (dims 2d: the 512 x 256 workload), traffic_c3.json (c3: the
    1024 x 512 checkpointed workload) or traffic_c5.json (3d: the 256^3 workload) from
    two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of a run of that workload and of
    the copy probe: per sweep kind, HBM bytes per launch = mean counter (KiB) x 1024 x
    (copy bytes / the copy kernel's reading of the same counter), averaged over the
    kind's kernel variants (e.g. background launches that store, read or skip
    checkpoints) weighted by their launch counts."""
    import csv
    import glob
    import re

    import fixtures as F

    def sums(d):
        f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0]
        acc = {}
        for r in csv.DictReader(open(f)):
            a = acc.setdefault(r["Kernel_Name"], [0.0, 0])
            a[0] += float(r["Counter_Value"])
            a[1] += 1
        return acc

    copy_bytes = copy_mib * (1 << 20)
    cf = [v[0] / v[1] for k, v in sums(copy_fetch_dir).items() if "copyBuffer" in k][0]
    cw = [v[0] / v[1] for k, v in sums(copy_write_dir).items() if "copyBuffer" in k][0]
    f_fac = copy_bytes / (cf * 1024.0)
    w_fac = copy_bytes / (cw * 1024.0)
    fe, wr = sums(fetch_dir), sums(write_dir)
    acc = {}
    for name in fe:
        if dims == "3d":
            m = re.search(r"k_step3d<float, (\d), (\d)>", name)
            ok = m is not None
        else:
            m = re.search(r"k_sweep2d<float, (\d), (\d), (\d)>", name)
            ok = m is not None and m.group(2) == "2"
        if not ok or name not in wr:
            continue
        a = acc.setdefault(KIND_OF_MODE[m.group(1)], {"kernels": [], "fetch": 0.0, "write": 0.0, "launches": 0})
        a["kernels"].append(name)
        a["fetch"] += fe[name][0]
        a["write"] += wr[name][0]
        a["launches"] += fe[name][1]
    kernels = {}
    for kind, a in acc.items():
        n = a["launches"]
        kernels[kind] = {"kernel": a["kernels"][0] if len(a["kernels"]) == 1 else a["kernels"], "launches": n,
                         "fetch_kib_raw": a["fetch"] / n, "write_kib_raw": a["write"] / n,
                         "bytes_per_launch": (a["fetch"] * f_fac + a["write"] * w_fac) * 1024.0 / n}
    rec_name, src_name = TRAFFIC[dims]
    rec = {"workload": {"3d": F.c5(), "c3": F.c3(), "2d": F.c2()}[dims].name, "launch_shots": LAUNCH_SHOTS[dims],
           "source_sha256": _sha(os.path.join(ROOT, "paper_1101_3615_amd", "csrc", src_name)),
           "fetch_scale": f_fac, "write_scale": w_fac, "copy_probe_bytes": copy_bytes, "kernels": kernels}
    with open(os.path.join(ROOT, "profiles", rec_name), "w") as f:
        json.dump(rec, f, indent=1)
    return rec


def volume_run(nt):
    """apply_H on the 256^3 workload with nt time steps (see apply_H_run)."""
    import fixtures as F
    return apply_H_run(F.c5().with_(nt=nt), volume=True)


def checkpointed_run(nt):
    """apply_H on the 1024 x 512 workload (128 shots, BF16 checkpoints every 4 steps) with
    nt time steps (see apply_H_run)."""
    import fixtures as F
    return apply_H_run(F.c3().with_(nt=nt))


def apply_H_run(w, volume=False):
    """One apply_H on workload w (inputs resident on the device): wall time, cell-steps per
    second and per-sweep device time per launch from the HIP events."""
    import torch

    import fixtures as F
    import paper_1101_3615_amd as M
    nt = w.nt
    c = F.medium(w)
    P = M.Problem.from_spec(w, timing=True)
    P.set_background(torch.from_numpy(c).to("cuda:0"))
    y = F.wavepackets(w, c, 15, 64) if volume else F.trials(w, c)[0]
    y = torch.from_numpy(y).to("cuda:0")
    torch.cuda.synchronize()
    P.stats()
    t0 = time.perf_counter()
    P.apply_H(y)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = P.stats()
    sweeps = {k: {"ms": round(st["ms_sweep"][k], 3), "launches": st["launches_sweep"][k],
                  "us_per_launch": round(1e3 * st["ms_sweep"][k] / st["launches_sweep"][k], 1)}
              for k in st["ms_sweep"] if st["launches_sweep"][k]}
    cs = w.prop_cells * nt * w.ns
    return {"workload": w.name, "steps": nt, "shots": w.ns, "snapshots": w.snap, "apply_H_s": round(wall, 3),
            "gcell_steps_per_s": round(cs / wall / 1e9, 2), "sweeps": sweeps}


CURVELETS = dict(nscales=4, nangles=8, mask_stride=4, nfan=16)   # frame and mask of the curvelet trials
GEN_SIZES = [(0, 0, 0), (0, 1, 1), (0, 2, 2), (1, 0, 2), (1, 2, 2)]   # (Fourier m, angular a, TL degree r): p = 1, 4, 9, 21, 63


def generalization_run(ns=(1, 2, 4)):
    """Rn generalization (relative MSE on an independent trial function) against the
    number of basis terms p, on the 128x128 FP64 workload."""
    import torch

    import fixtures as F
    import paper_1101_3615_amd as M
    from paper_1101_3615_amd.study import generalization, paper_bases
    w = F.c1()
    c = F.medium(w)
    P = M.Problem.from_spec(w)
    P.set_background(torch.from_numpy(c).to("cuda:0"))
    import numpy as np

    from paper_1101_3615_amd.curvelets import Curvelets
    wp = [torch.from_numpy(F.wavepackets(w, c, 100 + s, w.packets_per_trial)).to("cuda:0") for s in range(5)]
    cv = Curvelets(P, **CURVELETS)
    mask = cv.illumination(torch.from_numpy(c).to("cuda:0"))
    cu = [cv.trial(torch.from_numpy(F.normal_field(cv.coef_shape, 600 + s, np.float64)), mask).clone()
          for s in range(5)]
    bases = paper_bases(2, GEN_SIZES)
    out = []
    for kind, trials in (("wavepackets", wp), ("curvelets", cu)):
        for n in ns:
            for p, mse, relres, deficient in generalization(P, bases, trials[:n], trials[4]):
                out.append({"study": "generalization", "workload": w.name, "trials": kind, "preconditioner": f"R{n}",
                            "p": p, "relative_mse": round(mse, 6), "fit_relres": round(relres, 6),
                            "rank_deficient": deficient})
    # Kn, fitted on the Krylov pairs of the migrated image of a reflectivity, tested on the
    # same independent trial functions
    from paper_1101_3615_amd import inversion as I
    m = torch.from_numpy(F.reflectivity(w, c, seed=5).astype(np.float64)).to("cuda:0")
    kys, kxs = I.krylov_pairs(P, P.apply_H(m).clone(), 7)
    for kind, y_new in (("wavepackets", wp[4]), ("curvelets", cu[4])):
        for n in (1, 4, 7):
            for p, mse, relres, deficient in generalization(P, bases, kys[:n], y_new, xs_fit=kxs[:n]):
                out.append({"study": "generalization", "workload": w.name, "trials": kind, "preconditioner": f"K{n}",
                            "p": p, "relative_mse": round(mse, 6), "fit_relres": round(relres, 6),
                            "rank_deficient": deficient})
    return out


def curvelet_run(reps=3):
    """Curvelet trial synthesis and the ray-traced illumination mask on the 512x256 workload
    (FP32): device time per call and the mask's visible fraction."""
    import numpy as np
    import torch

    import fixtures as F
    import paper_1101_3615_amd as M
    from paper_1101_3615_amd.curvelets import Curvelets
    w = F.c2()
    c = torch.from_numpy(F.medium(w)).to("cuda:0")
    P = M.Problem.from_spec(w)
    cv = Curvelets(P, **CURVELETS)
    z = torch.from_numpy(F.normal_field(cv.coef_shape, 700)).to("cuda:0")

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            r = fn()
        torch.cuda.synchronize()
        return r, (time.perf_counter() - t) * 1e3 / reps

    mask, ms_mask = timed(lambda: cv.illumination(c))
    _, ms_trial = timed(lambda: cv.trial(z, mask))
    img = torch.from_numpy(F.normal_field(w.model_shape, 701)).to("cuda:0")
    _, ms_an = timed(lambda: cv.analysis(img))
    nz, nx = w.model_shape
    s = CURVELETS["mask_stride"]
    nodes = -(-nz // s) * -(-nx // s)
    ndir = len({(A, l) for j, l, A in cv.wedges if j > 0})
    rays = 2 * nodes * ndir * CURVELETS["nfan"]
    return {"study": "curvelets", "workload": w.name, "wedges": cv.nw, "mask_nodes": nodes, "directions": ndir,
            "rays": rays, "illumination_ms": round(ms_mask, 2), "rays_per_s": float(f"{rays / ms_mask * 1e3:.4g}"),
            "visible_fraction": round(float(mask.float().mean()), 4), "trial_ms": round(ms_trial, 2),
            "analysis_ms": round(ms_an, 2)}


def gauss_newton_records(P, w, c, refl, basis, trial, outer=3, inner=5):
    """Gauss-Newton from the background c towards m = 1/c^2 + refl, on data modelled at the
    true velocity: misfits and model errors per outer iteration, with CG inner solves
    (plain or preconditioned) and with steps given by a probed inverse alone (K1 fitted on
    the migrated residual, or R1 on a trial function, refitted at every iterate)."""
    import torch

    from paper_1101_3615_amd import inversion as I
    import paper_1101_3615_amd as M
    c0 = torch.from_numpy(c).to("cuda:0").double()
    m0 = 1.0 / (c0 * c0)
    P.set_background(1.0 / torch.sqrt(m0 + refl))
    d_obs = P.model().clone()

    def r1(problem, b):
        coef, _, _ = M.probe_fit(problem, basis, [trial], [problem.apply_H(trial)], strict=False)
        return I.preconditioner(problem, basis, coef)

    def k1(problem, b):
        coef, _, _ = I.fit_krylov(problem, basis, b, 1)
        return I.preconditioner(problem, basis, coef)

    out = []
    for name, pre, cg, ls in (("none", None, inner, False), ("K1", k1, inner, False), ("K1", k1, 0, False),
                              ("R1", r1, 0, False), ("K1", k1, 0, True), ("R1", r1, 0, True)):
        torch.cuda.synchronize()
        t = time.perf_counter()
        rec = {"study": "gauss_newton", "workload": w.name, "preconditioner": name, "p": basis.p, "outer": outer,
               "inner_cg": cg, "line_search": ls}
        try:
            cs, Js = I.gauss_newton(P, c0, d_obs, outer, cg, precond_at=pre, line_search=ls)
        except ValueError as e:   # a step that leaves m = 1/c^2 non-positive
            out.append(dict(rec, error=str(e)))
            continue
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3 / outer
        err = [round(I.relative_mse(P, 1.0 / (ck * ck) - m0, refl), 6) for ck in cs]
        out.append(dict(rec, ms_per_outer=round(ms, 1),
                        misfit=[float(f"{j:.6g}") for j in Js], model_error=err))
    P.set_background(c0)
    return out


def inversion_run(gd_steps=200, cg_iters=20):
    """Linearised inversion of a synthetic reflectivity on the 128x128 FP64 workload: the
    migrated image b = H m, the reference image after gd_steps exact-step descent steps,
    the Rn / Kn fitted inverses applied to b (relative MSE against the reference and
    against m, for each basis size), and CG with and without a fitted preconditioner."""
    import numpy as np
    import torch

    import fixtures as F
    import paper_1101_3615_amd as M
    from paper_1101_3615_amd import inversion as I
    from paper_1101_3615_amd.curvelets import Curvelets
    from paper_1101_3615_amd.study import paper_bases
    w = F.c1()
    c = F.medium(w)
    P = M.Problem.from_spec(w)
    P.set_background(torch.from_numpy(c).to("cuda:0"))
    m = torch.from_numpy(F.reflectivity(w, c, seed=5).astype(np.float64)).to("cuda:0")
    b = P.apply_H(m)
    torch.cuda.synchronize()
    t = time.perf_counter()
    x_gd, phis = I.steepest_descent(P, b, gd_steps)
    torch.cuda.synchronize()
    ms_gd = (time.perf_counter() - t) * 1e3 / gd_steps
    r = b - P.apply_H(x_gd)
    out = [{"study": "inversion", "workload": w.name, "image": f"descent{gd_steps}", "ms_per_step": round(ms_gd, 3),
            "relres": round((P.dot(r, r) / P.dot(b, b)) ** 0.5, 6),
            "mse_vs_true": round(I.relative_mse(P, x_gd, m), 6)}]
    a = float((b * x_gd).sum() / (b * b).sum())
    out.append({"study": "inversion", "workload": w.name, "image": "migrated (best scalar multiple)",
                "mse_vs_descent": round(I.relative_mse(P, a * b, x_gd), 6), "mse_vs_true": round(I.relative_mse(P, a * b, m), 6)})
    trials = [torch.from_numpy(F.wavepackets(w, c, 100 + s, w.packets_per_trial)).to("cuda:0") for s in range(4)]
    Htrials = [P.apply_H(y) for y in trials]
    # randomized curvelet trials on the illuminated set, and the projection onto it that
    # the paper applies before comparing with the true model
    cv = Curvelets(P, **CURVELETS)
    mask = cv.illumination(torch.from_numpy(c).to("cuda:0"))
    ctrials = [cv.trial(torch.from_numpy(F.normal_field(cv.coef_shape, 500 + s, np.float64)), mask) for s in range(4)]
    Hctrials = [P.apply_H(y) for y in ctrials]
    m_vis = cv.project(m, mask).clone()
    kys, kxs = I.krylov_pairs(P, b, 4)
    # the other trial functions of Sec. 2.4: white noise in model space, H applied to it,
    # white data noise migrated; and the fit on the true model itself
    white = [torch.from_numpy(F.normal_field(w.model_shape, 800 + s, np.float64)).to("cuda:0") for s in range(4)]
    Hwhite = [P.apply_H(z).clone() for z in white]
    HHwhite = [P.apply_H(y) for y in Hwhite]
    mig = [P.apply_Fadj(torch.from_numpy(F.normal_field(P.data_shape, 900 + s, np.float64)).to("cuda:0")).clone()
           for s in range(4)]
    Hmig = [P.apply_H(y) for y in mig]
    # H-applied noise whose curvelet coefficients are set to their sign above a small
    # threshold (a tenth of their RMS) and to zero below it, resynthesised with the atom norms
    thr = []
    for y in Hwhite:
        coef = cv.analysis(y)
        rms = (P.dot(coef, coef) / coef.numel()) ** 0.5
        cv.sign_threshold(coef, 0.1 * rms)
        thr.append(cv.synthesis(coef, None, cv.norms()).clone())
    Hthr = [P.apply_H(y) for y in thr]
    fits = {"R1": (trials[:1], Htrials[:1]), "R4": (trials, Htrials),
            "R1c": (ctrials[:1], Hctrials[:1]), "R4c": (ctrials, Hctrials),
            "R4w": (white, Hwhite), "R4Hw": (Hwhite, HHwhite), "R4d": (mig, Hmig), "R4t": (thr, Hthr),
            "Rtrue": ([m], [b]),
            "K1": (kys[:1], kxs[:1]), "K2": (kys[:2], kxs[:2]), "K4": (kys, kxs)}
    bases = paper_bases(2, GEN_SIZES)
    precs = {}
    for name, (ys, xs) in fits.items():
        for B in bases:
            coef, relres, deficient = M.probe_fit(P, B, ys, xs, strict=False)
            torch.cuda.synchronize()
            t = time.perf_counter()
            img = M.apply_Hinv(P, B, coef, b)
            torch.cuda.synchronize()
            apply_ms = (time.perf_counter() - t) * 1e3
            out.append({"study": "inversion", "workload": w.name, "preconditioner": name, "p": B.p,
                        "mse_vs_descent": round(I.relative_mse(P, img, x_gd), 6),
                        "mse_vs_true": round(I.relative_mse(P, img, m), 6),
                        "mse_vs_true_visible": round(I.relative_mse(P, cv.project(img, mask), m_vis), 6),
                        "fit_relres": round(relres, 6),
                        "rank_deficient": deficient, "apply_ms": round(apply_ms, 3)})
            if B.p == 21:
                precs[name] = I.preconditioner(P, B, coef)
    out += gauss_newton_records(P, w, c, m, bases[3], trials[0])
    for name in ("none", "R4", "K1"):
        torch.cuda.synchronize()
        t = time.perf_counter()
        x, norms = I.conjugate_gradient(P, b, cg_iters, precond=precs.get(name))
        torch.cuda.synchronize()
        out.append({"study": "inversion", "workload": w.name, "solver": "CG", "preconditioner": name, "p": 21,
                    "iters": len(norms) - 1, "ms_per_iter": round((time.perf_counter() - t) * 1e3 / cg_iters, 3),
                    "relres": [round(v / norms[0], 6) for v in norms],
                    "mse_vs_descent": round(I.relative_mse(P, x, x_gd), 6), "mse_vs_true": round(I.relative_mse(P, x, m), 6)})
    return out


def wave_size_for(w_full, free_bytes):
    """Shots per wave the engine uses for workload w_full on a device with free_bytes free:
    the largest even count whose one-wave footprint fits 90 % of free memory (the
    library's default budget), then the fewest waves split evenly in pairs."""
    import paper_1101_3615_amd as M
    P = M.Problem.from_spec(w_full)
    budget = 0.9 * free_bytes
    fit = 0
    for k in range(2, w_full.ns + 1, 2):
        if P.footprint("H", nshots=k) <= budget:
            fit = k
    P.close()
    if fit < 2:
        raise RuntimeError("the device cannot hold one pair of shots of the workload")
    ngr, cgr = w_full.ns // 2, fit // 2
    nw = -(-ngr // cgr)
    return -(-ngr // nw) * 2


def per_launch(st, k):
    n = st["launches_sweep"][k]
    return (st["ms_sweep"][k] / 1e3 / n, st["steps_sweep"][k] / n) if n else (None, None)


def sweep_table(st, bytes_of):
    out = {}
    for k in st["ms_sweep"]:
        t, sl = per_launch(st, k)
        if t is None:
            continue
        out[k] = {"ms": round(st["ms_sweep"][k], 3), "launches": st["launches_sweep"][k],
                  "steps_per_launch": round(sl, 3), "us_per_launch": round(1e6 * t, 3),
                  "alg_GBs": round(bytes_of(k, sl) / t / 1e9, 1)}
    return out


def roofline_of(st, w, bytes_of, copy_gbs, nsh):
    """The sweep kind with the most device time: algorithmic bytes per launch over its
    average launch time (HIP events on the call's stream), against the 8 TB/s peak; nsh:
    shots per launch."""
    kind = max(st["ms_sweep"], key=lambda k: st["ms_sweep"][k])
    avg_s, spl = per_launch(st, kind)
    alg = bytes_of(kind, spl)
    achieved = alg / avg_s / 1e9
    r = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
         "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic_for(kind, w, nsh), "kernel": kind,
         "alg_bytes_per_launch": alg, "avg_launch_us": round(avg_s * 1e6, 3), "steps_per_launch": round(spl, 3)}
    if copy_gbs:
        r.update(copy_GBs=round(copy_gbs, 1), frac_of_copy=round(achieved / copy_gbs, 4))
    return r


def copy_rate(dev):
    """A plain device copy of 1 GiB on the same GPU (read + write bytes over time): the
    practical bandwidth ceiling of the moment."""
    import torch
    src_buf = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    dst_buf = torch.empty_like(src_buf)
    dst_buf.copy_(src_buf)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst_buf.copy_(src_buf)
    e1.record()
    torch.cuda.synchronize()
    return 2 * 4 * (1 << 28) * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9


def c2_leg(steps, copy_gbs):
    """The 512 x 256 FP32 workload (full 3000-step record, 64 shots, FP32 g history): the
    whole probing pass (background, H on both trials, the fit, the fitted inverse on the
    remigrated image of a reflectivity) timed over `steps` passes."""
    import torch

    import fixtures as F
    import paper_1101_3615_amd as M
    w = F.c2()
    c = F.medium(w)
    ys = F.trials(w, c)
    refl = F.reflectivity(w, c)
    dev = torch.device("cuda:0")
    c_dev = torch.from_numpy(c).to(dev)
    y_dev = [torch.from_numpy(y).to(dev) for y in ys]
    P = M.Problem.from_spec(w, timing=True)
    P.set_background(c_dev)
    img = P.apply_H(torch.from_numpy(refl).to(dev))
    B = M.Basis(w.legendre, w.qs, w.ndim)
    xs = [torch.empty_like(img) for _ in ys]
    out = torch.empty_like(img)

    def step():
        P.set_background(c_dev)
        for y, x in zip(y_dev, xs):
            P.apply_H(y, out=x)
        coef, _, _ = M.probe_fit(P, B, y_dev, xs, strict=False)
        M.apply_Hinv(P, B, coef, img, out=out)

    step()
    torch.cuda.synchronize()
    P.stats()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    st = P.stats()
    bytes_of = lambda k, sl: kernel_bytes(k, w, round(sl))
    res = {"workload": w.name, "value": round(len(ys) * w.cell_steps / wall / 1e9, 3), "unit": "Gcell-steps/s",
           "ms_per_step": round(1e3 * wall, 2), "steps": steps, "dtype": "f32", "snapshots": "fp32 full g history",
           "value_is": "apply_H cell-steps of both trials per second of the pass; the first application "
                       "computes and keeps the g history, the second reuses it (no background sweep)",
           "roofline": roofline_of(st, w, bytes_of, copy_gbs, w.ns), "sweeps": sweep_table(st, bytes_of)}
    P.close()
    return res


def c3_leg(nt, copy_gbs):
    """The 1024 x 512 workload with BF16 checkpoints every 4 steps: one application of H over
    nt of its 4000 steps, 128 shots in waves of 64 (the wave size of the full record)."""
    import torch

    import fixtures as F
    import paper_1101_3615_amd as M
    w = F.c3().with_(nt=nt)
    c = F.medium(w)
    y = torch.from_numpy(F.trials(w, c)[0]).to("cuda:0")
    os.environ["MP_MAX_WAVE"] = "64"
    try:
        P = M.Problem.from_spec(w, timing=True)
        P.set_background(torch.from_numpy(c).to("cuda:0"))
        P.apply_H(y)
        torch.cuda.synchronize()
        P.stats()
        t0 = time.perf_counter()
        P.apply_H(y)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = P.stats()
        waves = st["waves"]
    finally:
        os.environ.pop("MP_MAX_WAVE", None)
    nsh = w.ns // waves
    # a 2D launch covers the wave's shots; its bytes scale with them
    bytes_of = lambda k, sl: kernel_bytes(k, w.with_(src=w.src[:nsh]), round(sl))
    res = {"workload": w.name, "value": round(w.cell_steps / wall / 1e9, 3), "unit": "Gcell-steps/s",
           "record_steps": F.c3().nt, "steps": nt, "waves": waves, "dtype": "f32",
           "snapshots": "bf16 checkpoints every 4 steps",
           "roofline": roofline_of(st, w, bytes_of, copy_gbs, nsh), "sweeps": sweep_table(st, bytes_of)}
    P.close()
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--record-steps", type=int, default=40,
                    help="time steps of the 2000-step record applied per H in a benchmark step")
    ap.add_argument("--cpu-steps", type=int, default=2, help="time steps of the CPU-baseline sample")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="run only the headline workload with this many record steps, no extra legs (counter "
                         "collection; the printed line is then marked and is not a benchmark result)")
    ap.add_argument("--full-record", action="store_true",
                    help="only apply H once over the full 2000-step record of the 256^3 workload (with the "
                         "benchmark's wave size) and print its rate: the check of the extrapolated value")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="only run a device-to-device copy of this many MiB (counter calibration)")
    ap.add_argument("--volume-steps", type=int, default=0,
                    help="only run apply_H on the 256^3 workload (32 shots, BF16 checkpoints) with this "
                         "many time steps and print its sweep times (3D measurement and profiling)")
    ap.add_argument("--leg", choices=("c2", "c3"), default=None,
                    help="run one extra leg alone (the 512x256 pass or the 1024x512 application) and print its "
                         "JSON: the command the counter and trace summaries of those workloads are taken on")
    ap.add_argument("--checkpointed-steps", type=int, default=0,
                    help="only run apply_H on the 1024x512 workload (128 shots, BF16 checkpoints every 4 steps) "
                         "with this many time steps and print its sweep times")
    ap.add_argument("--generalization", action="store_true",
                    help="only run the generalization study of the probed inverse (128x128 FP64 workload, "
                         "R1/R2/R4 fitted on 1/2/4 trial functions, tested on an independent one, bases of the "
                         "paper's expansion with growing p) and print one JSON line per fit")
    ap.add_argument("--inversion", action="store_true",
                    help="only run the linearised inversion study (128x128 FP64 workload: 200 descent steps as "
                         "the reference image, Rn/Kn fitted inverses applied to the migrated image, CG with and "
                         "without a fitted preconditioner) and print one JSON line per result")
    ap.add_argument("--curvelets", action="store_true",
                    help="only time the curvelet trial synthesis and the ray-traced illumination mask on the "
                         "512x256 workload and print one JSON line")
    ap.add_argument("--cpu-workers", type=int, default=min(8, os.cpu_count() or 1))
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the 512x256 and 1024x512 legs")
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="length of the Poisson serving run (0: skip the serving leg)")
    ap.add_argument("--ingest-counters", nargs=5,
                    metavar=("DIMS", "FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="DIMS = 2d, c3 or 3d: write profiles/traffic.json, traffic_c3.json or traffic_c5.json "
                         "from rocprofv3 --pmc output folders and exit")
    args = ap.parse_args()
    if args.ingest_counters:
        dims, *dirs = args.ingest_counters
        print(json.dumps(ingest_counters(*dirs, 1024, dims), indent=1))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (shots would shard "
              "across GPUs with one all-reduce of the image; that path is not built)", file=sys.stderr)
        sys.exit(2)

    if args.copy_probe_mb:
        import torch
        n = args.copy_probe_mb * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n}))
        return
    if args.leg:
        import torch
        copy_gbs = copy_rate(torch.device("cuda:0"))
        print(json.dumps(c2_leg(1, copy_gbs) if args.leg == "c2" else c3_leg(400, copy_gbs)))
        return
    if args.checkpointed_steps:
        print(json.dumps(checkpointed_run(args.checkpointed_steps)))
        return
    if args.volume_steps:
        print(json.dumps(volume_run(args.volume_steps)))
        return
    if args.generalization:
        for rec in generalization_run():
            print(json.dumps(rec), flush=True)
        return
    if args.curvelets:
        print(json.dumps(curvelet_run()), flush=True)
        return
    if args.inversion:
        for rec in inversion_run():
            print(json.dumps(rec), flush=True)
        return

    import fixtures as F

    w_full = F.c5()
    nt_b = args.profile_steps or args.record_steps
    if args.full_record:
        nt_b = w_full.nt
    w = w_full.with_(nt=nt_b)
    t_in = time.perf_counter()
    c = F.medium(w)
    ys = F.trials(w, c)                          # the workload's 4 trials of 4096 packets
    print(f"inputs ready in {time.perf_counter() - t_in:.1f} s", file=sys.stderr, flush=True)
    # CPU baseline before anything touches the GPU: forked workers must not inherit a
    # HIP runtime
    run_cpu = not (args.no_cpu or args.profile_steps or args.full_record)
    cpu = cpu_baseline(w_full, c, ys[0], args.cpu_steps, args.cpu_workers) if run_cpu else None
    if cpu:
        print(f"cpu baseline {cpu['value']:.4f} Gcell-steps/s", file=sys.stderr, flush=True)

    import torch

    import paper_1101_3615_amd as M
    dev = torch.device("cuda:0")
    free = torch.cuda.mem_get_info(dev)[0]
    wave = wave_size_for(w_full, free)
    os.environ["MP_MAX_WAVE"] = str(wave)
    c_dev = torch.from_numpy(c).to(dev)
    y_dev = [torch.from_numpy(y).to(dev) for y in ys]
    if args.full_record:
        # one apply_H over the full 2000-step record, shot waves as the engine plans them
        P = M.Problem.from_spec(w, timing=True)
        P.set_background(c_dev)
        torch.cuda.synchronize()
        P.stats()
        print(f"apply_H over {w.nt} steps, waves of {wave} shots", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        P.apply_H(y_dev[0])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = P.stats()
        bytes_of = lambda k, sl: kernel_bytes3d(k, w, wave)
        print(json.dumps({"workload": w.name, "record_steps": w.nt, "shots": w.ns, "wave_shots": wave,
                          "waves": st["waves"], "apply_H_s": round(wall, 3),
                          "gcell_steps_per_s": round(w.cell_steps / wall / 1e9, 3),
                          "sweeps": sweep_table(st, bytes_of)}), flush=True)
        return
    P = M.Problem.from_spec(w, timing=True)
    P.set_background(c_dev)
    B = M.Basis(w.legendre, w.qs, w.ndim)
    xs = [torch.empty_like(y) for y in y_dev]
    out = torch.empty_like(y_dev[0])

    def step():
        P.set_background(c_dev)
        for y, x in zip(y_dev, xs):
            P.apply_H(y, out=x)
        coef, relres, deficient = M.probe_fit(P, B, y_dev, xs, strict=False)
        M.apply_Hinv(P, B, coef, xs[0], out=out)
        return relres, deficient

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    P.stats()                                   # restart the sweep timers
    t0 = time.perf_counter()
    for _ in range(args.steps):
        relres, deficient = step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = P.stats()
    waves = st["waves"]
    # the fitted inverse applied to x_0 against y_0 (the fit's own training pair)
    rec_err = ((P.dot(out - y_dev[0], out - y_dev[0]) / P.dot(y_dev[0], y_dev[0])) ** 0.5
               if out.dtype == y_dev[0].dtype else None)
    P.close()
    del P, xs, out, y_dev
    torch.cuda.empty_cache()
    os.environ.pop("MP_MAX_WAVE", None)
    print(f"headline: {wall / args.steps:.3f} s per step", file=sys.stderr, flush=True)
    copy_gbs = copy_rate(dev)
    extra = {}
    if not (args.no_extra or args.profile_steps):
        extra["c2"] = c2_leg(3, copy_gbs)
        print("c2 leg done", file=sys.stderr, flush=True)
        extra["c3"] = c3_leg(400, copy_gbs)
        print("c3 leg done", file=sys.stderr, flush=True)
    serving = serve_leg(args.serve_seconds) if (args.serve_seconds > 0 and not args.profile_steps) else None

    ms_per_step = 1e3 * wall / args.steps
    cell_steps = len(ys) * w.cell_steps
    value = cell_steps / (wall / args.steps) / 1e9
    bytes_of = lambda k, sl: kernel_bytes3d(k, w, wave)
    line = {
        "metric": "Gcell-steps/s for H=F*F (fraction of HBM roofline); served p50/p99 latency",
        "value": round(value, 3),
        "unit": "Gcell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "model_grid": [w.nx, w.ny, w.nz], "prop_grid": list(reversed(w.prop_shape)),
                   "shots": w.ns, "receivers": w.nr, "record_steps": w_full.nt, "steps_per_apply_H": w.nt,
                   "wave_shots": wave, "waves": waves, "trials": len(ys), "packets_per_trial": w.packets_per_trial,
                   "p": w.p, "snapshots": "bf16 checkpoints every 8 steps, fp32 scales, recomputation",
                   "image": "fp64", "apply_H_cell_steps_per_step": cell_steps,
                   "value_is": f"apply_H rate over {w.nt} of the {w_full.nt} record steps per application, "
                               "extrapolated to the full record (same launches per step)"},
        "roofline": roofline_of(st, w, bytes_of, copy_gbs, wave),
        "cpu_baseline": cpu,
        "serving": serving,
        "sweeps": sweep_table(st, bytes_of),
        "profile_run": bool(args.profile_steps),
        "fit_relres": relres,
        "fit_rank_deficient": deficient,
        "hinv_x0_vs_y0": rec_err,
    }
    line.update(extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
