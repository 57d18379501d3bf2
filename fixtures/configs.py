"""The five synthetic workloads, as plain parameter records.

Each record fixes the grid, the acquisition, the time sampling, the
precision and snapshot mode, the probing basis and the seeds of every random
input.  Nothing here computes anything of the method.

Positions are model-grid indices: (ix, iz) in 2D, (ix, iy, iz) in 3D, with
row iz = 0 the surface.  A model grid of NX x NZ (x NY) cells is surrounded on
every side by an absorbing layer of ``nb`` cells.
"""
from dataclasses import dataclass, field, replace
from typing import List, Optional, Tuple

import numpy as np


@dataclass
class Workload:
    name: str
    ndim: int
    nx: int
    nz: int
    ny: int = 1
    h: float = 10.0
    nb: int = 20
    dt: float = 1.0e-3
    nt: int = 800
    f_peak: float = 15.0
    t0: Optional[float] = None          # wavelet delay; 1/f_peak when None
    src: np.ndarray = None              # int32 [ns][ndim]
    rec: np.ndarray = None              # int32 [nr][ndim]
    dtype: str = "f64"                  # field precision: "f32" | "f64"
    snap: str = "full"                  # "full" | "ckpt_f32" | "ckpt_bf16"
    ckpt_every: int = 0
    medium: dict = field(default_factory=dict)
    sponge_R: float = 1.0e-3
    # probing: one Legendre degree per model axis, numpy axis order (z, [y,] x)
    legendre: List[Tuple[int, ...]] = field(default_factory=list)
    qs: Tuple[int, ...] = (0, 1, 2, 3)
    trial_seeds: Tuple[int, ...] = ()
    packets_per_trial: int = 64
    refl_seed: Optional[int] = None

    @property
    def ns(self):
        return int(self.src.shape[0])

    @property
    def nr(self):
        return int(self.rec.shape[0])

    @property
    def wavelet_t0(self):
        return 1.0 / self.f_peak if self.t0 is None else self.t0

    @property
    def model_shape(self):
        """numpy shape of a model-grid array, slowest axis first."""
        if self.ndim == 2:
            return (self.nz, self.nx)
        return (self.nz, self.ny, self.nx)

    @property
    def prop_shape(self):
        return tuple(n + 2 * self.nb for n in self.model_shape)

    @property
    def prop_cells(self):
        return int(np.prod(self.prop_shape))

    @property
    def model_cells(self):
        return int(np.prod(self.model_shape))

    @property
    def cell_steps(self):
        """Propagation-grid cell-steps of one sweep over all shots."""
        return self.prop_cells * self.nt * self.ns

    @property
    def p(self):
        return len(self.legendre) * len(self.qs)

    def with_(self, **kw):
        return replace(self, **kw)


def _row0(xs, ndim, ys=None):
    xs = np.asarray(xs, dtype=np.int32)
    if ndim == 2:
        return np.stack([xs, np.zeros_like(xs)], axis=1).astype(np.int32)
    ys = np.asarray(ys, dtype=np.int32)
    return np.stack([xs, ys, np.zeros_like(xs)], axis=1).astype(np.int32)


def _even_sources(nx, ns):
    return [int((s + 0.5) * nx / ns) for s in range(ns)]


def c1():
    """Plain method, FP64, 128 x 128 at 10 m, 4 sources, 128 receivers."""
    return Workload(
        name="c1_2d_128x128_f64", ndim=2, nx=128, nz=128, h=10.0, nb=20,
        dt=1.0e-3, nt=800, f_peak=15.0,
        src=_row0(_even_sources(128, 4), 2),
        rec=_row0(np.arange(128), 2),
        dtype="f64", snap="full",
        medium=dict(kind="gradient_bump", c0=1500.0, grad=0.5, bump=200.0,
                    sigma=150.0),
        legendre=[(0, 0), (1, 0), (2, 0)], trial_seeds=(1,), packets_per_trial=64)


def c2():
    """Plain method, FP32, 512 x 256 at 10 m, 64 sources, 256 receivers."""
    return Workload(
        name="c2_2d_512x256_f32", ndim=2, nx=512, nz=256, h=10.0, nb=20,
        dt=0.8e-3, nt=3000, f_peak=12.0,
        src=_row0(4 + 8 * np.arange(64), 2),
        rec=_row0(2 * np.arange(256), 2),
        dtype="f32", snap="full",
        medium=dict(kind="smooth_random", cmin=1500.0, cmax=4000.0,
                    corr=300.0, seed=2),
        legendre=[(a, 0) for a in range(5)], trial_seeds=(3, 4),
        packets_per_trial=512, refl_seed=5)


def c3():
    """Differentiation: 1024 x 512, 128 sources, 512 receivers, BF16 ckpt/4."""
    return Workload(
        name="c3_2d_1024x512_f32_bf16ckpt", ndim=2, nx=1024, nz=512, h=10.0,
        nb=20, dt=0.8e-3, nt=4000, f_peak=12.0,
        src=_row0(4 + 8 * np.arange(128), 2),
        rec=_row0(2 * np.arange(512), 2),
        dtype="f32", snap="ckpt_bf16", ckpt_every=4,
        medium=dict(kind="smooth_random", cmin=1500.0, cmax=4000.0,
                    corr=300.0, seed=6),
        legendre=[(a, 0) for a in range(5)], trial_seeds=(7,),
        packets_per_trial=512, refl_seed=9)


SERVE_SHAPES = ((256, 128), (512, 256), (1024, 512))
SERVE_SHOTS = (16, 32, 64)


def serve_steps(nx, nz):
    """Step count scaled with the grid diagonal: 104 at 256 x 128, the Ricker delay
    1/f_peak = 83 ms at dt = 0.8 ms, so the wavelet's peak enters every grid (416
    steps, 333 ms, at 1024 x 512).  Longer records would offer more work at 20
    requests/s than one GPU serves."""
    return int(round(104.0 * np.hypot(nx, nz) / np.hypot(256, 128)))


def c4(nx=256, nz=128, ns=16, seed=10):
    """Serving request shape: C2 physics, BF16 ckpt every 4."""
    return Workload(
        name=f"c4_2d_{nx}x{nz}_s{ns}", ndim=2, nx=nx, nz=nz, h=10.0, nb=20,
        dt=0.8e-3, nt=serve_steps(nx, nz), f_peak=12.0,
        src=_row0(_even_sources(nx, ns), 2),
        rec=_row0(2 * np.arange(nx // 2), 2),
        dtype="f32", snap="ckpt_bf16", ckpt_every=4,
        medium=dict(kind="smooth_random", cmin=1500.0, cmax=4000.0,
                    corr=300.0, seed=seed),
        legendre=[(0, 0)], trial_seeds=())


def c4_union(nx=256, nz=128, seed=10):
    """A serving shape with the source sets of every shot count in one acquisition.

    Returns (workload, groups): groups[ns] lists the acquisition indices of the
    ns sources placed at (s + 1/2) NX / ns.
    """
    xs, groups = [], {}
    for ns in SERVE_SHOTS:
        groups[ns] = list(range(len(xs), len(xs) + ns))
        xs += _even_sources(nx, ns)
    w = c4(nx, nz, SERVE_SHOTS[0], seed).with_(src=_row0(xs, 2), name=f"c4_2d_{nx}x{nz}_union")
    return w, groups


def c5():
    """3D: 256^3 at 12.5 m, 32 sources, 64 x 64 receivers, BF16 ckpt/8."""
    sx, sy = np.meshgrid(16 + 32 * np.arange(8), 32 + 64 * np.arange(4))
    rx, ry = np.meshgrid(4 * np.arange(64) + 2, 4 * np.arange(64) + 2)
    leg = [(i, j, k) for i in range(3) for j in range(3) for k in range(3)
           if i + j + k <= 2]
    return Workload(
        name="c5_3d_256cube_f32_bf16ckpt", ndim=3, nx=256, ny=256, nz=256,
        h=12.5, nb=20, dt=1.0e-3, nt=2000, f_peak=10.0,
        src=_row0(sx.ravel(), 3, sy.ravel()),
        rec=_row0(rx.ravel(), 3, ry.ravel()),
        dtype="f32", snap="ckpt_bf16", ckpt_every=8,
        medium=dict(kind="smooth_random", cmin=1500.0, cmax=4500.0,
                    corr=400.0, seed=14),
        legendre=leg, trial_seeds=(15, 16, 17, 18), packets_per_trial=4096)


ALL = {"c1": c1, "c2": c2, "c3": c3, "c4": c4, "c5": c5}
