"""Python binding of the operators: argument marshalling only.

Every step of F, F*, H, the probing fit and the fitted inverse runs in the HIP
kernels of libmatprobe.so; torch provides device memory and the stream.
Arrays use numpy axis order (z, [y,] x); positions are (x, [y,] z) model-grid
indices like the C ABI.
"""
import ctypes

import numpy as np
import torch

from . import _lib as L

_DT = {"f32": (L.MP_F32, torch.float32), "f64": (L.MP_F64, torch.float64)}
_SNAP = {"full": L.MP_SNAP_FULL, "ckpt_f32": L.MP_SNAP_CKPT_F32, "ckpt_bf16": L.MP_SNAP_CKPT_BF16}


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Problem:
    """One grid, acquisition and background; owns an mp_ctx."""

    def __init__(self, *, ndim, nx, nz, ny=1, h, nb, src, rec, f_peak, t0, dt, nt,
                 dtype="f32", snap="full", ckpt_every=0, budget_bytes=0, sponge_R=1e-3,
                 timing=False, device="cuda:0"):
        lib = L.lib()
        self.ndim = int(ndim)
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.nt = int(nt)
        self.device = torch.device(device)
        self.dtype_code, self.torch_dtype = _DT[dtype]
        self.src = np.ascontiguousarray(src, dtype=np.int32)
        self.rec = np.ascontiguousarray(rec, dtype=np.int32)
        self.ns = int(self.src.shape[0])
        self.nr = int(self.rec.shape[0])
        g = L.Grid(self.ndim, (ctypes.c_int * 3)(self.nx, self.ny, self.nz), float(h), int(nb))
        a = L.Acq(self.ns, self.src.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), self.nr,
                  self.rec.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), float(f_peak), float(t0),
                  float(dt), self.nt)
        o = L.Opts(self.dtype_code, _SNAP[snap], int(ckpt_every), int(budget_bytes), float(sponge_R),
                   1 if timing else 0)
        ctx = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            L.check(lib.mp_create(ctypes.byref(g), ctypes.byref(a), ctypes.byref(o), ctypes.byref(ctx)))
        self._ctx = ctx
        self._lib = lib

    @classmethod
    def from_spec(cls, w, **kw):
        """Build from any object carrying the workload attributes (ndim, nx, ...)."""
        args = dict(ndim=w.ndim, nx=w.nx, nz=w.nz, ny=w.ny, h=w.h, nb=w.nb, src=w.src, rec=w.rec,
                    f_peak=w.f_peak, t0=w.wavelet_t0, dt=w.dt, nt=w.nt, dtype=w.dtype,
                    snap=w.snap, ckpt_every=w.ckpt_every, sponge_R=w.sponge_R)
        args.update(kw)
        return cls(**args)

    @property
    def model_shape(self):
        return (self.nz, self.nx) if self.ndim == 2 else (self.nz, self.ny, self.nx)

    @property
    def data_shape(self):
        return (self.ns, self.nt, self.nr)

    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            self._lib.mp_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _model(self, t, name):
        if not isinstance(t, torch.Tensor):
            t = torch.as_tensor(np.asarray(t))
        t = t.to(device=self.device, dtype=self.torch_dtype).contiguous()
        if tuple(t.shape) != self.model_shape:
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {self.model_shape}")
        return t

    def set_background(self, c, stream=None):
        c = self._model(c, "c")
        self._c = c
        L.check(self._lib.mp_set_background(self._ctx, _ptr(c), _stream(stream)))

    def apply_F(self, dm, out=None, stream=None):
        dm = self._model(dm, "dm")
        d = out if out is not None else torch.empty(self.data_shape, dtype=self.torch_dtype,
                                                    device=self.device)
        L.check(self._lib.mp_apply_F(self._ctx, _ptr(dm), _ptr(d), _stream(stream)))
        return d

    def model(self, out=None, stream=None):
        """Nonlinear modelling at the current background: d[s][n][r] = u_s^{n+1}(x_r)."""
        d = out if out is not None else torch.empty(self.data_shape, dtype=self.torch_dtype, device=self.device)
        if tuple(d.shape) != self.data_shape or d.dtype != self.torch_dtype or not d.is_contiguous():
            raise ValueError(f"out must be a contiguous {self.torch_dtype} tensor of shape {self.data_shape}")
        L.check(self._lib.mp_model(self._ctx, _ptr(d), _stream(stream)))
        return d

    def apply_Fadj(self, d, out=None, stream=None):
        if not isinstance(d, torch.Tensor):
            d = torch.as_tensor(np.asarray(d))
        d = d.to(device=self.device, dtype=self.torch_dtype).contiguous()
        if tuple(d.shape) != self.data_shape:
            raise ValueError(f"d has shape {tuple(d.shape)}, expected {self.data_shape}")
        img = out if out is not None else torch.empty(self.model_shape, dtype=self.torch_dtype,
                                                      device=self.device)
        L.check(self._lib.mp_apply_Fadj(self._ctx, _ptr(d), _ptr(img), _stream(stream)))
        return img

    def apply_H(self, dm, out=None, stream=None):
        dm = self._model(dm, "dm")
        o = out if out is not None else torch.empty(self.model_shape, dtype=self.torch_dtype,
                                                    device=self.device)
        L.check(self._lib.mp_apply_H(self._ctx, _ptr(dm), _ptr(o), _stream(stream)))
        return o

    def footprint(self, op="H", nshots=0):
        """Device bytes the operator needs for nshots shots (0: all acquisition shots)."""
        code = {"F": L.MP_OP_F, "Fadj": L.MP_OP_FADJ, "H": L.MP_OP_H, "fit": L.MP_OP_FIT,
                "Hinv": L.MP_OP_HINV}[op]
        b = ctypes.c_size_t()
        L.check(self._lib.mp_footprint(self._ctx, code, int(nshots), ctypes.byref(b)))
        return b.value

    def apply_H_batch(self, dms, shot_lists, outs=None, stream=None):
        """out[r] = sum over shot_lists[r] of F_s* F_s dms[r], all requests in one sweep."""
        dms = [self._model(d, "dm") for d in dms]
        if outs is None:
            outs = [torch.empty(self.model_shape, dtype=self.torch_dtype, device=self.device) for _ in dms]
        n = len(dms)
        counts = np.ascontiguousarray([len(s) for s in shot_lists], dtype=np.int32)
        shots = np.ascontiguousarray(np.concatenate([np.asarray(s, dtype=np.int32) for s in shot_lists]))
        dp = (ctypes.c_void_p * n)(*[d.data_ptr() for d in dms])
        op = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
        L.check(self._lib.mp_apply_H_batch(self._ctx, n, counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                           shots.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), dp, op,
                                           _stream(stream)))
        self._keep = dms                     # inputs must outlive the enqueued work
        return outs

    _BATCH_OPS = {"F": L.MP_OP_F, "Fadj": L.MP_OP_FADJ, "H": L.MP_OP_H}

    def footprint_batch(self, op, nshots, nreq):
        """Device bytes of apply_batch for nreq requests over nshots shots."""
        b = ctypes.c_size_t()
        L.check(self._lib.mp_footprint_batch(self._ctx, self._BATCH_OPS[op], int(nshots), int(nreq),
                                             ctypes.byref(b)))
        return b.value

    def apply_batch(self, op, xs, shots, outs=None, stream=None):
        """op in {"F", "Fadj", "H"} applied to every request xs[r] over the common shot
        list `shots`, the background of each shot propagated once for all requests.
        F: model -> data [len(shots)][nt][nr]; Fadj: such data -> image; H: model -> image."""
        shots = np.ascontiguousarray(np.asarray(shots, dtype=np.int32).ravel())
        ns = int(shots.size)
        dshape = (ns, self.data_shape[1], self.data_shape[2])
        if op == "Fadj":
            ins = []
            for x in xs:
                t = x if isinstance(x, torch.Tensor) else torch.as_tensor(np.asarray(x))
                t = t.to(device=self.device, dtype=self.torch_dtype).contiguous()
                if tuple(t.shape) != dshape:
                    raise ValueError(f"data has shape {tuple(t.shape)}, expected {dshape}")
                ins.append(t)
        else:
            ins = [self._model(x, "dm") for x in xs]
        oshape = dshape if op == "F" else self.model_shape
        if outs is None:
            outs = [torch.empty(oshape, dtype=self.torch_dtype, device=self.device) for _ in ins]
        for o in outs:
            if tuple(o.shape) != oshape or o.dtype != self.torch_dtype or not o.is_contiguous():
                raise ValueError(f"outputs must be contiguous {self.torch_dtype} tensors of shape {oshape}")
        n = len(ins)
        ip = (ctypes.c_void_p * n)(*[t.data_ptr() for t in ins])
        op_ = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
        L.check(self._lib.mp_apply_batch(self._ctx, self._BATCH_OPS[op], n, ns,
                                         shots.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), ip, op_,
                                         _stream(stream)))
        self._keep = ins                     # inputs must outlive the enqueued work
        return outs

    # ---- vector kernels of the solvers (FP64 accumulation, fixed order) ----
    def _vec(self, t, name):
        if not (isinstance(t, torch.Tensor) and t.device == self.device and t.dtype == self.torch_dtype
                and t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous {self.torch_dtype} tensor on {self.device}")
        return t

    def dot(self, a, b, stream=None):
        """sum_i a_i b_i (FP64, fixed summation order); a and b of equal size."""
        a, b = self._vec(a, "a"), self._vec(b, "b")
        if a.numel() != b.numel():
            raise ValueError("dot of vectors of different sizes")
        out = ctypes.c_double()
        L.check(self._lib.mp_vec_dot(self._ctx, a.numel(), _ptr(a), _ptr(b), ctypes.byref(out), _stream(stream)))
        return out.value

    def dot_noalloc(self, a, b, out, stream=None):
        """out[0] = sum_i a_i b_i on the device, as dot() (same bits), allocating nothing and
        not synchronising; out is a float64 device tensor of at least one element."""
        a, b = self._vec(a, "a"), self._vec(b, "b")
        if a.numel() != b.numel():
            raise ValueError("dot of vectors of different sizes")
        if not (isinstance(out, torch.Tensor) and out.device == self.device and out.dtype == torch.float64
                and out.numel() >= 1 and out.is_contiguous()):
            raise ValueError(f"out must be a contiguous float64 tensor on {self.device}")
        L.check(self._lib.mp_vec_dot_noalloc(self._ctx, a.numel(), _ptr(a), _ptr(b), _ptr(out), _stream(stream)))
        return out

    def axpby(self, alpha, x, beta, y, stream=None):
        """y = alpha x + beta y in place (FP64 arithmetic, rounded to the field precision);
        beta = 0 overwrites y without reading it."""
        x, y = self._vec(x, "x"), self._vec(y, "y")
        if x.numel() != y.numel():
            raise ValueError("axpby of vectors of different sizes")
        L.check(self._lib.mp_vec_axpby(self._ctx, x.numel(), float(alpha), _ptr(x), float(beta), _ptr(y),
                                       _stream(stream)))
        return y

    def velocity_update(self, c, dm, stream=None):
        """c <- (c^-2 + dm)^(-1/2) in place on the model grid (a Gauss-Newton step in m = 1/c^2)."""
        c, dm = self._vec(c, "c"), self._vec(dm, "dm")
        if tuple(c.shape) != self.model_shape or tuple(dm.shape) != self.model_shape:
            raise ValueError(f"c and dm must have the model shape {self.model_shape}")
        L.check(self._lib.mp_velocity_update(self._ctx, _ptr(c), _ptr(dm), _stream(stream)))
        return c

    def release_cache(self):
        L.check(self._lib.mp_release_cache(self._ctx))

    def stats(self):
        s = L.Stats()
        L.check(self._lib.mp_last_stats(self._ctx, ctypes.byref(s)))
        return dict(cell_steps=s.cell_steps, waves=s.waves,
                    background_cached=bool(s.background_cached), bytes_reserved=s.bytes_reserved,
                    ms_sweep={k: s.ms_sweep[i] for i, k in enumerate(L.SWEEP_KINDS)},
                    launches_sweep={k: s.launches_sweep[i] for i, k in enumerate(L.SWEEP_KINDS)},
                    steps_sweep={k: s.steps_sweep[i] for i, k in enumerate(L.SWEEP_KINDS)})


class Basis:
    """Probing basis (see mp_basis_desc).  Basis(legendre, qs, ndim): Legendre position
    factors (degrees in numpy axis order) x powers of rho.  Basis.fourier_angular(...):
    the expansion of Sec. 1.2 — Fourier modes in x x angular harmonics of k x rational
    Chebyshev functions of |k| x |k|^order."""

    _P = ctypes.POINTER(ctypes.c_int)

    def __init__(self, legendre, qs, ndim):
        self.family = 0
        self.legendre = [tuple(int(v) for v in a) for a in legendre]
        self.qs = [int(q) for q in qs]
        self.ndim = int(ndim)
        # C ABI takes degrees in axis order (x, [y,] z)
        degs = np.ascontiguousarray([list(reversed(a)) for a in self.legendre], dtype=np.int32)
        qs_arr = np.ascontiguousarray(self.qs, dtype=np.int32)
        self._create(L.BasisDesc(self.ndim, len(self.legendre), degs.ctypes.data_as(self._P), len(self.qs),
                                 qs_arr.ctypes.data_as(self._P), 0, None, None, 0, 1.0))
        self._na, self._nq = len(self.legendre), len(self.qs)

    @classmethod
    def fourier_angular(cls, modes, mults, ndim, order=1, tl_scale=0.5):
        """modes: (m per numpy axis..., phase 0 cos / 1 sin); mults: (angular index,
        rational Chebyshev degree); order: power of rho; tl_scale: L of TL_n."""
        self = cls.__new__(cls)
        self.family = 1
        self.ndim = int(ndim)
        self.modes = [tuple(int(v) for v in m) for m in modes]
        self.mults = [tuple(int(v) for v in q) for q in mults]
        self.order, self.tl_scale = int(order), float(tl_scale)
        rows = []
        for m in self.modes:   # numpy axis order (z, [y,] x) -> ABI (x, y, z)
            ms, phase = list(m[:-1]), m[-1]
            x, z = ms[-1], ms[0]
            y = ms[1] if self.ndim == 3 else 0
            rows.append([x, y, z, phase])
        marr = np.ascontiguousarray(rows, dtype=np.int32)
        qarr = np.ascontiguousarray(self.mults, dtype=np.int32)
        self._create(L.BasisDesc(self.ndim, len(self.modes), None, len(self.mults), None, 1,
                                 marr.ctypes.data_as(self._P), qarr.ctypes.data_as(self._P), self.order,
                                 self.tl_scale))
        self._na, self._nq = len(self.modes), len(self.mults)
        return self

    def _create(self, d):
        lib = L.lib()
        h = ctypes.c_void_p()
        L.check(lib.mp_basis_create(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        self._lib = lib

    @property
    def p(self):
        return self._na * self._nq

    def __del__(self):
        try:
            if self._h.value:
                self._lib.mp_basis_destroy(self._h)
        except Exception:
            pass


def probe_fit(problem, basis, ys, xs, stream=None, strict=True):
    """Least-squares symbol coefficients c (numpy float64) and the relative residual.

    With strict=False a numerically rank-deficient system returns
    (c, relres, True) with the minimum-norm coefficients instead of raising.
    """
    ys = [problem._model(y, "y") for y in ys]
    xs = [problem._model(x, "x") for x in xs]
    T = len(ys)
    yp = (ctypes.c_void_p * T)(*[y.data_ptr() for y in ys])
    xp = (ctypes.c_void_p * T)(*[x.data_ptr() for x in xs])
    c = np.zeros(basis.p, dtype=np.float64)
    rel = ctypes.c_double()
    rc = problem._lib.mp_probe_fit(problem._ctx, basis._h, T, yp, xp,
                                   c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(rel),
                                   _stream(stream))
    if not strict:
        if rc not in (L.MP_OK, L.MP_ENUMERIC):
            L.check(rc)
        return c, rel.value, rc == L.MP_ENUMERIC
    L.check(rc)
    return c, rel.value


def apply_Hinv(problem, basis, c, img, out=None, stream=None):
    img = problem._model(img, "img")
    c = np.ascontiguousarray(c, dtype=np.float64)
    if c.shape != (basis.p,):
        raise ValueError(f"c has shape {c.shape}, expected ({basis.p},)")
    o = out if out is not None else torch.empty_like(img)
    L.check(problem._lib.mp_apply_Hinv(problem._ctx, basis._h,
                                       c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                       _ptr(img), _ptr(o), _stream(stream)))
    return o
