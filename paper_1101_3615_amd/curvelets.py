"""Curvelet-space trial functions with an illumination mask (Sec. 1.5 and Sec. 2 of the
paper) on a 2D problem's model grid.  Argument marshalling over the C ABI
(mp_curvelet_*, mp_illumination); the frame, the ray tracing and the synthesis run in the
library's kernels.

    cv = Curvelets(problem, nscales=4, nangles=8)
    mask = cv.illumination(c)                      # [nwedges, nz, nx] uint8, rays in c
    y = cv.trial(z, mask, sigma=1.0)               # z: [nwedges, nz, nx] N(0, 1) draws
"""
import ctypes

import numpy as np
import torch

from . import _lib as L
from .problem import _ptr, _stream


class Curvelets:
    def __init__(self, problem, nscales=4, nangles=8, mask_stride=4, nfan=16, max_steps=4000, ray_rtol=1e-4):
        self.problem = problem          # the context must outlive the handle's use
        self._lib = L.lib()
        d = L.CurveletDesc(int(nscales), int(nangles), int(mask_stride), int(nfan), int(max_steps),
                           float(ray_rtol))
        h = ctypes.c_void_p()
        L.check(self._lib.mp_curvelet_create(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        n = ctypes.c_int()
        L.check(self._lib.mp_curvelet_wedges(self._h, ctypes.byref(n), None))
        lst = np.zeros(3 * n.value, dtype=np.int32)
        L.check(self._lib.mp_curvelet_wedges(self._h, ctypes.byref(n),
                                             lst.ctypes.data_as(ctypes.POINTER(ctypes.c_int))))
        self.wedges = [tuple(int(v) for v in lst[3 * w:3 * w + 3]) for w in range(n.value)]
        self.nscales, self.nangles, self.mask_stride, self.nfan = nscales, nangles, mask_stride, nfan

    @property
    def nw(self):
        return len(self.wedges)

    @property
    def coef_shape(self):
        return (self.nw,) + tuple(self.problem.model_shape)

    def norms(self, stream=None):
        out = np.zeros(self.nw, dtype=np.float64)
        L.check(self._lib.mp_curvelet_norms(self.problem._ctx, self._h,
                                            out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream(stream)))
        return out

    def _coef(self, t):
        t = torch.as_tensor(t).to(device=self.problem.device, dtype=self.problem.torch_dtype).contiguous()
        if tuple(t.shape) != self.coef_shape:
            raise ValueError(f"coefficients have shape {tuple(t.shape)}, expected {self.coef_shape}")
        return t

    def _mask(self, m):
        if m is None:
            return None
        m = torch.as_tensor(m).to(device=self.problem.device, dtype=torch.uint8).contiguous()
        if tuple(m.shape) != self.coef_shape:
            raise ValueError(f"mask has shape {tuple(m.shape)}, expected {self.coef_shape}")
        return m

    def illumination(self, c, stream=None):
        c = self.problem._model(c, "c")
        mask = torch.empty(self.coef_shape, dtype=torch.uint8, device=self.problem.device)
        L.check(self._lib.mp_illumination(self.problem._ctx, self._h, _ptr(c), _ptr(mask), _stream(stream)))
        return mask

    def synthesis(self, coef, mask=None, weights=None, out=None, stream=None):
        coef = self._coef(coef)
        mask = self._mask(mask)
        w = None
        if weights is not None:
            w = np.ascontiguousarray(weights, dtype=np.float64)
            if w.shape != (self.nw,):
                raise ValueError(f"weights have shape {w.shape}, expected ({self.nw},)")
        o = out if out is not None else torch.empty(self.problem.model_shape, dtype=self.problem.torch_dtype,
                                                    device=self.problem.device)
        L.check(self._lib.mp_curvelet_synthesis(
            self.problem._ctx, self._h, _ptr(coef), None if mask is None else _ptr(mask),
            None if w is None else w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _ptr(o), _stream(stream)))
        self._keep = (coef, mask)       # inputs must outlive the enqueued work
        return o

    def analysis(self, img, out=None, stream=None):
        img = self.problem._model(img, "img")
        o = out if out is not None else torch.empty(self.coef_shape, dtype=self.problem.torch_dtype,
                                                    device=self.problem.device)
        L.check(self._lib.mp_curvelet_analysis(self.problem._ctx, self._h, _ptr(img), _ptr(o), _stream(stream)))
        return o

    def sign_threshold(self, coef, threshold, stream=None):
        """In place: coefficients of magnitude >= threshold become their sign, the rest 0."""
        coef = self._coef(coef) if not (isinstance(coef, torch.Tensor) and coef.is_cuda) else coef
        if tuple(coef.shape) != self.coef_shape or coef.dtype != self.problem.torch_dtype or not coef.is_contiguous():
            raise ValueError(f"coefficients must be a contiguous {self.problem.torch_dtype} array {self.coef_shape}")
        L.check(self._lib.mp_curvelet_sign_threshold(self.problem._ctx, self._h, _ptr(coef), float(threshold),
                                                     _stream(stream)))
        return coef

    def trial(self, z, mask, sigma=1.0, stream=None):
        """Randomized curvelet trial function: coefficients sigma ||phi_w|| z on the mask."""
        return self.synthesis(z, mask, sigma * self.norms(stream), stream=stream)

    def project(self, img, mask, stream=None):
        """The image's components on the masked curvelets: synthesis(mask * analysis(img))."""
        return self.synthesis(self.analysis(img, stream=stream), mask, stream=stream)

    def __del__(self):
        try:
            if self._h.value:
                self._lib.mp_curvelet_destroy(self._h)
        except Exception:
            pass
