"""Closed-form wavefields of a point source in a constant medium (test pins).

For ``m u_tt - Lap u = delta(x) w(t)`` with ``m = 1/c^2`` and a wavelet that
is zero before t = 0 (the discrete source starts at step 0):

* 3D: u(r, t) = w(t - r/c) / (4 pi r);
* 2D: u(r, t) = (1 / 2 pi) * integral_0^{acosh(c t / r)} w(t - (r/c) cosh s) ds
  for t > r/c, and 0 before (the 2D Green's function 1/(2 pi c sqrt(c^2 t^2 -
  r^2)) convolved with c^2 w, after the substitution t - tau = (r/c) cosh s).
"""
import numpy as np
from scipy import integrate


def green2d(w, r, c, t):
    """2D field at distance r and times t (array) for wavelet callable w."""
    out = np.zeros(len(t))
    for i, ti in enumerate(t):
        if c * ti <= r:
            continue
        smax = np.arccosh(c * ti / r)
        val, _ = integrate.quad(lambda s: w(ti - (r / c) * np.cosh(s)), 0.0, smax,
                                limit=400, epsabs=1e-13, epsrel=1e-11)
        out[i] = val / (2.0 * np.pi)
    return out


def green3d(w, r, c, t):
    tt = np.asarray(t) - r / c
    return np.where(tt >= 0.0, w(tt), 0.0) / (4.0 * np.pi * r)
