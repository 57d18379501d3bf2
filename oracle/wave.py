"""FP64 CPU oracle of the wave-equation operators F, F* and H = F*F.

Test infrastructure only: imported by the tests, the smoke check and the CPU
baseline of the benchmark, never by the product path.  Plain numpy, a Python
loop over time, no blocking or fusion.  Arrays may carry leading batch axes
(several model perturbations at once); the last ``ndim`` axes are space.

What is computed (paper Sec. 1.1 and Sec. 2):

* background field, constant-density acoustics ``m0 u_tt - Lap u = f_s`` with a
  point source times a Ricker wavelet on the surface (Sec. 2, equation of the
  incident field);
* the Born (linearised) field ``m0 du_tt - Lap du = -dm (u0)_tt`` sampled at the
  receivers: ``F dm`` (Sec. 2, linearised wave equation; F is the Frechet
  derivative of the modelling map, Sec. 1.1);
* the migration ``F* d`` (reverse-time migration, Sec. 1.1);
* the normal operator ``H = F* F`` (Sec. 1.1), stacked over shots (Sec. 2).

Discretisation (the paper uses spectral differences and a PML; the workloads
fix 8th-order finite differences and a sponge instead):

* propagation grid = model grid plus ``nb`` absorbing cells on every side;
  ``c`` is extended into the layer by edge replication; ``kappa = c^2 dt^2``;
* Laplacian: 8th-order central differences per axis, field taken as zero
  outside the propagation grid, so the discrete Laplacian is symmetric;
* damped leapfrog: ``u+ = a (2u + kappa (L u + f)) - b u-`` with
  ``a = 1 / (1 + eta dt / 2)``, ``b = (1 - eta dt / 2) a`` and a quadratic
  damping profile ``eta``;
* ``g^n = c^2 (L u^n + f^n)`` is the scheme's own second time derivative of
  the background; the Born update is the exact derivative of the discrete
  scheme with respect to ``m = 1/c^2`` (``a``, ``b`` held fixed);
* data ``d[s][n][r] = du^{n+1}(x_r)``;
* the adjoint is the exact transpose of the discrete Born map: the same
  recurrence run backwards with the data injected at the receivers, and the
  image ``I = -sum_k g^{k-1} nu^k``.

Inner products are plain sums of squares of components (Sec. 1.1).
"""
import numpy as np

# Central 8th-order weights of the second derivative: w0, w1..w4.
FD8 = np.array([-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0])
RADIUS = 4


def ricker(f_peak, t0, dt, nt):
    """Ricker wavelet (second derivative of a Gaussian, Sec. 2) at t_n = n dt."""
    t = np.arange(nt, dtype=np.float64) * dt - t0
    a = (np.pi * f_peak * t) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def laplacian(u, h, ndim):
    """8th-order Laplacian over the last ``ndim`` axes, zero outside the grid."""
    pad = [(0, 0)] * (u.ndim - ndim) + [(RADIUS, RADIUS)] * ndim
    up = np.pad(u, pad)
    lead = (slice(None),) * (u.ndim - ndim)
    core = [slice(RADIUS, RADIUS + n) for n in u.shape[u.ndim - ndim:]]
    out = (ndim * FD8[0]) * u
    for ax in range(ndim):
        n = u.shape[u.ndim - ndim + ax]
        for j in range(1, RADIUS + 1):
            plus = list(core)
            minus = list(core)
            plus[ax] = slice(RADIUS + j, RADIUS + j + n)
            minus[ax] = slice(RADIUS - j, RADIUS - j + n)
            out = out + FD8[j] * (up[lead + tuple(plus)] + up[lead + tuple(minus)])
    return out / (h * h)


def cfl_limit(ndim):
    """Largest stable c dt / h of the undamped scheme: 2 / sqrt(ndim * 2048/315)."""
    lam = -(FD8[0] + 2.0 * sum(FD8[j] * (-1.0) ** j for j in range(1, RADIUS + 1)))
    return 2.0 / np.sqrt(ndim * lam)


class Problem:
    """The discretised operators for one workload and one background velocity."""

    def __init__(self, w, c_model):
        self.w = w
        self.nd = w.ndim
        self.nb = w.nb
        self.h = float(w.h)
        self.dt = float(w.dt)
        self.nt = int(w.nt)
        c = np.asarray(c_model, dtype=np.float64)
        assert c.shape == w.model_shape
        self.c_model = c
        self.c_pad = np.pad(c, self.nb, mode="edge")
        self.kappa = self.c_pad ** 2 * self.dt ** 2
        self.csq = self.c_pad ** 2
        self.model_slice = tuple(slice(self.nb, self.nb + n) for n in w.model_shape)
        self._sponge(float(np.max(c)), float(w.sponge_R))
        self.wavelet = ricker(w.f_peak, w.wavelet_t0, self.dt, self.nt)
        # positions: workload gives (x, [y,] z); numpy axes are (z, [y,] x)
        self.src = [self._cell(p) for p in np.asarray(w.src)]
        rec = [self._cell(p) for p in np.asarray(w.rec)]
        self.rec = tuple(np.array([r[d] for r in rec]) for d in range(self.nd))

    def _cell(self, p):
        p = [int(v) + self.nb for v in p]
        return tuple(reversed(p))

    def _sponge(self, cmax, R):
        nb, h = self.nb, self.h
        eta_max = 3.0 * cmax * np.log(1.0 / R) / (2.0 * nb * h) if nb > 0 else 0.0
        eta = np.zeros(self.c_pad.shape)
        for ax, n in enumerate(self.w.model_shape):
            i = np.arange(n + 2 * nb)
            dist = np.maximum(np.maximum(nb - i, i - (n + nb - 1)), 0)
            prof = eta_max * (dist / max(nb, 1)) ** 2
            eta = eta + prof.reshape([-1 if k == ax else 1 for k in range(self.nd)])
        self.eta = eta
        self.a = 1.0 / (1.0 + eta * self.dt / 2.0)
        self.b = (1.0 - eta * self.dt / 2.0) * self.a

    # -- extension / restriction between model grid and propagation grid --
    def extend(self, v):
        """Zero extension E of model-grid arrays (leading batch axes allowed)."""
        v = np.asarray(v, dtype=np.float64)
        out = np.zeros(v.shape[: v.ndim - self.nd] + self.c_pad.shape)
        out[(Ellipsis,) + self.model_slice] = v
        return out

    def restrict(self, u):
        return u[(Ellipsis,) + self.model_slice]

    def source_term(self, s, n):
        f = np.zeros(self.c_pad.shape)
        f[self.src[s]] = self.wavelet[n] / self.h ** self.nd
        return f

    # -- background --
    def background(self, s, kappa=None, keep_g=True, snapshots=None, source=True):
        """Background sweep of shot s.

        Returns (g, traces): g[n] = c^2 (L u^n + f^n) on the model grid for
        n = 0..nt-1 (None unless keep_g), traces[n][r] = u^{n+1}(x_r).
        ``kappa`` replaces dt^2 / m0 for nonlinear modelling at another m.
        ``snapshots`` (dict) receives the full field u^n for every n >= 0 of the
        sweep when given.  ``source=False`` runs the free recurrence from
        u^{-1} = u^0 given in ``snapshots[-1]``, ``snapshots[0]``.
        """
        kap = self.kappa if kappa is None else kappa
        if source:
            u_prev = np.zeros(self.c_pad.shape)
            u = np.zeros(self.c_pad.shape)
        else:
            u_prev = np.array(snapshots[-1], dtype=np.float64)
            u = np.array(snapshots[0], dtype=np.float64)
        g = np.empty((self.nt,) + self.w.model_shape) if keep_g else None
        traces = np.empty((self.nt, len(self.rec[0])))
        if snapshots is not None:
            snapshots[0] = u.copy()
        for n in range(self.nt):
            lam = laplacian(u, self.h, self.nd)
            if source:
                lam = lam + self.source_term(s, n)
            if keep_g:
                g[n] = self.restrict(self.csq * lam)
            u_next = self.a * (2.0 * u + kap * lam) - self.b * u_prev
            traces[n] = u_next[self.rec]
            if snapshots is not None:
                snapshots[n + 1] = u_next.copy()
            u_prev, u = u, u_next
        return g, traces

    def model_data(self, m_pad):
        """Nonlinear modelling F[m] (Sec. 1.1): traces of every shot.

        ``m_pad`` = 1/c^2 on the propagation grid; the damping profile stays
        the background's.
        """
        kap = self.dt ** 2 / np.asarray(m_pad, dtype=np.float64)
        return np.stack([self.background(s, kappa=kap, keep_g=False)[1]
                         for s in range(len(self.src))])

    # -- Born and adjoint of one shot --
    def born(self, s, dm, g):
        """F_s dm: traces d[..., n, r] = du^{n+1}(x_r)."""
        dmbar = self.extend(dm)
        batch = dmbar.shape[: dmbar.ndim - self.nd]
        du_prev = np.zeros(dmbar.shape)
        du = np.zeros(dmbar.shape)
        d = np.empty(batch + (self.nt, len(self.rec[0])))
        for n in range(self.nt):
            src = dmbar * self.extend(g[n])
            du_next = (self.a * (2.0 * du + self.kappa * (laplacian(du, self.h, self.nd) - src))
                       - self.b * du_prev)
            d[(Ellipsis, n, slice(None))] = du_next[(Ellipsis,) + self.rec]
            du_prev, du = du, du_next
        return d

    def adjoint(self, s, d, g):
        """F_s* d: image on the model grid, I = -sum_k g^{k-1} nu^k."""
        d = np.asarray(d, dtype=np.float64)
        batch = d.shape[:-2]
        nu1 = np.zeros(batch + self.c_pad.shape)      # nu^{k+1}
        nu2 = np.zeros(batch + self.c_pad.shape)      # nu^{k+2}
        img = np.zeros(batch + self.w.model_shape)
        for k in range(self.nt, 0, -1):
            lam = laplacian(nu1, self.h, self.nd)
            inj = np.zeros(lam.shape)
            np.add.at(inj, (Ellipsis,) + self.rec, d[..., k - 1, :])
            nu = self.a * (2.0 * nu1 + self.kappa * (lam + inj)) - self.b * nu2
            img = img - g[k - 1] * self.restrict(nu)
            nu2, nu1 = nu1, nu
        return img

    # -- the operators over all shots --
    def apply_F(self, dm):
        """d[..., s, n, r] for every shot."""
        out = []
        for s in range(len(self.src)):
            g, _ = self.background(s)
            out.append(self.born(s, dm, g))
        return np.stack(out, axis=-3)

    def apply_Fadj(self, d):
        """sum over shots of F_s* d_s, shots added in increasing order."""
        d = np.asarray(d, dtype=np.float64)
        img = None
        for s in range(len(self.src)):
            g, _ = self.background(s)
            part = self.adjoint(s, d[..., s, :, :], g)
            img = part if img is None else img + part
        return img

    def apply_H(self, dm, shots=None):
        """H dm = sum_s F_s* F_s dm (shots in increasing order)."""
        img = None
        for s in (range(len(self.src)) if shots is None else shots):
            g, _ = self.background(s)
            part = self.adjoint(s, self.born(s, dm, g), g)
            img = part if img is None else img + part
        return img
