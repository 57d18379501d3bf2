"""Seeded synthetic inputs: velocity models, trial functions, reflectivity.

Every array is produced in float64 and rounded to float32 once; the rounded
values are what both the oracle and the GPU path consume.  The recipes stand in
for the Marmousi model and the curvelet-masked noise of the paper (Sec. 2 and
Sec. 1.5), which are not available here:

* smooth random media: seeded N(0,1) noise filtered by a periodic Gaussian of
  standard deviation ``corr`` metres, then mapped affinely onto
  [cmin, cmax];
* trial functions: sums of randomly signed, anisotropic Gaussian wavepackets
  whose normal lies within 30 degrees of vertical and whose wavenumber is the
  normal-incidence imaged wavenumber 2 omega / c at the peak frequency, i.e.
  phase-space points that surface acquisition illuminates;
* reflectivity: dipping Gaussian lines of +-5 % of the mean of 1/c^2.
"""
import numpy as np

from .rng import Stream


def _axes_m(shape, h):
    """Coordinates in metres of a model-grid array, one 1D array per axis."""
    return [np.arange(n) * h for n in shape]


def medium(w):
    """Velocity c [m/s] on the model grid (numpy shape w.model_shape), float32."""
    m = w.medium
    shape = w.model_shape
    if m["kind"] == "gradient_bump":
        ax = _axes_m(shape, w.h)
        z = ax[0].reshape((-1,) + (1,) * (w.ndim - 1))
        xc = [(n - 1) * w.h / 2.0 for n in shape]
        r2 = np.zeros(shape)
        for d in range(w.ndim):
            a = ax[d].reshape([-1 if i == d else 1 for i in range(w.ndim)])
            r2 = r2 + (a - xc[d]) ** 2
        c = m["c0"] + m["grad"] * z + m["bump"] * np.exp(-r2 / (2 * m["sigma"] ** 2))
        c = np.broadcast_to(c, shape)
    elif m["kind"] == "smooth_random":
        st = Stream(m["seed"])
        noise = st.normal(int(np.prod(shape))).reshape(shape)
        sig = m["corr"] / w.h
        k2 = np.zeros(shape)
        for d, n in enumerate(shape):
            k = 2 * np.pi * np.fft.fftfreq(n)
            k2 = k2 + (k ** 2).reshape([-1 if i == d else 1 for i in range(w.ndim)])
        s = np.fft.ifftn(np.fft.fftn(noise) * np.exp(-0.5 * sig ** 2 * k2)).real
        s = (s - s.min()) / (s.max() - s.min())
        c = m["cmin"] + (m["cmax"] - m["cmin"]) * s
    elif m["kind"] == "constant":
        c = np.full(shape, float(m["c"]))
    else:
        raise ValueError(m["kind"])
    return np.ascontiguousarray(c, dtype=np.float64).astype(np.float32)


def wavepackets(w, c, seed, npk, window=4.0):
    """Sum of ``npk`` seeded wavepackets on the model grid, max |y| = 1, float32.

    Packet j has centre x_j, unit normal n_j, wavenumber k_j = 4 pi f / c(x_j),
    widths sigma_perp = pi / k_j across and sigma_par = 2 pi / k_j along the
    wavefront, sign s_j = +-1, and is evaluated within ``window`` sigma_par of
    its centre.
    """
    st = Stream(seed)
    shape = w.model_shape
    nd = w.ndim
    h = w.h
    cmax = float(np.max(c))
    sig_par_max = 2 * np.pi / (4 * np.pi * w.f_peak / cmax)
    margin = 3.0 * sig_par_max
    ext = [(n - 1) * h for n in shape]          # axis extents, z first
    lo = [10 * h] + [margin] * (nd - 1)
    hi = [ext[0] - margin] + [e - margin for e in ext[1:]]
    if any(l >= u for l, u in zip(lo, hi)):
        raise ValueError("model too small for the packet margin")
    cen = np.stack([st.uniform(npk, l, u) for l, u in zip(lo, hi)], axis=1)
    if nd == 2:
        th = np.deg2rad(st.uniform(npk, -30.0, 30.0))
        normals = np.stack([np.cos(th), np.sin(th)], axis=1)       # (z, x)
    else:
        cth = st.uniform(npk, np.cos(np.deg2rad(30.0)), 1.0)
        sth = np.sqrt(1.0 - cth ** 2)
        ph = st.uniform(npk, 0.0, 2 * np.pi)
        normals = np.stack([cth, sth * np.sin(ph), sth * np.cos(ph)], axis=1)
    sgn = st.signs(npk)
    if nd == 3:
        y = _packets3d(shape, h, cen, normals, sgn, w.f_peak, c, window)
    else:
        y = np.zeros(shape)
        for j in range(npk):
            idx = tuple(min(int(round(cen[j, d] / h)), shape[d] - 1) for d in range(nd))
            kj = 4 * np.pi * w.f_peak / float(c[idx])
            sperp = np.pi / kj
            spar = 2 * np.pi / kj
            r = window * spar
            sl, grids = [], []
            for d in range(nd):
                a = max(int(np.floor((cen[j, d] - r) / h)), 0)
                b = min(int(np.ceil((cen[j, d] + r) / h)) + 1, shape[d])
                sl.append(slice(a, b))
                grids.append(np.arange(a, b) * h - cen[j, d])
            mesh = np.meshgrid(*grids, indexing="ij")
            rho_perp = sum(mesh[d] * normals[j, d] for d in range(nd))
            r2 = sum(m_ ** 2 for m_ in mesh)
            rho_par2 = np.maximum(r2 - rho_perp ** 2, 0.0)
            env = np.exp(-rho_par2 / (2 * spar ** 2) - rho_perp ** 2 / (2 * sperp ** 2))
            y[tuple(sl)] += sgn[j] * env * np.cos(kj * rho_perp)
    y /= np.max(np.abs(y))
    return y.astype(np.float32)


def _packets3d(shape, h, cen, normals, sgn, f_peak, c, window):
    """The 3D packet sum of ``wavepackets`` in factored form.

    With rho_perp = sum_d n_d g_d (g_d the offsets along each axis) and
    beta = 1/(2 sigma_perp^2) - 1/(2 sigma_par^2), each packet is
    Re prod_d [exp(-g_d^2/(2 sigma_par^2) - beta n_d^2 g_d^2 + i k n_d g_d)]
    times exp(-2 beta n_d n_e g_d g_e) for the three axis pairs: the same
    function, built from 1D and 2D factors so the box costs a few products.  The
    box products run in torch (multi-threaded, exact IEEE products; every
    transcendental is taken in numpy on the 1D and 2D factors).
    """
    import torch
    y = torch.zeros(shape, dtype=torch.float64)
    for j in range(cen.shape[0]):
        idx = tuple(min(int(round(cen[j, d] / h)), shape[d] - 1) for d in range(3))
        kj = 4 * np.pi * f_peak / float(c[idx])
        sperp = np.pi / kj
        spar = 2 * np.pi / kj
        r = window * spar
        sl, g = [], []
        for d in range(3):
            a = max(int(np.floor((cen[j, d] - r) / h)), 0)
            b = min(int(np.ceil((cen[j, d] + r) / h)) + 1, shape[d])
            sl.append(slice(a, b))
            g.append(np.arange(a, b) * h - cen[j, d])
        n = normals[j]
        beta = 1.0 / (2 * sperp ** 2) - 1.0 / (2 * spar ** 2)
        one = [np.exp(-g[d] ** 2 / (2 * spar ** 2) - beta * (n[d] * g[d]) ** 2) for d in range(3)]
        ph = [kj * n[d] * g[d] for d in range(3)]
        zy = np.exp(-2 * beta * n[0] * n[1] * np.outer(g[0], g[1]))
        zx = np.exp(-2 * beta * n[0] * n[2] * np.outer(g[0], g[2]))
        yx = np.exp(-2 * beta * n[1] * n[2] * np.outer(g[1], g[2]))
        # (z, y) and (y, x) complex factors, real and imaginary parts
        a2 = np.outer(one[0], one[1]) * zy
        ar = a2 * np.cos(np.add.outer(ph[0], ph[1]))
        ai = a2 * np.sin(np.add.outer(ph[0], ph[1]))
        b2 = one[2][None, :] * yx
        br = b2 * np.cos(ph[2])[None, :]
        bi = b2 * np.sin(ph[2])[None, :]
        t = lambda v: torch.from_numpy(np.ascontiguousarray(v))
        box = (t(ar)[:, :, None] * t(br)[None, :, :] - t(ai)[:, :, None] * t(bi)[None, :, :]) * t(zx)[:, None, :]
        y[tuple(sl)] += float(sgn[j]) * box
    return y.numpy()


def trials(w, c=None):
    """The workload's trial functions, one float32 array per seed."""
    if c is None:
        c = medium(w)
    return [wavepackets(w, c, s, w.packets_per_trial) for s in w.trial_seeds]


def reflectivity(w, c=None, seed=None, nrefl=12, width_cells=1.5,
                 max_dip_deg=20.0, rel_amp=0.05):
    """Dipping Gaussian-line reflectors (2D), float32, on the model grid."""
    if w.ndim != 2:
        raise ValueError("reflectivity is defined for 2D workloads")
    if c is None:
        c = medium(w)
    st = Stream(w.refl_seed if seed is None else seed)
    m0 = 1.0 / np.asarray(c, dtype=np.float64) ** 2
    amp = rel_amp * float(np.mean(m0))
    nz, nx = w.model_shape
    z = (np.arange(nz) * w.h)[:, None]
    x = (np.arange(nx) * w.h)[None, :]
    zc = st.uniform(nrefl, 0.1 * (nz - 1) * w.h, 0.9 * (nz - 1) * w.h)
    xc = st.uniform(nrefl, 0.25 * (nx - 1) * w.h, 0.75 * (nx - 1) * w.h)
    dip = np.deg2rad(st.uniform(nrefl, -max_dip_deg, max_dip_deg))
    sgn = st.signs(nrefl)
    sw = width_cells * w.h
    out = np.zeros((nz, nx))
    for l in range(nrefl):
        dist = -(x - xc[l]) * np.sin(dip[l]) + (z - zc[l]) * np.cos(dip[l])
        out += sgn[l] * amp * np.exp(-dist ** 2 / (2 * sw ** 2))
    return out.astype(np.float32)


def normal_field(shape, seed, dtype=np.float32):
    """i.i.d. N(0,1) array of the given shape (model vectors, data vectors)."""
    st = Stream(seed)
    return st.normal(int(np.prod(shape))).reshape(shape).astype(dtype)


def tiny(ndim=2, n=16, nb=8, nt=200, ns=2, nr=16, h=10.0, dt=1.0e-3,
         f_peak=20.0, c=2000.0, dtype="f64", snap="full", ckpt_every=0,
         kind="constant", seed=21):
    """A small workload for brute-force and unit checks."""
    from .configs import Workload, _row0
    if kind == "constant":
        med = dict(kind="constant", c=c)
    else:
        med = dict(kind="smooth_random", cmin=0.8 * c, cmax=1.2 * c,
                   corr=4 * h, seed=seed)
    srcx = [int((s + 0.5) * n / ns) for s in range(ns)]
    recx = np.linspace(0, n - 1, nr).round().astype(int)
    if ndim == 2:
        src = _row0(srcx, 2)
        rec = _row0(recx, 2)
    else:
        src = _row0(srcx, 3, [n // 2] * ns)
        rec = _row0(recx, 3, [(n // 2 + i) % n for i in range(nr)])
    return Workload(name=f"tiny{ndim}d_{n}", ndim=ndim, nx=n, nz=n,
                    ny=(n if ndim == 3 else 1), h=h, nb=nb, dt=dt, nt=nt,
                    f_peak=f_peak, src=src, rec=rec, dtype=dtype, snap=snap,
                    ckpt_every=ckpt_every, medium=med,
                    legendre=[(0,) * ndim, (1,) + (0,) * (ndim - 1)],
                    trial_seeds=(seed + 1,), packets_per_trial=2)


def bandlimited_data(shape, seed, dt, f_peak):
    """Seeded data traces [..., nt, nr] with a Ricker amplitude spectrum, float32.

    White N(0,1) samples filtered along time by |R(f)| = f^2 / f_peak^2
    exp(1 - f^2 / f_peak^2) (peak 1 at f_peak), then scaled to unit RMS: data of
    the band that the sources put into the medium, for applying F* to traces
    other than Born data of a known model.
    """
    x = normal_field(shape, seed, np.float64)
    nt = shape[-2]
    f = np.fft.rfftfreq(nt, dt)
    amp = (f / f_peak) ** 2 * np.exp(1.0 - (f / f_peak) ** 2)
    y = np.fft.irfft(np.fft.rfft(x, axis=-2) * amp[:, None], n=nt, axis=-2)
    y /= np.sqrt(np.mean(y * y))
    return y.astype(np.float32)
