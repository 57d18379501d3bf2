"""FP64 CPU oracle of curvelet-space trial functions with an illumination mask (test
infrastructure only: used by the tests, never by the product path).

Sec. 1.5 of the paper: a randomized trial function is a curvelet expansion with i.i.d.
Gaussian coefficients, of variance proportional to the atom's squared norm, on the set S of
curvelets whose centre (x_mu, k_mu) is visible in the acquisition (a ray pair from x_mu,
specular about the normal k_mu, links x_mu to the source manifold and to the receiver
manifold), and zero elsewhere; Sec. 2 (other tests) builds S from straight lines in a uniform
medium and from ray tracing (the Hamiltonian system of geometrical optics, adaptive
Runge-Kutta) in smooth media.

The curvelet frame here is undecimated and built in the frequency domain on the periodic
model grid (nz x nx, powers of two), 2D only:
  * normalised frequency u = (f_x / (nx/2), f_z / (nz/2)), radius r = |u|, angle
    theta = atan2(u_z, u_x) mod pi (the same angle as the physical wavevector's);
  * smooth step nu(t) = t^4 (35 - 84 t + 70 t^2 - 20 t^3) on [0, 1] (nu(t) + nu(1-t) = 1);
  * octave lowpass Phi(s) = 1 (s <= 1), cos(pi/2 nu(s - 1)) (1 < s < 2), 0 (s >= 2);
  * J scales: L_j(r) = Phi(r / 2^(j - J + 1)) for j < J - 1, L_(J-1) = 1; W_0 = L_0 (the
    lowpass), W_j = sqrt(L_j^2 - L_(j-1)^2) for j >= 1, so sum_j W_j^2 = 1;
  * band j >= 1 has A_j = A_1 2^floor((j-1)/2) directions over a half turn (parabolic
    scaling), centres theta_l = (l + 1/2) pi / A_j, and angular windows V_(j,l) from the
    same smooth step with sum_l V_(j,l)^2 = 1;
  * wedge windows U = W_j V_(j,l) (U_0 = W_0), real and even in the frequency, so
    sum_w U_w^2 = 1 and the atoms phi_w(x - x_k) = IFFT(U_w)(x - x_k), one per grid point
    x_k, form a tight frame: analysis C_w = IFFT(U_w FFT f), synthesis
    f = sum_w IFFT(U_w FFT C_w).
"""
import numpy as np

# ---------------------------------------------------------------- windows --


def smooth_step(t):
    """nu(t): 0 for t <= 0, 1 for t >= 1, t^4 (35 - 84 t + 70 t^2 - 20 t^3) between."""
    t = np.clip(np.asarray(t, dtype=np.float64), 0.0, 1.0)
    return t ** 4 * (35.0 - 84.0 * t + 70.0 * t ** 2 - 20.0 * t ** 3)


def lowpass(s):
    """Phi(s): 1 up to s = 1, a smooth cosine roll-off to 0 at s = 2."""
    s = np.asarray(s, dtype=np.float64)
    return np.where(s <= 1.0, 1.0, np.where(s >= 2.0, 0.0, np.cos(0.5 * np.pi * smooth_step(s - 1.0))))


def directions(j, A1):
    """A_j, the number of directions of band j >= 1 over a half turn."""
    return A1 * 2 ** ((j - 1) // 2)


def wedges(J, A1):
    """[(j, l, A_j)] in the frame's order: the lowpass (0, 0, 0), then band by band."""
    out = [(0, 0, 0)]
    for j in range(1, J):
        A = directions(j, A1)
        out += [(j, l, A) for l in range(A)]
    return out


def frequency_grid(nz, nx):
    """r and theta (mod pi) of every FFT bin of an nz x nx grid (numpy FFT order)."""
    fz = np.fft.fftfreq(nz) * nz / (nz / 2.0)
    fx = np.fft.fftfreq(nx) * nx / (nx / 2.0)
    uz, ux = np.meshgrid(fz, fx, indexing="ij")
    r = np.hypot(ux, uz)
    theta = np.mod(np.arctan2(uz, ux), np.pi)
    return r, theta


def radial_windows(r, J):
    """[W_0 .. W_(J-1)] at radii r."""
    L = [lowpass(r / 2.0 ** (j - J + 1)) for j in range(J - 1)] + [np.ones_like(r)]
    W = [L[0]]
    for j in range(1, J):
        W.append(np.sqrt(np.maximum(L[j] ** 2 - L[j - 1] ** 2, 0.0)))
    return W


def angular_window(theta, l, A):
    """V_(l) of A directions over [0, pi): sin(pi/2 nu(s)) rising, cos(pi/2 nu(s - 1))
    falling, s = (theta A / pi - l + 1/2) mod A; centred at theta_l = (l + 1/2) pi / A."""
    s = np.mod(np.asarray(theta, dtype=np.float64) * A / np.pi - l + 0.5, A)
    return np.where(s < 1.0, np.sin(0.5 * np.pi * smooth_step(s)),
                    np.where(s < 2.0, np.cos(0.5 * np.pi * smooth_step(s - 1.0)), 0.0))


def windows(nz, nx, J, A1):
    """U[w] on the FFT grid, w in the order of wedges(J, A1).  The Nyquist row and column
    alias +f and -f, so the raw windows are not even there; every window is replaced by the
    root mean square of its values at xi and -xi, which keeps sum_w U_w^2 = 1 and makes
    each U_w even (elsewhere it changes nothing: sqrt(a^2) = a)."""
    r, theta = frequency_grid(nz, nx)
    W = radial_windows(r, J)
    U = np.stack([W[0] if j == 0 else W[j] * angular_window(theta, l, A) for j, l, A in wedges(J, A1)])
    Um = U[:, (-np.arange(nz)) % nz][:, :, (-np.arange(nx)) % nx]
    return np.sqrt(0.5 * (U * U + Um * Um))


def atom_norms(U):
    """||phi_w||_2 = sqrt(sum_xi U_w^2 / N) (Parseval with numpy's FFT normalisation)."""
    N = U.shape[-1] * U.shape[-2]
    return np.sqrt(np.sum(U ** 2, axis=(-2, -1)) / N)


def analysis(f, U):
    """C[w] = IFFT(U_w FFT f) (correlation with the real, even atoms)."""
    F = np.fft.fft2(np.asarray(f, dtype=np.float64))
    return np.real(np.fft.ifft2(U * F[None]))


def synthesis(C, U, mask=None, weights=None):
    """sum_w IFFT(U_w FFT(weights_w mask_w C_w))."""
    C = np.asarray(C, dtype=np.float64)
    if mask is not None:
        C = C * mask
    if weights is not None:
        C = C * np.asarray(weights, dtype=np.float64)[:, None, None]
    return np.real(np.fft.ifft2(np.sum(U * np.fft.fft2(C), axis=0)))


def trial(z, U, mask, sigma=1.0):
    """A randomized curvelet trial function (Sec. 1.5): coefficients sigma ||phi_w|| z on the
    visible set (z i.i.d. N(0, 1), passed in), zero elsewhere, synthesised."""
    return synthesis(z, U, mask, sigma * atom_norms(U))


# -------------------------------------------------------------- rays --

# Dormand-Prince 5(4) tableau (Dormand and Prince, 1980)
DP_A = [
    [],
    [1 / 5],
    [3 / 40, 9 / 40],
    [44 / 45, -56 / 15, 32 / 9],
    [19372 / 6561, -25360 / 2187, 64448 / 6561, -212 / 729],
    [9017 / 3168, -355 / 33, 46732 / 5247, 49 / 176, -5103 / 18656],
    [35 / 384, 0.0, 500 / 1113, 125 / 192, -2187 / 6784, 11 / 84],
]
DP_B5 = [35 / 384, 0.0, 500 / 1113, 125 / 192, -2187 / 6784, 11 / 84, 0.0]
DP_B4 = [5179 / 57600, 0.0, 7571 / 16695, 393 / 640, -92097 / 339200, 187 / 2100, 1 / 40]


class Medium:
    """Bilinear interpolation of c and of its centred-difference gradient (one-sided at the
    edges) between the model-grid nodes (x, z) = (ix h, iz h); positions are clamped to the
    grid's box."""

    def __init__(self, c, h):
        self.c = np.asarray(c, dtype=np.float64)
        self.h = float(h)
        self.nz, self.nx = self.c.shape
        self.gx = np.gradient(self.c, self.h, axis=1, edge_order=1) if self.nx > 1 else np.zeros_like(self.c)
        self.gz = np.gradient(self.c, self.h, axis=0, edge_order=1) if self.nz > 1 else np.zeros_like(self.c)

    def _bilinear(self, a, x, z):
        fx = np.clip(x / self.h, 0.0, self.nx - 1.0)
        fz = np.clip(z / self.h, 0.0, self.nz - 1.0)
        ix = np.minimum(np.floor(fx).astype(np.int64), self.nx - 2) if self.nx > 1 else np.zeros_like(fx, np.int64)
        iz = np.minimum(np.floor(fz).astype(np.int64), self.nz - 2) if self.nz > 1 else np.zeros_like(fz, np.int64)
        tx, tz = fx - ix, fz - iz
        ix1 = np.minimum(ix + 1, self.nx - 1)
        iz1 = np.minimum(iz + 1, self.nz - 1)
        top = a[iz, ix] * (1.0 - tx) + a[iz, ix1] * tx
        bot = a[iz1, ix] * (1.0 - tx) + a[iz1, ix1] * tx
        return top * (1.0 - tz) + bot * tz

    def eval(self, x, z):
        return self._bilinear(self.c, x, z), self._bilinear(self.gx, x, z), self._bilinear(self.gz, x, z)


def ray_rhs(med, y):
    """Kinematic ray equations with the traveltime as parameter: dx/dt = c^2 p,
    dp/dt = -grad(c) / c, y = (x, z, p_x, p_z) (rows)."""
    c, cx, cz = med.eval(y[0], y[1])
    return np.stack([c * c * y[2], c * c * y[3], -cx / c, -cz / c])


def trace_to_depth(med, x0, z0, dx, dz, z_s, rtol=1e-4, max_steps=4000):
    """Trace rays from (x0, z0) with unit initial directions (dx, dz) (z down) until they
    cross the depth z_s upwards.  Returns (reached, x_cross): reached is False for rays that
    leave the box [0, (nx-1)h] x [.., (nz-1)h] first, turn away for good, or run out of
    steps.  Step control: the 5th/4th-order position difference e per step must satisfy
    |e| <= rtol h; a rejected step halves dt, an accepted one with |e| < rtol h / 32 doubles
    it, the step length capped at 8 h.  The crossing point is linear between the last two
    positions.  Vectorised over rays; each ray's arithmetic is its own."""
    x0, z0, dx, dz = (np.atleast_1d(np.asarray(v, dtype=np.float64)) for v in (x0, z0, dx, dz))
    n = x0.size
    h = med.h
    xmax, zmax = (med.nx - 1) * h, (med.nz - 1) * h
    c0 = med.eval(x0, z0)[0]
    y = np.stack([x0, z0, dx / c0, dz / c0])
    dt = 0.5 * h / c0
    tol2 = (rtol * h) ** 2
    reached = np.zeros(n, dtype=bool)
    xc = np.full(n, np.nan)
    # a ray starting on the manifold's depth is there at once; one above it never gets there
    at = z0 <= z_s
    reached[at] = z0[at] == z_s
    xc[reached] = x0[reached]
    live = ~at
    for _ in range(max_steps):
        if not live.any():
            break
        idx = np.nonzero(live)[0]
        yi = y[:, idx]
        hi = dt[idx]
        k = []
        for s in range(7):
            ys = yi.copy()
            for m, a in enumerate(DP_A[s]):
                if a != 0.0:
                    ys = ys + hi * a * k[m]
            k.append(ray_rhs(med, ys))
        y5 = yi.copy()
        y4 = yi.copy()
        for m in range(7):
            if DP_B5[m] != 0.0:
                y5 = y5 + hi * DP_B5[m] * k[m]
            if DP_B4[m] != 0.0:
                y4 = y4 + hi * DP_B4[m] * k[m]
        e2 = (y5[0] - y4[0]) ** 2 + (y5[1] - y4[1]) ** 2
        ok = e2 <= tol2
        # rejected: halve and retry
        dt[idx[~ok]] = hi[~ok] * 0.5
        acc = idx[ok]
        if acc.size:
            yo, yn = yi[:, ok], y5[:, ok]
            cross = yn[1] <= z_s
            out = (~cross) & ((yn[0] < 0.0) | (yn[0] > xmax) | (yn[1] > zmax))
            # crossing: linear between the two positions
            f = (yo[1] - z_s) / (yo[1] - yn[1])
            xcr = yo[0] + (yn[0] - yo[0]) * f
            inside = cross & (xcr >= 0.0) & (xcr <= xmax)
            r = acc[inside]
            reached[r] = True
            xc[r] = xcr[inside]
            live[acc[cross | out]] = False
            y[:, acc] = yn
            grow = e2[ok] < tol2 / 1024.0
            nd = np.where(grow, hi[ok] * 2.0, hi[ok])
            cn = med.eval(yn[0], yn[1])[0]
            dt[acc] = np.minimum(nd, 8.0 * h / cn)
    return reached, xc


# -------------------------------------------------------------- illumination --


def mask_nodes(n, stride):
    """Coarse node centres along one axis: min(a s + (s - 1) // 2, n - 1), a = 0 .. ceil(n/s) - 1."""
    return np.minimum(np.arange((n + stride - 1) // stride) * stride + (stride - 1) // 2, n - 1)


def direction_set(J, A1):
    """Distinct normal directions of the directional bands: [(A, l)] for each distinct A_j in
    increasing order, l = 0 .. A - 1; theta = (l + 1/2) pi / A."""
    As = sorted({directions(j, A1) for j in range(1, J)})
    return [(A, l) for A in As for l in range(A)]


def ray_pairs(A, l, nfan):
    """Unit directions (dx, dz) of the ray pairs of normal theta = (l + 1/2) pi / A: the normal
    pointing up, n = -(cos theta, sin theta), turned by +alpha and -alpha,
    alpha_i = (i + 1/2) (pi/2) / nfan.  Returns (plus, minus), each of shape (nfan, 2)."""
    th = (l + 0.5) * np.pi / A
    nx_, nz_ = -np.cos(th), -np.sin(th)
    al = (np.arange(nfan) + 0.5) * 0.5 * np.pi / nfan
    ca, sa = np.cos(al), np.sin(al)
    plus = np.stack([nx_ * ca - nz_ * sa, nx_ * sa + nz_ * ca], 1)
    minus = np.stack([nx_ * ca + nz_ * sa, -nx_ * sa + nz_ * ca], 1)
    return plus, minus


def manifold(points, h):
    """(depth, x_lo, x_hi) of a set of model-grid cells (x, z) on one depth row; the interval
    is widened by half a cell on each side."""
    p = np.asarray(points)
    zs = np.unique(p[:, -1])
    if zs.size != 1:
        raise ValueError("the manifold's points must share one depth row")
    return float(zs[0]) * h, (p[:, 0].min() - 0.5) * h, (p[:, 0].max() + 0.5) * h


def ray_crossings(c, h, src, rec, J, A1, stride, nfan, rtol=1e-4, max_steps=4000, nodes=None):
    """Crossings of every ray of the fans: for each direction d of direction_set, coarse node
    (a, b) (all, or the (a, b) pairs listed in ``nodes``) and fan angle i, the ray turned by
    +alpha_i (k = 0) and by -alpha_i (k = 1).  Returns a dict of arrays of shape
    [ndir, nnodes, nfan, 2]: okS, xS (source row), okR, xR (receiver row), and the node
    list.  All rays are traced together; each ray's arithmetic is its own."""
    med = Medium(c, h)
    nz, nx = med.c.shape
    zi, xi = mask_nodes(nz, stride), mask_nodes(nx, stride)
    if nodes is None:
        nodes = [(a, b) for a in range(zi.size) for b in range(xi.size)]
    nodes = np.asarray(nodes, dtype=np.int64).reshape(-1, 2)
    zS, _, _ = manifold(src, h)
    zR, _, _ = manifold(rec, h)
    dirs = direction_set(J, A1)
    D, P = len(dirs), len(nodes)
    dvec = np.zeros((D, nfan, 2, 2))
    for d, (A, l) in enumerate(dirs):
        plus, minus = ray_pairs(A, l, nfan)
        dvec[d, :, 0], dvec[d, :, 1] = plus, minus
    x0 = np.broadcast_to((xi[nodes[:, 1]] * h)[None, :, None, None], (D, P, nfan, 2)).ravel()
    z0 = np.broadcast_to((zi[nodes[:, 0]] * h)[None, :, None, None], (D, P, nfan, 2)).ravel()
    dx = np.broadcast_to(dvec[:, None, :, :, 0], (D, P, nfan, 2)).ravel()
    dz = np.broadcast_to(dvec[:, None, :, :, 1], (D, P, nfan, 2)).ravel()
    okS, xS = trace_to_depth(med, x0, z0, dx, dz, zS, rtol, max_steps)
    if zR == zS:
        okR, xR = okS, xS
    else:
        okR, xR = trace_to_depth(med, x0, z0, dx, dz, zR, rtol, max_steps)
    shp = (D, P, nfan, 2)
    return dict(okS=okS.reshape(shp), xS=xS.reshape(shp), okR=okR.reshape(shp), xR=xR.reshape(shp), nodes=nodes)


def visibility_of(cross, src, rec, h, widen=0.0):
    """vis[d, node] from ray crossings: some fan angle has one ray of the pair inside the
    source span and the other inside the receiver span (spans from manifold(), grown by
    ``widen`` metres, > 0, or shrunk, < 0, for tie margins)."""
    _, sl, sh = manifold(src, h)
    _, rl, rh = manifold(rec, h)
    with np.errstate(invalid="ignore"):
        s_in = cross["okS"] & (cross["xS"] >= sl - widen) & (cross["xS"] <= sh + widen)
        r_in = cross["okR"] & (cross["xR"] >= rl - widen) & (cross["xR"] <= rh + widen)
    pair = (s_in[..., 0] & r_in[..., 1]) | (r_in[..., 0] & s_in[..., 1])
    return np.any(pair, axis=-1)


def visibility(c, h, src, rec, J, A1, stride, nfan, rtol=1e-4, max_steps=4000, widen=0.0):
    """vis[d, a, b] for each direction of direction_set and coarse node (a, b)."""
    nz, nx = np.asarray(c).shape
    cross = ray_crossings(c, h, src, rec, J, A1, stride, nfan, rtol, max_steps)
    v = visibility_of(cross, src, rec, h, widen)
    return v.reshape(v.shape[0], mask_nodes(nz, stride).size, mask_nodes(nx, stride).size)


def expand_mask(vis, J, A1, nz, nx, stride):
    """mask[w, iz, ix] (uint8) from the node visibilities: wedge (j, l) takes its direction's
    value at the node of (iz // stride, ix // stride); the lowpass is visible where any
    direction of band 1 is."""
    dirs = direction_set(J, A1)
    pos = {d: k for k, d in enumerate(dirs)}
    iz, ix = np.arange(nz) // stride, np.arange(nx) // stride
    out = []
    for j, l, A in wedges(J, A1):
        if j == 0:
            A_1 = directions(1, A1)
            v = np.any(vis[[pos[(A_1, m)] for m in range(A_1)]], axis=0)
        else:
            v = vis[pos[(A, l)]]
        out.append(v[np.ix_(iz, ix)])
    return np.stack(out).astype(np.uint8)


def straight_visibility(h, nz, nx, src, rec, J, A1, stride, nfan):
    """vis for a uniform medium from straight lines in closed form (Sec. 2: the fan of line
    pairs from each curvelet centre): a line of direction (dx, dz), dz < 0, from (x0, z0)
    meets depth zs at x0 + (zs - z0) dx / dz."""
    zi, xi = mask_nodes(nz, stride), mask_nodes(nx, stride)
    Z, X = np.meshgrid(zi * h, xi * h, indexing="ij")
    zS, sl, sh = manifold(src, h)
    zR, rl, rh = manifold(rec, h)
    xmax = (nx - 1) * h
    dirs = direction_set(J, A1)
    vis = np.zeros((len(dirs), zi.size, xi.size), dtype=bool)

    def meets(dx, dz, zs, lo, hi):
        on = (Z == zs) & (X >= lo) & (X <= hi)      # a node on the manifold's row is there at once
        if dz >= 0.0:
            return on
        xs = X + (zs - Z) * dx / dz
        return on | ((Z > zs) & (xs >= 0.0) & (xs <= xmax) & (xs >= lo) & (xs <= hi))

    for d, (A, l) in enumerate(dirs):
        plus, minus = ray_pairs(A, l, nfan)
        hit = np.zeros(Z.shape, dtype=bool)
        for i in range(nfan):
            sp, rp = meets(*plus[i], zS, sl, sh), meets(*plus[i], zR, rl, rh)
            sm, rm = meets(*minus[i], zS, sl, sh), meets(*minus[i], zR, rl, rh)
            hit |= (sp & rm) | (rp & sm)
        vis[d] = hit
    return vis
