"""FP64 CPU oracle of the probing fit and of the fitted inverse (test infrastructure only).

Basis (paper Sec. 1.2, eq. (1) and the expansion H^-1 = sum_i c_i B_i):
elementary operators of product form, a smooth function of position times a
Fourier multiplier, quantised as in eq. (1) (the multiplier acts first, the
position factor multiplies the result):

    B_(a,q) v = P_a(x~) * Re IFFT( rho^q * FFT(v) ),

with ``P_a`` a tensor product of Legendre polynomials in the cell-centre
coordinates ``x~ = -1 + (2i+1)/N`` of each model axis, ``rho = |k| h / pi`` the
wavenumber normalised to 1 at the Nyquist frequency of each axis, and a
periodic FFT on the model grid.

Fit (Sec. 1.4): with x_t = H y_t, minimise over c the stacked residual
||sum_i c_i B_i x_t - y_t|| over all trials t (the normal equations of this
least-squares problem are the paper's M c = (B x)^T y with
M_ij = x^T B_i^T B_j x).  Solved here by Householder QR of the stacked matrix.

Fast application (Sec. 1.5, last paragraph): out = sum_i c_i B_i img.
"""
import numpy as np


def legendre(deg, t):
    """P_deg(t) by Bonnet's recurrence (n+1) P_{n+1} = (2n+1) t P_n - n P_{n-1}."""
    t = np.asarray(t, dtype=np.float64)
    p0 = np.ones_like(t)
    if deg == 0:
        return p0
    p1 = t.copy()
    for n in range(1, deg):
        p0, p1 = p1, ((2 * n + 1) * t * p1 - n * p0) / (n + 1)
    return p1


def cell_centres(n):
    """x~_i = -1 + (2 i + 1) / n, the cell centres of [-1, 1]."""
    return -1.0 + (2.0 * np.arange(n) + 1.0) / n


def position_factor(degs, shape):
    """prod_axes P_{deg_axis}(x~_axis) on a grid of the given numpy shape."""
    out = np.ones(shape)
    for ax, (deg, n) in enumerate(zip(degs, shape)):
        out = out * legendre(deg, cell_centres(n)).reshape(
            [-1 if k == ax else 1 for k in range(len(shape))])
    return out


def rho(shape, h):
    """|k| h / pi on the FFT grid, k_axis = 2 pi fftfreq(N_axis, h)."""
    k2 = np.zeros(shape)
    for ax, n in enumerate(shape):
        k = 2.0 * np.pi * np.fft.fftfreq(n, d=h)
        k2 = k2 + (k ** 2).reshape([-1 if j == ax else 1 for j in range(len(shape))])
    return np.sqrt(k2) * h / np.pi


def basis_list(legendre_degs, qs):
    """Index i <-> (a, q), position factor outer, power of rho inner."""
    return [(tuple(a), int(q)) for a in legendre_degs for q in qs]


def apply_basis(v, h, legendre_degs, qs):
    """All B_i v, shape (p,) + v.shape."""
    v = np.asarray(v, dtype=np.float64)
    r = rho(v.shape, h)
    V = np.fft.fftn(v)
    out = []
    for a, q in basis_list(legendre_degs, qs):
        filt = np.fft.ifftn(V * r ** q).real
        out.append(position_factor(a, v.shape) * filt)
    return np.stack(out)


def fit(ys, xs, h, legendre_degs, qs, rank_tol=1e-12):
    """Least-squares coefficients c with y_t ~ sum_i c_i B_i x_t for all t.

    Returns (c, relres, rank_deficient): relres = ||A c - b|| / ||b|| over the
    stacked system; when sigma_min / sigma_max < rank_tol the minimum-norm
    solution is returned and rank_deficient is True.
    """
    A = np.concatenate([apply_basis(x, h, legendre_degs, qs).reshape(-1, np.size(x)).T
                        for x in xs], axis=0)
    b = np.concatenate([np.asarray(y, dtype=np.float64).ravel() for y in ys])
    sv = np.linalg.svd(A, compute_uv=False)
    deficient = bool(sv[-1] <= rank_tol * sv[0])
    if deficient:
        c = np.linalg.lstsq(A, b, rcond=rank_tol)[0]
    else:
        Q, R = np.linalg.qr(A)
        c = np.linalg.solve(R, Q.T @ b)
    relres = float(np.linalg.norm(A @ c - b) / np.linalg.norm(b))
    return c, relres, deficient


def gram(xs, ys, h, legendre_degs, qs):
    """M = A^T A and r = A^T b of the stacked system (the paper's M and (Bx)^T y)."""
    A = np.concatenate([apply_basis(x, h, legendre_degs, qs).reshape(-1, np.size(x)).T
                        for x in xs], axis=0)
    b = np.concatenate([np.asarray(y, dtype=np.float64).ravel() for y in ys])
    return A.T @ A, A.T @ b


def apply_Hinv(c, img, h, legendre_degs, qs):
    """sum_i c_i B_i img."""
    Bv = apply_basis(img, h, legendre_degs, qs)
    return np.tensordot(np.asarray(c, dtype=np.float64), Bv, axes=1)


# ---- The paper's own expansion (Sec. 1.2, the two compressed symbol expansions) ----
# Elementary operators with symbol  e^{i lambda.x} e^{i q1 theta} TL_q2(|k|) |k|^e: a
# Fourier mode in x times an angular harmonic of the direction of k times a rational
# Chebyshev function of |k|, times the power e of |k| that sets the symbol order (the
# expansion of H carries |k|; that of the inverse, whose order is -1, takes e = -1).
# Real forms are used throughout, so every B_i is a real operator:
#   position  cos(pi m.x~) or sin(pi m.x~) on the cell centres x~ of [-1, 1]^d;
#   angle     2D: 1, cos(j theta), sin(j theta) (index 0, 2j-1, 2j), theta = arg(k_x + i k_z);
#             3D: the real spherical harmonics of degree <= 2 (the paper replaces angular
#             exponentials by spherical harmonics in 3D), as polynomials of n = k/|k|;
#   radius    TL_n(r) = T_n((r - L)/(r + L)) with r = rho = |k| h / pi, times r^e.
# At k = 0 the direction is undefined: the angular factor is 1 for index 0 and 0
# otherwise, and r^e is 1 for e = 0 and 0 for e != 0.


def fourier_factor(mode, shape):
    """cos / sin(pi sum_axis m_axis x~_axis); mode = (m per numpy axis..., phase 0 cos / 1 sin)."""
    *ms, phase = mode
    arg = np.zeros(shape)
    for ax, (m, n) in enumerate(zip(ms, shape)):
        arg = arg + (np.pi * m * cell_centres(n)).reshape([-1 if k == ax else 1 for k in range(len(shape))])
    return np.sin(arg) if phase else np.cos(arg)


def wavevector(shape, h):
    """Physical wavenumbers per numpy axis on the FFT grid, broadcast to the grid."""
    ks = []
    for ax, n in enumerate(shape):
        k = 2.0 * np.pi * np.fft.fftfreq(n, d=h)
        ks.append(np.broadcast_to(k.reshape([-1 if j == ax else 1 for j in range(len(shape))]), shape))
    return ks


def angular(index, shape, h):
    """Angular harmonic `index` of the direction of k on the FFT grid (see the list above)."""
    ks = wavevector(shape, h)
    kn = np.sqrt(sum(k * k for k in ks))
    dc = kn == 0.0
    safe = np.where(dc, 1.0, kn)
    if len(shape) == 2:
        kz, kx = ks
        theta = np.arctan2(kz, kx)
        if index == 0:
            return np.ones(shape)
        j = (index + 1) // 2
        out = np.cos(j * theta) if index % 2 == 1 else np.sin(j * theta)
        return np.where(dc, 0.0, out)
    kz, ky, kx = ks
    nx, ny, nz = kx / safe, ky / safe, kz / safe
    table = [np.ones(shape), nx, ny, nz, nx * ny, ny * nz, 3.0 * nz * nz - 1.0, nx * nz, nx * nx - ny * ny]
    if index == 0:
        return table[0]
    return np.where(dc, 0.0, table[index])


def rational_chebyshev(n, r, L):
    """TL_n(r) = T_n((r - L)/(r + L)), T_n by T_{n+1} = 2 t T_n - T_{n-1}."""
    t = (np.asarray(r, dtype=np.float64) - L) / (np.asarray(r, dtype=np.float64) + L)
    t0, t1 = np.ones_like(t), t
    if n == 0:
        return t0
    for _ in range(1, n):
        t0, t1 = t1, 2.0 * t * t1 - t0
    return t1


def paper_multiplier(mult, shape, h, order, L):
    """Multiplier of the angular index mult[0] and rational Chebyshev degree mult[1]."""
    a, q2 = mult
    r = rho(shape, h)
    if order == 0:
        rp = np.ones(shape)
    else:
        rp = np.where(r == 0.0, 0.0, np.where(r == 0.0, 1.0, r) ** order)
    return angular(a, shape, h) * rational_chebyshev(q2, r, L) * rp


def paper_basis_list(modes, mults):
    """Index i <-> (mode, mult): position factor outer, multiplier inner."""
    return [(tuple(m), tuple(q)) for m in modes for q in mults]


def apply_paper_basis(v, h, modes, mults, order, L):
    """All B_i v for the paper's expansion, shape (p,) + v.shape."""
    v = np.asarray(v, dtype=np.float64)
    V = np.fft.fftn(v)
    out = []
    for mode, mult in paper_basis_list(modes, mults):
        filt = np.fft.ifftn(V * paper_multiplier(mult, v.shape, h, order, L)).real
        out.append(fourier_factor(mode, v.shape) * filt)
    return np.stack(out)


def fit_with(apply, ys, xs, rank_tol=1e-12):
    """The least-squares fit of `fit` for any basis: apply(v) returns all B_i v."""
    A = np.concatenate([apply(x).reshape(-1, np.size(x)).T for x in xs], axis=0)
    b = np.concatenate([np.asarray(y, dtype=np.float64).ravel() for y in ys])
    sv = np.linalg.svd(A, compute_uv=False)
    deficient = bool(sv[-1] <= rank_tol * sv[0])
    if deficient:
        c = np.linalg.lstsq(A, b, rcond=rank_tol)[0]
    else:
        Q, R = np.linalg.qr(A)
        c = np.linalg.solve(R, Q.T @ b)
    relres = float(np.linalg.norm(A @ c - b) / np.linalg.norm(b))
    return c, relres, deficient
