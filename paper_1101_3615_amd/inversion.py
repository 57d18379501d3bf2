"""Linearised inversion around the probed inverse (Sec. 1 and Sec. 2 of the paper).

The normal equations H dm = b, b = F* d the migrated image, solved by steepest
descent with exact steps (Sec. 2 takes 200 gradient-descent steps as the reference
image) or by conjugate gradients preconditioned with a fitted inverse (the paper's
motivation, Sec. 1).  Two fitted preconditioners (Sec. 2): Rn from n random trial
functions (probe_fit on (y_t, H y_t)) and Kn from the Krylov subspace of the
migrated image, the pairs (H^(j-1) b, H^j b), j = 1..n.

Every step runs in the library's kernels: the operators (apply_H, apply_Hinv, probe_fit,
model, apply_Fadj) and the solvers' vector work (dot products with FP64 accumulation,
y = alpha x + beta y, the velocity update of Gauss-Newton); torch only holds the vectors.
"""
import torch

from . import _lib as L
from .problem import apply_Hinv, probe_fit


def relative_mse(problem, m, ref):
    """||m - ref||_2 / ||ref||_2 (the paper's relative MSE between models, Sec. 2: a ratio
    of norms, not of squared norms), with the library's vector kernels (FP64 dot in a
    fixed order).  m and ref are cast to the problem's precision and device."""
    P = problem
    ref = ref.to(device=P.device, dtype=P.torch_dtype).contiguous()
    diff = m.to(device=P.device, dtype=P.torch_dtype).contiguous().clone()
    P.axpby(-1.0, ref, 1.0, diff)
    return (P.dot(diff, diff) / P.dot(ref, ref)) ** 0.5


def krylov_pairs(problem, b, n):
    """([y_1..y_n], [x_1..x_n]) with y_1 = b, x_j = H y_j, y_{j+1} = x_j."""
    ys, xs = [], []
    y = b
    for _ in range(n):
        x = problem.apply_H(y)
        ys.append(y)
        xs.append(x)
        y = x
    return ys, xs


def fit_krylov(problem, basis, b, n):
    """Kn: coefficients fitted on the Krylov pairs of b (c, relres, rank_deficient)."""
    ys, xs = krylov_pairs(problem, b, n)
    return probe_fit(problem, basis, ys, xs, strict=False)


def preconditioner(problem, basis, c):
    """v -> sum_i c_i B_i v (the fitted inverse as a function)."""
    return lambda v: apply_Hinv(problem, basis, c, v)


def steepest_descent(problem, b, steps):
    """x <- x + alpha r with r = b - H x and alpha = r.r / r.Hr, from x = 0.  Returns x
    and the values of the functional 1/2 x.Hx - b.x = -1/2 (x.b + x.r), one per iterate
    (the first for x = 0); exact steps make them non-increasing."""
    P = problem
    x = torch.zeros_like(b)
    r = b.clone()
    phis = [0.0]
    for _ in range(steps):
        Hr = P.apply_H(r)
        rr, rHr = P.dot(r, r), P.dot(r, Hr)
        if rHr <= 0.0 or rr == 0.0:
            break
        alpha = rr / rHr
        P.axpby(alpha, r, 1.0, x)
        P.axpby(-alpha, Hr, 1.0, r)
        phis.append(-0.5 * (P.dot(x, b) + P.dot(x, r)))
    return x, phis


def conjugate_gradient(problem, b, iters, precond=None):
    """(Preconditioned) conjugate gradients on H x = b from x = 0; returns x and the
    residual norms (one per iteration, the first for x = 0)."""
    P = problem
    x = torch.zeros_like(b)
    r = b.clone()
    z = precond(r) if precond is not None else r.clone()
    p = z.clone()
    rz = P.dot(r, z)
    norms = [P.dot(r, r) ** 0.5]
    for _ in range(iters):
        Hp = P.apply_H(p)
        pHp = P.dot(p, Hp)
        if pHp == 0.0:
            break
        alpha = rz / pHp
        P.axpby(alpha, p, 1.0, x)
        P.axpby(-alpha, Hp, 1.0, r)
        norms.append(P.dot(r, r) ** 0.5)
        z = precond(r) if precond is not None else r.clone()
        rz_new = P.dot(r, z)
        P.axpby(1.0, z, rz_new / rz, p)
        rz = rz_new
    return x, norms


def misfit(problem, d_obs):
    """Residual data r = d - F[m] at the current background and J = 1/2 r.r (Sec. 1.1)."""
    r = problem.model()
    problem.axpby(1.0, d_obs, -1.0, r)
    return r, 0.5 * problem.dot(r, r)


def gauss_newton(problem, c0, d_obs, outer, inner, precond_at=None, line_search=False):
    """Gauss-Newton on J[m] = 1/2 ||d - F[m]||^2 over m = 1/c^2 (Sec. 1.1).

    At c_k: r = d - F[m_k] (nonlinear modelling), the migrated residual b = F* r
    (minus the gradient of J), the step dm from `inner` CG iterations on H dm = b
    (preconditioned by precond_at(problem, b), a probed inverse fitted at c_k: Rn, or Kn
    on the Krylov pairs of b), or with inner = 0 the preconditioner applied to b (the
    fitted inverse in place of H^-1, Sec. 2.2), scaled with line_search by
    alpha = dm.b / dm.H dm (the minimum of the quadratic model along it);
    m_{k+1} = m_k + dm, c_{k+1} = m_{k+1}^(-1/2)
    (in the library's kernel, which refuses a step that makes m non-positive).  Leaves the
    problem's background at the last iterate; returns the velocity iterates and the
    misfits J(c_k)."""
    d_obs = problem._vec(d_obs, "d_obs")
    c = c0.to(device=problem.device, dtype=problem.torch_dtype).contiguous().clone()
    cs, Js = [c], []
    for _ in range(outer):
        problem.set_background(c)
        r, J = misfit(problem, d_obs)
        Js.append(J)
        b = problem.apply_Fadj(r)
        if inner == 0:
            dm = precond_at(problem, b)(b)
            if line_search:
                alpha = problem.dot(dm, b) / problem.dot(dm, problem.apply_H(dm))
                problem.axpby(0.0, dm, alpha, dm)
        else:
            dm, _ = conjugate_gradient(problem, b, inner,
                                       precond=None if precond_at is None else precond_at(problem, b))
        c = c.clone()
        try:
            problem.velocity_update(c, dm)
        except L.MatprobeError as e:
            if e.code == L.MP_ENUMERIC:
                raise ValueError("Gauss-Newton step leaves m = 1/c^2 non-positive") from e
            raise
        cs.append(c)
    problem.set_background(c)
    Js.append(misfit(problem, d_obs)[1])
    return cs, Js
