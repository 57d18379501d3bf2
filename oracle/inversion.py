"""FP64 CPU oracle of the linearised inversion around the probed inverse (test
infrastructure only).

Sec. 1 of the paper: the normal equations H dm = b with b = F* d the migrated image
(least squares for the linearised modelling), solved by brute-force descent (Sec. 2:
200 gradient-descent steps give the reference image) or, as the paper suggests, by a
Krylov solver with the fitted inverse as preconditioner.  Two kinds of fitted
preconditioners (Sec. 2):
  Rn  fitted from n random trial functions y_t and x_t = H y_t (Sec. 1.4);
  Kn  fitted from the Krylov subspace of the migrated image: the pairs
      (y_j, x_j) = (H^(j-1) b, H^j b), j = 1..n, so that the fit maps H^j b back to
      H^(j-1) b (K1: migrated and remigrated image).
The solvers take the operator as a function (matvec) so that they can be pinned on
small dense matrices.  Errors between models are relative mean-square errors.
"""
import numpy as np


def relative_mse(m, ref):
    """||m - ref||_2 / ||ref||_2: the paper's relative mean-squared error between a
    reference model and another one (Sec. 2), a ratio of 2-norms (not squared)."""
    m = np.asarray(m, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(m - ref) / np.linalg.norm(ref))


def krylov_pairs(matvec, b, n):
    """[(y_j, x_j)] = [(H^(j-1) b, H^j b)] for j = 1..n."""
    out = []
    y = np.asarray(b, dtype=np.float64)
    for _ in range(n):
        x = matvec(y)
        out.append((y, x))
        y = x
    return out


def steepest_descent(matvec, b, steps, x0=None):
    """Gradient descent on 1/2 x.Hx - b.x with the exact step along the residual:
    r = b - H x, alpha = r.r / r.Hr, x <- x + alpha r."""
    x = np.zeros_like(np.asarray(b, dtype=np.float64)) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - matvec(x)
    for _ in range(steps):
        Hr = matvec(r)
        rr, rHr = float(np.sum(r * r)), float(np.sum(r * Hr))
        if rHr <= 0.0 or rr == 0.0:
            break
        alpha = rr / rHr
        x = x + alpha * r
        r = r - alpha * Hr
    return x


def conjugate_gradient(matvec, b, iters, precond=None, x0=None):
    """(Preconditioned) conjugate gradients on H x = b:
    r0 = b - H x0, z = M r, p = z; alpha = r.z / p.Hp; x += alpha p; r -= alpha Hp;
    z' = M r; beta = r'.z' / r.z; p = z' + beta p.  Returns x and the residual norms."""
    x = np.zeros_like(np.asarray(b, dtype=np.float64)) if x0 is None else np.array(x0, dtype=np.float64)
    M = precond if precond is not None else (lambda v: v)
    r = b - matvec(x)
    z = M(r)
    p = z.copy()
    rz = float(np.sum(r * z))
    norms = [float(np.linalg.norm(r))]
    for _ in range(iters):
        Hp = matvec(p)
        pHp = float(np.sum(p * Hp))
        if pHp == 0.0:
            break
        alpha = rz / pHp
        x = x + alpha * p
        r = r - alpha * Hp
        norms.append(float(np.linalg.norm(r)))
        z = M(r)
        rz_new = float(np.sum(r * z))
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, norms


def misfit(P, c, d_obs):
    """Residual data r = d - F[m] at m = 1/c^2 and J = 1/2 r.r (Sec. 1.1, output least squares)."""
    r = np.asarray(d_obs, dtype=np.float64) - P.model_data(1.0 / P.c_pad ** 2)
    return r, 0.5 * float(np.sum(r * r))


def gauss_newton(problem_at, c0, d_obs, outer, inner, precond_at=None, line_search=False):
    """Gauss-Newton iterations on J[m] = 1/2 ||d - F[m]||^2 over m = 1/c^2 (Sec. 1.1).

    At c_k (problem_at(c_k) gives the operators linearised there): residual data
    r = d - F[m_k]; the gradient is -F* r, so the Newton step with the Hessian
    replaced by H = F*F solves H dm = F* r, here by `inner` CG iterations from zero
    (preconditioned by precond_at(P, b) when given; b = F* r lets it fit Kn).  With
    inner = 0 the step is the preconditioner applied to the migrated residual,
    dm = P F* r: the fitted inverse in place of H^-1, as Sec. 2.2 describes for the
    iterations after the first; with line_search the step is scaled to minimise the
    quadratic model 1/2 dm.H dm - b.dm along it: alpha = dm.b / dm.H dm.
    m_{k+1} = m_k + dm on the model grid, c_{k+1} = m_{k+1}^(-1/2).  Returns the velocity
    iterates and the misfits J(c_k), the last one at the final velocity."""
    c = np.asarray(c0, dtype=np.float64)
    cs, Js = [c], []
    for _ in range(outer):
        P = problem_at(c)
        r, J = misfit(P, c, d_obs)
        Js.append(J)
        b = P.apply_Fadj(r)
        if inner == 0:
            dm = precond_at(P, b)(b)
            if line_search:
                dm = dm * (float(np.sum(dm * b)) / float(np.sum(dm * P.apply_H(dm))))
        else:
            M = None if precond_at is None else precond_at(P, b)
            dm, _ = conjugate_gradient(P.apply_H, b, inner, precond=M)
        m = 1.0 / c ** 2 + dm
        if np.any(m <= 0.0):
            raise ValueError("Gauss-Newton step leaves m = 1/c^2 non-positive")
        c = 1.0 / np.sqrt(m)
        cs.append(c)
    Js.append(misfit(problem_at(c), c, d_obs)[1])
    return cs, Js
