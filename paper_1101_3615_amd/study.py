"""Generalization of the probed inverse (Sec. 2.2 of the paper, "Rn" preconditioners).

The preconditioner Rn fits the inverse-Hessian symbol from n trial functions y_t
and their images x_t = H y_t (Sec. 1.4), then is evaluated on a trial function y'
drawn independently of them: the relative mean-squared error (defined in the
paper's numerical section as a ratio of 2-norms, not of their squares) of
reconstructing y' from H y' through the fitted series,

    MSE = || sum_i c_i B_i (H y') - y' ||_2 / || y' ||_2,

as a function of the number p of basis terms.  Below 1, the preconditioner helps.
Everything runs through the library's operators (apply_H, probe_fit, apply_Hinv).
"""
import numpy as np

from .inversion import relative_mse
from .problem import apply_Hinv, probe_fit


def paper_bases(ndim, sizes, order=-1, tl_scale=0.5):
    """Nested bases of the paper's expansion with growing p: for each (m, a, r) in
    sizes, Fourier modes with |m_axis| <= m (cos and sin, the constant once), angular
    indices 0..a and rational Chebyshev degrees 0..r (order -1: the symbol order of
    the inverse Hessian)."""
    import itertools

    from .problem import Basis
    out = []
    for m, a, r in sizes:
        modes = [(0,) * ndim + (0,)]
        for ms in itertools.product(range(m + 1), repeat=ndim):
            if any(ms):
                modes += [tuple(ms) + (0,), tuple(ms) + (1,)]
        mults = [(ai, ri) for ai in range(a + 1) for ri in range(r + 1)]
        if len(modes) * len(mults) > 64:
            raise ValueError("at most 64 basis terms")
        out.append(Basis.fourier_angular(modes, mults, ndim, order=order, tl_scale=tl_scale))
    return out


def generalization(problem, bases, ys_fit, y_new, xs_fit=None):
    """[(p, relative MSE on y_new, relative residual of the fit, rank deficient), ...]
    for the preconditioner fitted on the pairs (ys_fit, H ys_fit), or (ys_fit, xs_fit)
    when given (Kn: the Krylov pairs of the migrated image), with each basis (torch
    tensors on the problem's device)."""
    xs = [problem.apply_H(y).clone() for y in ys_fit] if xs_fit is None else list(xs_fit)
    x_new = problem.apply_H(y_new).clone()
    out = []
    for B in bases:
        c, relres, deficient = probe_fit(problem, B, ys_fit, xs, strict=False)
        rec = apply_Hinv(problem, B, c, x_new)
        mse = relative_mse(problem, rec, y_new)
        out.append((B.p, mse, float(relres), bool(deficient)))
    return out
