"""Dense F and H = F^T F on tiny grids (test pins: brute force, E[M]).

Builds F column by column from the oracle's Born map applied to every unit
model vector at once (a batch), then H = F^T F.  Only for grids of a few
hundred model cells.
"""
import numpy as np

from .wave import Problem


def dense_F(P: Problem):
    n = int(np.prod(P.w.model_shape))
    eye = np.eye(n).reshape((n,) + P.w.model_shape)
    d = P.apply_F(eye)                        # (n, ns, nt, nr)
    return d.reshape(n, -1).T                 # data x model


def dense_H(P: Problem):
    Fm = dense_F(P)
    return Fm.T @ Fm


def basis_matrices(shape, h, legendre_degs, qs):
    """Dense B_i (p, n, n): column j is B_i applied to the j-th unit vector."""
    from .symbol import apply_basis
    n = int(np.prod(shape))
    cols = []
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        cols.append(apply_basis(e.reshape(shape), h, legendre_degs, qs).reshape(-1, n))
    return np.stack(cols, axis=2)
