"""Dense direct solve of the discrete problem (tiny grids; test infrastructure only).

The matrix is assembled from its definition, A = S L_G S - diag(q + kappa2),
S = diag(sqrt(eps)), with L_G = -4 pi G^-1 for free and surface boundaries
(G the dense vacuum solver written out pairwise) and L_G the spectral
Laplacian for periodic boundaries.  A phi = -4 pi rho is solved by LU; for a
singular periodic operator (kappa2 = 0) the system is bordered with the
constraint sum sqrt(eps) phi = 0 that PCG implicitly selects.
"""
import numpy as np

from . import BC_PERIODIC
from .green import dense_green, dense_laplacian_periodic
from .stencil import q_field

FOUR_PI = 4.0 * np.pi


def dense_operator(eps, h, bc, fd_order=16, kappa2=None, surface_k0_offset=None):
    eps = np.asarray(eps, dtype=np.float64)
    shape = eps.shape
    s = np.sqrt(eps).ravel()
    qk = q_field(eps, h, bc, fd_order).ravel()
    if kappa2 is not None:
        qk = qk + np.broadcast_to(kappa2, shape).ravel()
    if bc == BC_PERIODIC:
        lap = dense_laplacian_periodic(shape, h)
    else:
        g = dense_green(shape, h, bc, surface_k0_offset)
        lap = -FOUR_PI * np.linalg.inv(g)
    return s[:, None] * lap * s[None, :] - np.diag(qk)


def dense_solve(rho, eps, h, bc, fd_order=16, kappa2=None, surface_k0_offset=None):
    rho = np.asarray(rho, dtype=np.float64)
    a = dense_operator(eps, h, bc, fd_order, kappa2, surface_k0_offset)
    b = -FOUR_PI * rho.ravel()
    n = b.size
    if bc == BC_PERIODIC and kappa2 is None:
        s = np.sqrt(np.asarray(eps, dtype=np.float64)).ravel()
        big = np.zeros((n + 1, n + 1))
        big[:n, :n] = a
        big[:n, n] = s
        big[n, :n] = s
        rhs = np.concatenate([b, [0.0]])
        sol = np.linalg.solve(big, rhs)
        return sol[:n].reshape(rho.shape)
    return np.linalg.solve(a, b).reshape(rho.shape)
