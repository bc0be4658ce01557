"""Adjoint gradient of ``J(kappa) = 0.5 ||u(kappa) - u_obs||^2`` (oracle).

``A(kappa) u = f`` is the harmonic-average Poisson operator of
``assembly``.  With the adjoint ``A^T lam = u - u_obs`` the gradient is
``dJ/dkappa_m = -lam^T (dA/dkappa_m) u``.  Each interior face ``(p, q)``
contributes ``w_f (u_p - u_q)`` to row p and ``w_f (u_q - u_p)`` to row
q (boundary values are zero), with ``w_f = kappa_f / h^2`` and
``kappa_f = 2 kappa_p kappa_q / (kappa_p + kappa_q)``, so

    dJ/dkappa_m = -sum_{faces f containing node m} (1/h^2)
                  (d kappa_f / d kappa_m) (u_p - u_q)(lam_p - lam_q),

with ``d kappa_f / d kappa_m = 2 kappa_o^2 / (kappa_m + kappa_o)^2`` for
the other node ``o`` of the face.  The gradient lives on the whole
``(nz+2, ny+2, nx+2)`` node grid (boundary nodes enter through the faces
of their interior neighbours).
"""
import numpy as np

from .assembly import stencil7, to_sparse


def grad_kappa(kappa, u, lam, nx, ny, nz):
    """``-lam^T (dA/dkappa) u`` on the node grid.

    Row p of ``A u`` is ``sum_q w_pq (u_p - u_q)`` over the six neighbours
    (``u_q = 0`` on the boundary); differentiating each ``w_pq`` with
    respect to its two node values gives the sum below, term by term.
    """
    kap = np.asarray(kappa, dtype=np.float64)
    hs = (1.0 / (nx + 1), 1.0 / (ny + 1), 1.0 / (nz + 1))
    U = np.zeros((nz + 2, ny + 2, nx + 2))
    U[1:-1, 1:-1, 1:-1] = np.asarray(u, dtype=np.float64).reshape(nz, ny, nx)
    lam3 = np.asarray(lam, dtype=np.float64).reshape(nz, ny, nx)
    g = np.zeros_like(kap)
    kp = kap[1:-1, 1:-1, 1:-1]
    up = U[1:-1, 1:-1, 1:-1]
    for (dx, dy, dz) in [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]:
        h = hs[0] if dx else (hs[1] if dy else hs[2])
        sl = (slice(1 + dz, nz + 1 + dz), slice(1 + dy, ny + 1 + dy), slice(1 + dx, nx + 1 + dx))
        kq = kap[sl]
        uq = U[sl]
        c = lam3 * (up - uq) / h ** 2
        dkp = 2.0 * kq ** 2 / (kp + kq) ** 2      # d kappa_f / d kappa_p
        dkq = 2.0 * kp ** 2 / (kp + kq) ** 2      # d kappa_f / d kappa_q
        g[1:-1, 1:-1, 1:-1] -= c * dkp
        g[sl] -= c * dkq
    return g


def objective(kappa, f, u_obs, n):
    """``J`` with a sparse direct solve (tiny grids only)."""
    import scipy.sparse.linalg as spla
    S = stencil7("poisson", n, n, n, kappa=kappa)
    u = spla.spsolve(to_sparse(S, n, n, n).tocsc(), f)
    return 0.5 * np.sum((u - u_obs) ** 2), u


def dense_reference_gradient(kappa, f, u_obs, n):
    """Dense FP64 reference: direct solves for ``u`` and ``lam``, then the
    face formula above."""
    S = stencil7("poisson", n, n, n, kappa=kappa)
    A = to_sparse(S, n, n, n).toarray()
    u = np.linalg.solve(A, f)
    lam = np.linalg.solve(A.T, u - u_obs)
    return grad_kappa(kappa, u, lam, n, n, n)
