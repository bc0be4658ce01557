"""7-point finite-difference operators on the unit cube (oracle).

Follows the problem statements of the paper: the variable-coefficient
Poisson equation discretised with the second-order 7-point star and the
harmonic average of kappa between neighbouring nodes (Sec. 6, eq.
poissonEquation); the convection-diffusion equation with first-order
upwind differences for the convective term (Sec. 7, eq. codi); the
Helmholtz operator -Lap u - (omega/c)^2 u (Sec. 8, eq. HelmVarVel) on the
7-point star instead of the 27-point FEM stencil.

Grid: ``nx, ny, nz`` interior nodes, spacing ``h_d = 1/(n_d+1)``, Dirichlet
zero on the boundary.  Unknown ``p = i + nx*(j + ny*k)`` (x fastest); a
plane is the set of unknowns with the same ``k``.

Stencil layout (shared convention of the C-ABI): 7 arrays of length N,
``S[0]`` centre, ``S[1]`` x-1, ``S[2]`` x+1, ``S[3]`` y-1, ``S[4]`` y+1,
``S[5]`` z-1, ``S[6]`` z+1, so ``(Au)_p = sum_m S[m,p] u_{nb_m(p)}``;
couplings to boundary nodes are zero.
"""
import numpy as np
import scipy.sparse as sp

# neighbour offsets (dx, dy, dz) in the order of the stencil layout
OFFSETS = [(0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]


def harmonic(a, b):
    """Harmonic mean ``2ab/(a+b)`` of the two node values of a face."""
    return 2.0 * a * b / (a + b)


def _interior_mask(nx, ny, nz, d):
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    dx, dy, dz = OFFSETS[d]
    ok = (i + dx >= 0) & (i + dx < nx) & (j + dy >= 0) & (j + dy < ny) & (k + dz >= 0) & (k + dz < nz)
    return ok.reshape(-1)


def recirculating_flow(x, y, z, a):
    """The recirculating flow b(x) of Sec. 7 (eq. codi) with wavenumber a:
    every trigonometric argument is a 2 pi times x, 1/8 + y, 1/8 + z or z
    as the equation prints them.  Returns (b_x, b_y, b_z); the field is
    divergence-free (the paper's "b_x + b_y + b_z = 0" is read as
    div b = 0, which the formula satisfies)."""
    t = 2.0 * np.pi * a
    X, Y8, Z8, Z = t * x, t * (0.125 + y), t * (0.125 + z), t * z
    bx = np.sin(X) * np.sin(Y8) + np.sin(Z8) * np.sin(X)
    by = np.cos(X) * np.cos(Y8) + np.cos(Y8) * np.cos(Z)
    bz = np.cos(X) * np.cos(Z8) + np.sin(Y8) * np.sin(Z)
    return bx, by, bz


def stencil7(kind, nx, ny, nz, kappa=None, beta_amp=0.0, beta_phase=0.0, c=None, omega=0.0, alpha=0.0,
             vortex=1.0):
    """Return the (7, N) stencil of the requested operator.

    kind: ``"poisson"`` (-div(kappa grad u)), ``"convdiff"``
    (-div(kappa grad u) + beta . grad u with beta_d(x) =
    beta_amp (1 + 0.5 sin(2 pi x + beta_phase)) in all three directions,
    upwinded at the node), ``"recirc"`` (-div(kappa grad u) +
    alpha b(x) . grad u with the recirculating flow of wavenumber
    ``vortex``, each component upwinded at the node), ``"helmholtz"``
    (-Lap u - omega^2/c^2 u).  ``kappa`` and ``c`` live on the
    (nz+2, ny+2, nx+2) node grid.
    """
    N = nx * ny * nz
    h = (1.0 / (nx + 1), 1.0 / (ny + 1), 1.0 / (nz + 1))
    if kappa is None:
        kappa = np.ones((nz + 2, ny + 2, nx + 2))
    kap = np.asarray(kappa, dtype=np.float64)
    assert kap.shape == (nz + 2, ny + 2, nx + 2)
    kc = kap[1:-1, 1:-1, 1:-1]
    S = np.zeros((7, N))
    for d in range(1, 7):
        dx, dy, dz = OFFSETS[d]
        kn = kap[1 + dz: nz + 1 + dz, 1 + dy: ny + 1 + dy, 1 + dx: nx + 1 + dx]
        axis = 0 if dx else (1 if dy else 2)
        w = (harmonic(kc, kn) / h[axis] ** 2).reshape(-1)
        S[0] += w
        S[d] = np.where(_interior_mask(nx, ny, nz, d), -w, 0.0)
    if kind == "poisson":
        pass
    elif kind == "convdiff":
        x = (np.arange(1, nx + 1) * h[0])
        b = beta_amp * (1.0 + 0.5 * np.sin(2.0 * np.pi * x + beta_phase))
        b = np.broadcast_to(b[None, None, :], (nz, ny, nx)).reshape(-1)
        bp, bm = np.maximum(b, 0.0), np.minimum(b, 0.0)
        for axis, (dm, dp) in enumerate([(1, 2), (3, 4), (5, 6)]):
            # beta+ (u_p - u_{p-e})/h + beta- (u_{p+e} - u_p)/h
            S[0] += (bp - bm) / h[axis]
            S[dm] += np.where(_interior_mask(nx, ny, nz, dm), -bp / h[axis], 0.0)
            S[dp] += np.where(_interior_mask(nx, ny, nz, dp), bm / h[axis], 0.0)
    elif kind == "recirc":
        zz, yy, xx = np.meshgrid(np.arange(1, nz + 1) * h[2], np.arange(1, ny + 1) * h[1],
                                 np.arange(1, nx + 1) * h[0], indexing="ij")
        comps = recirculating_flow(xx, yy, zz, vortex)
        for axis, (dm, dp) in enumerate([(1, 2), (3, 4), (5, 6)]):
            b = alpha * comps[axis].reshape(-1)
            bp, bm = np.maximum(b, 0.0), np.minimum(b, 0.0)
            S[0] += (bp - bm) / h[axis]
            S[dm] += np.where(_interior_mask(nx, ny, nz, dm), -bp / h[axis], 0.0)
            S[dp] += np.where(_interior_mask(nx, ny, nz, dp), bm / h[axis], 0.0)
    elif kind == "helmholtz":
        cc = np.asarray(c, dtype=np.float64)[1:-1, 1:-1, 1:-1].reshape(-1)
        S[0] -= omega ** 2 / cc ** 2
    else:
        raise ValueError(kind)
    return S


def to_sparse(S, nx, ny, nz):
    """CSR matrix of a (7, N) stencil."""
    N = nx * ny * nz
    rows, cols, vals = [], [], []
    p = np.arange(N)
    for d in range(7):
        dx, dy, dz = OFFSETS[d]
        m = (S[d] != 0) if d else np.ones(N, bool)
        q = p + dx + nx * (dy + ny * dz)
        rows.append(p[m]); cols.append(q[m]); vals.append(S[d][m])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))


def apply_stencil(S, u, nx, ny, nz, transpose=False):
    """``A u`` (or ``A^T u``) directly from the stencil arrays."""
    return (to_sparse(S, nx, ny, nz).T if transpose else to_sparse(S, nx, ny, nz)) @ u


def plane_blocks(S, nx, ny, nz):
    """Block-tridiagonal view: lists ``D[k]`` (sparse B x B, B = nx*ny),
    ``A[k]`` (vector, coupling of plane k to k-1, None for k=0) and
    ``C[k]`` (vector, coupling of plane k to k+1, None for the last)."""
    B = nx * ny
    D, A, C = [], [], []
    for k in range(nz):
        sl = slice(k * B, (k + 1) * B)
        Sk = S[:, sl].copy()
        Sk[5:] = 0.0
        D.append(to_sparse(Sk, nx, ny, 1))
        A.append(S[5, sl].copy() if k > 0 else None)
        C.append(S[6, sl].copy() if k < nz - 1 else None)
    return D, A, C
