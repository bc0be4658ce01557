"""Trilinear finite elements on hexahedra for the Helmholtz equation of
Sec. 8 (eq. HelmVarVel), the 27-point operator (oracle, FP64).

Test infrastructure: this module is used by the tests, the smoke check and
the benchmark's CPU baseline only, never by the GPU path.

Problem: ``-Lap u - omega^2 / c(x)^2 u = f`` on the unit cube with
Dirichlet zero on the boundary (the paper's frequency f gives
``omega = 2 pi f``).  Discretisation: continuous piecewise-trilinear (Q1)
elements on the uniform hexahedral grid with ``nx, ny, nz`` interior nodes
per axis (spacing ``h_d = 1/(n_d+1)``, ``(n_d+1)`` elements per axis); the
boundary nodes are eliminated, so the unknowns are the interior nodes in
the usual order ``p = i + nx*(j + ny*k)``.

Element matrices on an element of size ``hx x hy x hz`` with the local
nodes ``a = (ax, ay, az)`` in {0,1}^3 and basis functions
``phi_a = prod_d l_{a_d}(xi_d)`` (``l_0 = 1 - xi``, ``l_1 = xi``):

* stiffness (``-Lap``): ``K_e = kx (x) my (x) mz + mx (x) ky (x) mz +
  mx (x) my (x) kz`` with the 1D element matrices
  ``k = [[1, -1], [-1, 1]] / h`` and ``m = [[2, 1], [1, 2]] h / 6``;
* mass weighted by ``kappa = omega^2 / c^2``: ``M_e[a, b] = hx hy hz *
  sum_q w_q kappa(q) phi_a(q) phi_b(q)`` with the 2 x 2 x 2 Gauss rule
  (points ``1/2 -+ 1/(2 sqrt 3)`` per axis on the reference cube, weights
  1/8), ``c(q)`` interpolated trilinearly from the element's node values of
  ``c`` (given on the (nz+2, ny+2, nx+2) node grid, boundary included).

``A = sum_e (K_e - M_e)`` restricted to interior nodes: 27 couplings per
row, stored as ``S[m, p]`` for the offsets ``(dx, dy, dz)`` in
{-1, 0, 1}^3 with ``m = (dx+1) + 3 (dy+1) + 9 (dz+1)`` (``m = 13`` is the
centre); couplings to boundary nodes are dropped.  Its plane blocks are
9-point in-plane matrices: ``D_k`` (dz = 0), ``A_k`` (dz = -1),
``C_k`` (dz = +1).

Reading (the paper uses PetIGA and does not print its quadrature): the
2-point Gauss rule integrates the Q1 mass exactly for a constant
coefficient; the velocity enters through its trilinear interpolant.
"""
import numpy as np
import scipy.sparse as sp

OFFSETS27 = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
GAUSS = (0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0))


def offset_index(dx, dy, dz):
    return (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)


def _basis(a, xi):
    """The 1D Q1 basis function l_a at xi."""
    return xi if a == 1 else 1.0 - xi


def element_stiffness(hx, hy, hz):
    """8 x 8 Q1 stiffness matrix of -Lap, local node a = ax + 2 ay + 4 az."""
    def k(h):
        return np.array([[1.0, -1.0], [-1.0, 1.0]]) / h

    def m(h):
        return np.array([[2.0, 1.0], [1.0, 2.0]]) * h / 6.0
    K = np.zeros((8, 8))
    for a in range(8):
        ax, ay, az = a & 1, (a >> 1) & 1, a >> 2
        for b in range(8):
            bx, by, bz = b & 1, (b >> 1) & 1, b >> 2
            K[a, b] = (k(hx)[ax, bx] * m(hy)[ay, by] * m(hz)[az, bz]
                       + m(hx)[ax, bx] * k(hy)[ay, by] * m(hz)[az, bz]
                       + m(hx)[ax, bx] * m(hy)[ay, by] * k(hz)[az, bz])
    return K


def stencil27(nx, ny, nz, c, omega):
    """Return the (27, N) stencil of -Lap - omega^2 / c^2 (Q1 elements)."""
    c = np.asarray(c, dtype=np.float64)
    assert c.shape == (nz + 2, ny + 2, nx + 2)
    hx, hy, hz = 1.0 / (nx + 1), 1.0 / (ny + 1), 1.0 / (nz + 1)
    N = nx * ny * nz
    K = element_stiffness(hx, hy, hz)
    # per element (ez, ey, ex): node values of c at the 8 local nodes
    cl = [c[az:az + nz + 1, ay:ay + ny + 1, ax:ax + nx + 1] for a in range(8)
          for ax, ay, az in [(a & 1, (a >> 1) & 1, a >> 2)]]
    # element mass matrices by the 2 x 2 x 2 Gauss rule, kappa from the interpolated c
    M = np.zeros((8, 8) + cl[0].shape)
    for qz in GAUSS:
        for qy in GAUSS:
            for qx in GAUSS:
                phi = [_basis(a & 1, qx) * _basis((a >> 1) & 1, qy) * _basis(a >> 2, qz) for a in range(8)]
                cq = sum(phi[a] * cl[a] for a in range(8))
                kq = omega ** 2 / cq ** 2 * (hx * hy * hz / 8.0)
                for a in range(8):
                    for b in range(8):
                        M[a, b] += kq * (phi[a] * phi[b])
    S = np.zeros((27, nz, ny, nx))
    for a in range(8):
        ax, ay, az = a & 1, (a >> 1) & 1, a >> 2
        for b in range(8):
            bx, by, bz = b & 1, (b >> 1) & 1, b >> 2
            val = K[a, b] - M[a, b]          # (nz+1, ny+1, nx+1) elements
            # row node of element e = (ez, ey, ex): grid node (e + a); interior index e + a - 1
            # element range so that the row node is interior
            sl = tuple(slice(1 - d, 1 - d + n) for d, n in ((az, nz), (ay, ny), (ax, nx)))
            S[offset_index(bx - ax, by - ay, bz - az)] += val[sl]
    S = S.reshape(27, N)
    # drop couplings to boundary nodes
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    for m, (dx, dy, dz) in enumerate(OFFSETS27):
        ok = ((i + dx >= 0) & (i + dx < nx) & (j + dy >= 0) & (j + dy < ny) & (k + dz >= 0) & (k + dz < nz))
        S[m] = np.where(ok.reshape(-1), S[m], 0.0)
    return S


def to_sparse27(S, nx, ny, nz):
    """CSR matrix of a (27, N) stencil."""
    N = nx * ny * nz
    p = np.arange(N)
    rows, cols, vals = [], [], []
    for m, (dx, dy, dz) in enumerate(OFFSETS27):
        keep = S[m] != 0 if m != 13 else np.ones(N, bool)
        q = p + dx + nx * (dy + ny * dz)
        rows.append(p[keep]); cols.append(q[keep]); vals.append(S[m][keep])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))


def plane_blocks27(S, nx, ny, nz):
    """Block-tridiagonal view of a 27-point operator: lists ``D[k]``,
    ``A[k]`` (coupling of plane k to plane k-1, None for k = 0) and
    ``C[k]`` (to plane k+1, None for the last), each a sparse B x B matrix
    with the 9-point in-plane pattern (B = nx*ny)."""
    B = nx * ny
    D, A, C = [], [], []
    for k in range(nz):
        sl = slice(k * B, (k + 1) * B)
        blocks = []
        for dz in (0, -1, 1):
            Sk = np.zeros((27, B))
            for m, (ox, oy, oz) in enumerate(OFFSETS27):
                if oz == dz:
                    Sk[offset_index(ox, oy, 0)] = S[m, sl]
            blocks.append(to_sparse27(Sk, nx, ny, 1))
        D.append(blocks[0])
        A.append(blocks[1] if k > 0 else None)
        C.append(blocks[2] if k < nz - 1 else None)
    return D, A, C


def waveguide_velocity(nx, ny=None, nz=None):
    """The waveguide velocity of eq. HelmVarVel on the (nz+2, ny+2, nx+2)
    node grid: ``c = 1.25 (1 - 0.4 exp(-32 ((x - 1/2)^2 + (y - 1/2)^2)))``."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    z, y, x = np.meshgrid(np.arange(nz + 2) / (nz + 1), np.arange(ny + 2) / (ny + 1), np.arange(nx + 2) / (nx + 1),
                          indexing="ij")
    return 1.25 * (1.0 - 0.4 * np.exp(-32.0 * ((x - 0.5) ** 2 + (y - 0.5) ** 2)))


def load_vector(nx, ny, nz, f, order=3):
    """``b_p = int f phi_p`` over the elements around each interior node by
    the ``order``-point Gauss rule per axis (``f(x, y, z)`` vectorised)."""
    from numpy.polynomial.legendre import leggauss
    g, w = leggauss(order)
    g, w = 0.5 * (g + 1.0), 0.5 * w
    hx, hy, hz = 1.0 / (nx + 1), 1.0 / (ny + 1), 1.0 / (nz + 1)
    ez, ey, ex = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    b = np.zeros((nz, ny, nx))
    for iz, qz in enumerate(g):
        for iy, qy in enumerate(g):
            for ix, qx in enumerate(g):
                fq = f((ex + qx) * hx, (ey + qy) * hy, (ez + qz) * hz) * (w[ix] * w[iy] * w[iz] * hx * hy * hz)
                for a in range(8):
                    ax, ay, az = a & 1, (a >> 1) & 1, a >> 2
                    val = fq * _basis(ax, qx) * _basis(ay, qy) * _basis(az, qz)
                    sl = tuple(slice(1 - d, 1 - d + n) for d, n in ((az, nz), (ay, ny), (ax, nx)))
                    b += val[sl]
    return b.reshape(-1)
