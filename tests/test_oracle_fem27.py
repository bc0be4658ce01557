"""Pins of the oracle's 27-point trilinear finite-element Helmholtz
operator (Sec. 8, eq. HelmVarVel) and of the cyclic reduction on its
9-point plane blocks."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fem27, dense_cr, hacr


def _ones(n):
    return np.ones((n + 2,) * 3)


def test_constant_coefficient_stencil_closed_form():
    """Interior rows with constant c: the Q1 Laplacian stencil h (8/3 centre,
    0 faces, -1/6 edges, -1/12 corners) minus kappa times the Q1 mass
    stencil h^3 (64, 16, 4, 1) / 216 (exact for Q1 with the 2-point Gauss
    rule), worked out from the 1D element matrices by hand."""
    n, om = 6, 3.0
    h = 1.0 / (n + 1)
    S = fem27.stencil27(n, n, n, 2.0 * _ones(n), om)
    kap = om ** 2 / 4.0
    p = 2 + n * (2 + n * 2)                  # an interior node away from the boundary
    for m, (dx, dy, dz) in enumerate(fem27.OFFSETS27):
        nnz = abs(dx) + abs(dy) + abs(dz)
        lap = {0: 8.0 / 3.0, 1: 0.0, 2: -1.0 / 6.0, 3: -1.0 / 12.0}[nnz] * h
        mass = {0: 64.0, 1: 16.0, 2: 4.0, 3: 1.0}[nnz] * h ** 3 / 216.0
        assert np.isclose(S[m, p], lap - kap * mass, rtol=1e-13, atol=1e-15), (dx, dy, dz)


def test_row_sums_partition_of_unity():
    """Constants lie in the kernel of the stiffness part (rows away from the
    boundary sum to zero) and the mass rows sum to int kappa phi_p."""
    n = 7
    c = 1.0 + 0.3 * np.random.default_rng(1).uniform(size=(n + 2,) * 3)
    S0 = fem27.stencil27(n, n, n, c, 0.0)
    S1 = fem27.stencil27(n, n, n, c, 2.5)
    A0 = fem27.to_sparse27(S0, n, n, n)
    inner = np.zeros((n, n, n), bool)
    inner[1:-1, 1:-1, 1:-1] = True
    rs = np.asarray(A0.sum(axis=1)).ravel()[inner.ravel()]
    assert np.max(np.abs(rs)) <= 1e-13 * np.abs(S0).max()
    # mass part: row sums = h^3 kappa-weighted partition of unity; with c = 2 constant: kappa h^3
    Sc = fem27.stencil27(n, n, n, 2.0 * _ones(n), 2.5) - fem27.stencil27(n, n, n, 2.0 * _ones(n), 0.0)
    ms = Sc.sum(axis=0).reshape(n, n, n)[inner]
    h = 1.0 / (n + 1)
    np.testing.assert_allclose(ms, -(2.5 ** 2 / 4.0) * h ** 3, rtol=1e-12)
    assert S1.shape == (27, n ** 3)


def test_symmetric():
    n = 6
    c = fem27.waveguide_velocity(n)
    A = fem27.to_sparse27(fem27.stencil27(n, n, n, c, 7.0), n, n, n)
    d = abs(A - A.T).max()
    assert d <= 1e-14 * abs(A).max()


def test_manufactured_solution_second_order():
    """u* = sin(pi x) sin(pi y) sin(pi z) with the waveguide velocity at a
    moderate frequency: the nodal error of the finite-element solution
    falls by about 4 per halving of h."""
    om = 2.0 * np.pi * 1.0
    errs = []
    for n in (7, 15):
        c = fem27.waveguide_velocity(n)
        S = fem27.stencil27(n, n, n, c, om)

        def cfun(x, y, z):
            return 1.25 * (1.0 - 0.4 * np.exp(-32.0 * ((x - 0.5) ** 2 + (y - 0.5) ** 2)))

        def f(x, y, z):
            u = np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z)
            return (3.0 * np.pi ** 2 - om ** 2 / cfun(x, y, z) ** 2) * u

        b = fem27.load_vector(n, n, n, f)
        u = spla.spsolve(fem27.to_sparse27(S, n, n, n).tocsc(), b)
        t = np.arange(1, n + 1) / (n + 1)
        z, y, x = np.meshgrid(t, t, t, indexing="ij")
        us = (np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z)).ravel()
        errs.append(np.max(np.abs(u - us)))
    assert 3.3 < errs[0] / errs[1] < 4.8, errs


def test_plane_blocks_reassemble():
    nx, ny, nz = 5, 4, 6
    c = 1.0 + 0.2 * np.random.default_rng(2).uniform(size=(nz + 2, ny + 2, nx + 2))
    S = fem27.stencil27(nx, ny, nz, c, 4.0)
    A = fem27.to_sparse27(S, nx, ny, nz).toarray()
    D, Al, Cl = fem27.plane_blocks27(S, nx, ny, nz)
    B = nx * ny
    for k in range(nz):
        np.testing.assert_array_equal(D[k].toarray(), A[k * B:(k + 1) * B, k * B:(k + 1) * B])
        if k > 0:
            np.testing.assert_array_equal(Al[k].toarray(), A[k * B:(k + 1) * B, (k - 1) * B:k * B])
        if k < nz - 1:
            np.testing.assert_array_equal(Cl[k].toarray(), A[k * B:(k + 1) * B, (k + 1) * B:(k + 2) * B])


@pytest.mark.parametrize("shape", [(5, 4, 6), (6, 6, 7), (4, 5, 2)])
def test_dense_cr_solves_the_27_point_system(shape):
    nx, ny, nz = shape
    c = fem27.waveguide_velocity(max(shape))[:nz + 2, :ny + 2, :nx + 2]
    S = fem27.stencil27(nx, ny, nz, c, 9.0)
    A = fem27.to_sparse27(S, nx, ny, nz).toarray()
    cr = dense_cr.DenseCR(*fem27.plane_blocks27(S, nx, ny, nz))
    g = np.random.default_rng(3).standard_normal(nx * ny * nz)
    np.testing.assert_allclose(cr.apply(g), np.linalg.solve(A, g), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(cr.apply_T(g), np.linalg.solve(A.T, g), rtol=1e-10, atol=1e-12)


def test_hacr_small_eps_equals_dense_cr_27_point():
    nx, ny, nz = 9, 8, 7
    c = fem27.waveguide_velocity(9)[:nz + 2, :ny + 2, :nx + 2]
    S = fem27.stencil27(nx, ny, nz, c, 12.0)
    H = hacr.HACR(S, nx, ny, nz, eps=1e-13, eta=2.0, leaf=8)
    cr = dense_cr.DenseCR(*fem27.plane_blocks27(S, nx, ny, nz))
    g = np.random.default_rng(4).standard_normal(nx * ny * nz)
    z, zr = H.apply(g), cr.apply(g)
    assert np.linalg.norm(z - zr) <= 1e-10 * np.linalg.norm(zr)
    y = np.random.default_rng(5).standard_normal(nx * ny * nz)
    assert abs(H.apply_T(y) @ g - y @ z) <= 1e-12 * np.linalg.norm(y) * np.linalg.norm(z)
