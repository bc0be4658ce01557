"""Pins of the exact dense cyclic reduction and the H-ACR oracle."""
import numpy as np
import pytest
import scipy.fft as sfft

import synth
from oracle import assembly, dense_cr, hacr


def _problem(kind, nx, ny, nz, seed=1):
    kap = synth.kappa_lognormal(nx, seed, nz=nz, ny=ny)
    if kind == "convdiff":
        S = assembly.stencil7(kind, nx, ny, nz, kappa=kap, beta_amp=40.0, beta_phase=0.7)
    elif kind == "helmholtz":
        c = np.ones((nz + 2, ny + 2, nx + 2))
        S = assembly.stencil7(kind, nx, ny, nz, c=c, omega=9.37)
    elif kind == "recirc":
        S = assembly.stencil7(kind, nx, ny, nz, kappa=kap, alpha=8.0, vortex=2.0)
    else:
        S = assembly.stencil7(kind, nx, ny, nz, kappa=kap)
    return S, assembly.to_sparse(S, nx, ny, nz).toarray()


@pytest.mark.parametrize("dims", [(3, 3, 3), (7, 7, 7), (4, 3, 2), (3, 5, 4), (5, 2, 5), (2, 3, 6), (6, 4, 7)])
@pytest.mark.parametrize("kind", ["poisson", "convdiff", "helmholtz", "recirc"])
def test_dense_cr_is_exact_solve(dims, kind):
    nx, ny, nz = dims
    S, A = _problem(kind, nx, ny, nz)
    cr = dense_cr.DenseCR(*assembly.plane_blocks(S, nx, ny, nz))
    b = synth.rhs_uniform(A.shape[0], 9)
    x = np.linalg.solve(A, b)
    xt = np.linalg.solve(A.T, b)
    assert np.linalg.norm(cr.apply(b) - x) <= 1e-10 * np.linalg.norm(x)
    assert np.linalg.norm(cr.apply_T(b) - xt) <= 1e-10 * np.linalg.norm(xt)


def test_dense_cr_reduced_system_is_schur_complement():
    """After level 0 the kept planes' blocks equal the Schur complement of
    the red/black-permuted matrix onto the kept planes."""
    nx, ny, nz = 3, 2, 7
    S, A = _problem("convdiff", nx, ny, nz)
    B = nx * ny
    cr = dense_cr.DenseCR(*assembly.plane_blocks(S, nx, ny, nz))
    E = list(range(0, nz, 2))
    K = list(range(1, nz, 2))
    iE = np.concatenate([np.arange(p * B, (p + 1) * B) for p in E])
    iK = np.concatenate([np.arange(p * B, (p + 1) * B) for p in K])
    Sch = A[np.ix_(iK, iK)] - A[np.ix_(iK, iE)] @ np.linalg.solve(A[np.ix_(iE, iE)], A[np.ix_(iE, iK)])
    lev1 = cr.levels[1]
    # level-1 stored couplings are the Schur complement's off-diagonal blocks
    for m, j in enumerate(K):
        if m > 0:
            np.testing.assert_allclose(lev1["A"][j], Sch[m * B:(m + 1) * B, (m - 1) * B:m * B], atol=1e-10)
        if m + 1 < len(K):
            np.testing.assert_allclose(lev1["C"][j], Sch[m * B:(m + 1) * B, (m + 1) * B:(m + 2) * B], atol=1e-10)
    for m, j in enumerate(lev1["E"]):
        pos = K.index(j)
        np.testing.assert_allclose(lev1["Dinv"][j], np.linalg.inv(Sch[pos * B:(pos + 1) * B, pos * B:(pos + 1) * B]),
                                   rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("n,nz", [(5, 15), (15, 31), (31, 63)])
def test_dense_cr_constant_kappa_mode_recurrence(n, nz):
    """Constant kappa, nz = 2^K - 1: every block is diagonal in the 2D
    DST basis; per mode d_{r+1} = d_r - 2 c_r^2/d_r, c_{r+1} = -c_r^2/d_r."""
    nx = ny = n
    S = assembly.stencil7("poisson", nx, ny, nz)
    cr = dense_cr.DenseCR(*assembly.plane_blocks(S, nx, ny, nz))
    hx = 1.0 / (nx + 1)
    hz = 1.0 / (nz + 1)
    a = np.arange(1, nx + 1)
    l1 = (2 - 2 * np.cos(np.pi * a / (nx + 1))) / hx ** 2
    d = (l1[:, None] + l1[None, :]).reshape(-1) + 2.0 / hz ** 2
    c = -np.ones_like(d) / hz ** 2
    Q = sfft.dst(np.eye(nx), type=1, norm="ortho")
    Q2 = np.kron(Q, Q)      # orthonormal 2D DST-I (x fastest)
    for lev in cr.levels:
        for i in lev["E"]:
            T = Q2.T @ lev["Dinv"][i] @ Q2
            np.testing.assert_allclose(np.diag(T), 1.0 / d, rtol=1e-10)
            assert np.abs(T - np.diag(np.diag(T))).max() < 1e-10 * np.abs(np.diag(T)).max()
        c, d = -c ** 2 / d, d - 2 * c ** 2 / d
    t, Dinv = cr.top
    np.testing.assert_allclose(np.diag(Q2.T @ Dinv @ Q2), 1.0 / d, rtol=1e-10)


# (31, 31, 7): the plane geometry of the 31^3 workload (961-point planes,
# several cluster levels, leaf 16) over three reduction levels
@pytest.mark.parametrize("dims,kind", [((15, 15, 15), "poisson"), ((13, 9, 6), "poisson"), ((13, 9, 6), "recirc"),
                                       ((31, 31, 7), "poisson")])
def test_hacr_eps_to_zero_matches_exact_cr(dims, kind):
    nx, ny, nz = dims
    S, A = _problem(kind, nx, ny, nz, seed=3)
    cr = dense_cr.DenseCR(*assembly.plane_blocks(S, nx, ny, nz))
    H = hacr.HACR(S, nx, ny, nz, eps=1e-13, eta=2.0, leaf=16)
    b = synth.rhs_uniform(A.shape[0], 5)
    z0 = cr.apply(b)
    assert np.linalg.norm(H.apply(b) - z0) <= 1e-10 * np.linalg.norm(z0)
    zt = cr.apply_T(b)
    assert np.linalg.norm(H.apply_T(b) - zt) <= 1e-10 * np.linalg.norm(zt)


def test_hacr_error_decreases_with_eps_and_transpose_is_exact():
    nx = ny = nz = 15
    S, A = _problem("convdiff", nx, ny, nz, seed=4)
    b = synth.rhs_uniform(A.shape[0], 6)
    y = synth.rhs_uniform(A.shape[0], 7)
    x = np.linalg.solve(A, b)
    errs = []
    for eps in (1e-2, 1e-4, 1e-6, 1e-8):
        H = hacr.HACR(S, nx, ny, nz, eps=eps, eta=2.0, leaf=32)
        errs.append(np.linalg.norm(H.apply(b) - x) / np.linalg.norm(x))
        # <M^-T y, b> = <y, M^-1 b> holds to round-off at any eps
        lhs, rhs = H.apply_T(y) @ b, y @ H.apply(b)
        assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(H.apply_T(y)) * np.linalg.norm(b)
        assert errs[-1] < 10 * eps
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1)), errs
    slope = np.polyfit(np.log10([1e-2, 1e-4, 1e-6, 1e-8]), np.log10(errs), 1)[0]
    assert 0.7 < slope < 1.3, slope


def test_hacr_one_iteration_at_tiny_eps():
    from oracle import krylov
    nx = ny = nz = 15
    S, A = _problem("poisson", nx, ny, nz, seed=8)
    H = hacr.HACR(S, nx, ny, nz, eps=1e-13, eta=2.0, leaf=32)
    b = synth.rhs_uniform(A.shape[0], 1)
    x, info = krylov.pcg(lambda v: A @ v, b, H.apply, tol=1e-8)
    assert info["iters"] == 1 and info["status"] == "ok"

def test_hacr_constant_kappa_against_dst_solve():
    """The H-matrix reduction at the headline eps on the 961-point planes of
    the 31^3 workload (31 x 31 x 7, constant kappa), against the exact solve
    by the 3D DST-I, whose eigenvalues are the sums of the 1D second-
    difference ones: the preconditioner is within 10 eps of A^-1 b."""
    nx = ny = 31
    nz = 7
    eps = 1e-4
    S = assembly.stencil7("poisson", nx, ny, nz)
    b = synth.rhs_uniform(nx * ny * nz, 9)
    hx, hz = 1.0 / (nx + 1), 1.0 / (nz + 1)
    lx = (2 - 2 * np.cos(np.pi * np.arange(1, nx + 1) / (nx + 1))) / hx ** 2
    lz = (2 - 2 * np.cos(np.pi * np.arange(1, nz + 1) / (nz + 1))) / hz ** 2
    lam = lz[:, None, None] + lx[None, :, None] + lx[None, None, :]
    x = sfft.idstn(sfft.dstn(b.reshape(nz, ny, nx), type=1, norm="ortho") / lam, type=1, norm="ortho").reshape(-1)
    A = assembly.to_sparse(S, nx, ny, nz)
    assert np.linalg.norm(A @ x - b) <= 1e-13 * np.linalg.norm(b)  # the closed form itself
    H = hacr.HACR(S, nx, ny, nz, eps=eps, eta=2.0, leaf=16)
    assert np.linalg.norm(H.apply(b) - x) <= 10 * eps * np.linalg.norm(x)
