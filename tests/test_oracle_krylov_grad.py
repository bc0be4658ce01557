"""Pins of the oracle's Krylov solvers and adjoint gradient."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import assembly, gradient, hacr, krylov


def test_pcg_matches_dense_solve():
    n = 8
    S = assembly.stencil7("poisson", n, n, n, kappa=synth.kappa_subcubes(n, 3))
    A = assembly.to_sparse(S, n, n, n)
    b = synth.rhs_uniform(n ** 3, 1)
    x_ref = spla.spsolve(A.tocsc(), b)
    x, info = krylov.pcg(lambda v: A @ v, b, tol=1e-12, maxit=5000)
    assert info["status"] == "ok"
    assert np.linalg.norm(b - A @ x) <= 1e-12 * np.linalg.norm(b)
    assert np.linalg.norm(x - x_ref) <= 1e-6 * np.linalg.norm(x_ref)
    xf, infof = krylov.pcg(lambda v: A @ v, b, tol=1e-12, maxit=5000, flexible=True)
    assert infof["status"] == "ok" and np.linalg.norm(xf - x_ref) <= 1e-6 * np.linalg.norm(x_ref)


def test_pcg_detects_indefinite_breakdown():
    A = np.diag([1.0, -2.0, 3.0])
    x, info = krylov.pcg(lambda v: A @ v, np.ones(3), tol=1e-12)
    assert info["status"] == "breakdown"


def test_gmres_full_space_is_exact():
    rng = np.random.default_rng(2)
    N = 40
    A = rng.standard_normal((N, N)) + 8 * np.eye(N)
    b = rng.standard_normal(N)
    x, info = krylov.gmres(lambda v: A @ v, b, restart=N, tol=1e-13, maxit=N)
    assert info["iters"] <= N
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-9)


def test_gmres_restarted_preconditioned_convdiff():
    n = 9
    S = assembly.stencil7("convdiff", n, n, n, kappa=synth.kappa_lognormal(n, 2), beta_amp=80.0, beta_phase=0.4)
    A = assembly.to_sparse(S, n, n, n)
    b = synth.rhs_uniform(n ** 3, 3)
    x_ref = spla.spsolve(A.tocsc(), b)
    H = hacr.HACR(S, n, n, n, eps=1e-3, eta=2.0, leaf=16)
    x, info = krylov.gmres(lambda v: A @ v, b, H.apply, restart=5, tol=1e-10)
    assert info["status"] == "ok"
    assert np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b) * 1.0001
    assert np.linalg.norm(x - x_ref) <= 1e-7 * np.linalg.norm(x_ref)
    x2, info2 = krylov.gmres(lambda v: A @ v, b, None, restart=10, tol=1e-10, maxit=3)
    assert info2["status"] == "notconv" and info2["iters"] == 3


@pytest.mark.parametrize("n", [3, 5])
def test_gradient_vs_central_differences(n):
    kap = synth.kappa_lognormal(n, 11)
    f = synth.rhs_uniform(n ** 3, 12)
    u_obs = synth.rhs_uniform(n ** 3, 13) * 0.01
    g = gradient.dense_reference_gradient(kap, f, u_obs, n)
    rng = np.random.default_rng(14)
    for _ in range(5):
        d = rng.standard_normal(kap.shape)
        d /= np.sqrt(np.mean(d ** 2))
        best = np.inf
        for delta in (1e-3, 1e-4, 1e-5):
            jp, _ = gradient.objective(kap * np.exp(delta * d), f, u_obs, n)
            jm, _ = gradient.objective(kap * np.exp(-delta * d), f, u_obs, n)
            fd = (jp - jm) / (2 * delta)
            an = np.sum(g * kap * d)           # chain rule through kappa = kappa0 exp(delta d)
            best = min(best, abs(fd - an) / max(abs(an), 1e-300))
        assert best < 1e-6, best


def test_gradient_taylor_second_order():
    n = 4
    kap = synth.kappa_lognormal(n, 21)
    f = synth.rhs_uniform(n ** 3, 22)
    u_obs = np.zeros(n ** 3)
    g = gradient.dense_reference_gradient(kap, f, u_obs, n)
    d = np.random.default_rng(3).standard_normal(kap.shape) * kap
    J0, _ = gradient.objective(kap, f, u_obs, n)
    r = []
    for delta in (1e-2, 5e-3):
        J1, _ = gradient.objective(kap + delta * d, f, u_obs, n)
        r.append(abs(J1 - J0 - delta * np.sum(g * d)))
    assert 3.0 < r[0] / r[1] < 5.0
