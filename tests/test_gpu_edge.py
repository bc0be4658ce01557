"""Degenerate shapes through the C ABI: a single plane (no cyclic-reduction
level, only the top inverse), two planes, 1 x 1 planes (scalar blocks), a
one-dimensional plane longer than a leaf, and planes of one leaf.  The
preconditioner against the oracle's H-matrix cyclic reduction and the
Krylov solution against a sparse direct solve."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import assembly, hacr

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1712_08872_amd as acr  # noqa: E402

SHAPES = [(8, 8, 1), (8, 8, 2), (1, 1, 9), (33, 1, 5), (1, 40, 3), (6, 5, 3)]


def _case(shape, kind, seed):
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    kappa = np.exp(rng.standard_normal((nz + 2, ny + 2, nx + 2)))
    kw = dict(kappa=kappa)
    if kind == "convdiff":
        kw.update(beta_amp=30.0, beta_phase=0.7)
    S = assembly.stencil7(kind, nx, ny, nz, **kw)
    f = rng.uniform(-1, 1, nx * ny * nz)
    return kappa, S, f


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("kind", ["poisson", "convdiff"])
def test_degenerate_shapes(shape, kind):
    nx, ny, nz = shape
    eps = 1e-7  # the smallest eps the library accepts
    kappa, S, f = _case(shape, kind, 11)
    H = hacr.HACR(S, nx, ny, nz, eps=eps, eta=2.0, leaf=16)
    A = assembly.to_sparse(S, nx, ny, nz).tocsc()
    h = acr.acr_setup(nx, ny, nz, acr.POISSON_HARMONIC if kind == "poisson" else acr.CONVDIFF_UPWIND,
                      kappa=torch.from_numpy(kappa.reshape(-1)).cuda(),
                      beta_amp=30.0 if kind == "convdiff" else 0.0, beta_phase=0.7 if kind == "convdiff" else 0.0,
                      eps=eps, leaf_size=16)
    fd = torch.from_numpy(f).cuda()
    z = acr.acr_apply(h, fd).cpu().numpy()
    zt = acr.acr_apply_T(h, fd).cpu().numpy()
    for mine, ref in ((z, H.apply(f)), (zt, H.apply_T(f))):
        assert np.linalg.norm(mine - ref) <= 10 * eps * np.linalg.norm(ref)
    method = acr.CG if kind == "poisson" else acr.GMRES
    x, info = acr.krylov_solve(h, fd, method=method, restart=20, rtol=1e-12, maxit=100)
    assert info["status"] == 0
    xs = spla.spsolve(A, f)
    assert np.linalg.norm(x.cpu().numpy() - xs) <= 1e-9 * np.linalg.norm(xs)
    h.close()


def test_degenerate_shape_mixed_precision():
    nx, ny, nz = 6, 5, 3
    kappa, S, f = _case((nx, ny, nz), "poisson", 12)
    A = assembly.to_sparse(S, nx, ny, nz).tocsc()
    h = acr.acr_setup(nx, ny, nz, acr.POISSON_HARMONIC, kappa=torch.from_numpy(kappa.reshape(-1)).cuda(),
                      eps=1e-6, leaf_size=16, precision=acr.MIXED_FP32)
    x, info = acr.krylov_solve(h, torch.from_numpy(f).cuda(), rtol=1e-12, maxit=100)
    assert info["status"] == 0
    xs = spla.spsolve(A, f)
    assert np.linalg.norm(x.cpu().numpy() - xs) <= 1e-9 * np.linalg.norm(xs)
    h.close()
