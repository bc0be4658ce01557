"""Pins of the oracle's H-matrix layer (Sec. 3.1, Sec. 4.2-4.3)."""
import numpy as np
import pytest

import synth
from oracle import assembly, hmatrix as hm


@pytest.mark.parametrize("nx,ny,leaf", [(31, 31, 32), (47, 47, 32), (13, 9, 16), (127, 127, 32), (5, 40, 8)])
def test_cluster_tree_bisection_rule(nx, ny, leaf):
    ct = hm.ClusterTree(nx, ny, leaf)
    assert sorted(ct.perm.tolist()) == list(range(nx * ny))
    for c in range(len(ct.box)):
        x0, x1, y0, y1 = ct.box[c]
        assert ct.size(c) == (x1 - x0) * (y1 - y0)
        if ct.is_leaf(c):
            assert ct.size(c) <= leaf
            pts = ct.perm[ct.lo[c]:ct.hi[c]]
            assert set(pts.tolist()) == {x + nx * y for y in range(y0, y1) for x in range(x0, x1)}
        else:
            assert ct.size(c) > leaf
            a, b = ct.children[c]
            sx, sy = x1 - x0, y1 - y0
            if sx >= sy:      # longer side split, ties split x, floor half first
                assert ct.box[a] == (x0, x0 + sx // 2, y0, y1) and ct.box[b] == (x0 + sx // 2, x1, y0, y1)
            else:
                assert ct.box[a] == (x0, x1, y0, y0 + sy // 2) and ct.box[b] == (x0, x1, y0 + sy // 2, y1)
            assert ct.lo[a] == ct.lo[c] and ct.hi[a] == ct.lo[b] and ct.hi[b] == ct.hi[c]


@pytest.mark.parametrize("eta", [0.5, 1.0, 2.0, 8.0])
def test_block_tree_partitions_and_admissibility(eta):
    ct = hm.ClusterTree(23, 17, 16)
    bt = hm.BlockTree(ct, eta)
    N = 23 * 17
    cover = np.zeros((N, N), dtype=np.int32)
    for (t, s), k in bt.kind.items():
        if k == "H":
            continue
        cover[ct.lo[t]:ct.hi[t], ct.lo[s]:ct.hi[s]] += 1
        # brute-force geometric check of the admissibility condition
        bx = lambda c: ct.box[c]
        tx0, tx1, ty0, ty1 = bx(t)
        sx0, sx1, sy0, sy1 = bx(s)
        P = np.array([(x, y) for x in range(tx0, tx1) for y in range(ty0, ty1)], float)
        Q = np.array([(x, y) for x in range(sx0, sx1) for y in range(sy0, sy1)], float)
        dmin = np.sqrt(((P[:, None, :] - Q[None, :, :]) ** 2).sum(-1)).min()
        dt = np.hypot(tx1 - 1 - tx0, ty1 - 1 - ty0)
        ds = np.hypot(sx1 - 1 - sx0, sy1 - 1 - sy0)
        adm = dmin > 0 and min(dt, ds) <= eta * dmin + 1e-12
        assert (k == "L") == adm
        if k == "D":
            assert ct.is_leaf(t) or ct.is_leaf(s)
    assert cover.min() == 1 and cover.max() == 1


def test_truncation_matches_svd():
    rng = np.random.default_rng(0)
    m, n, K = 60, 45, 20
    sig = 10.0 ** -np.arange(K)
    Qa, _ = np.linalg.qr(rng.standard_normal((m, K)))
    Qb, _ = np.linalg.qr(rng.standard_normal((n, K)))
    U, V = Qa * sig, Qb
    for eps in (3e-2, 3e-4, 3e-8):
        Ut, Vt = hm.truncate(U, V, eps)
        k = int(np.count_nonzero(sig > eps * sig[0]))
        assert Ut.shape[1] == k
        err = np.linalg.norm(U @ V.T - Ut @ Vt.T, 2)
        assert np.isclose(err, sig[k], rtol=1e-6)
    # rank-deficient and zero inputs
    Ut, Vt = hm.truncate(np.zeros((5, 3)), np.zeros((4, 3)), 1e-3)
    assert Ut.shape == (5, 0) and Vt.shape == (4, 0)
    Ut, Vt = hm.truncate(np.hstack([U[:, :2], U[:, :2]]), np.hstack([V[:, :2], V[:, :2]]), 1e-12)
    assert Ut.shape[1] == 2


def _plane_H(nx, ny, leaf, eta, seed=1):
    kap = synth.kappa_lognormal(nx, seed, nz=1, ny=ny)
    S = assembly.stencil7("poisson", nx, ny, 1, kappa=kap)
    D = assembly.plane_blocks(S, nx, ny, 1)[0][0]
    ct = hm.ClusterTree(nx, ny, leaf)
    bt = hm.BlockTree(ct, eta)
    Dp = D.toarray()[np.ix_(ct.perm, ct.perm)]
    return ct, bt, Dp


@pytest.mark.parametrize("eta", [1.0, 2.0, 6.0])
def test_level0_conversion_exact_and_matvec(eta):
    ct, bt, Dp = _plane_H(19, 14, 16, eta)
    H = hm.HM.from_dense(bt, Dp, 1e-15)
    np.testing.assert_allclose(H.to_dense(), Dp, atol=1e-9 * np.abs(Dp).max())
    x = np.random.default_rng(1).standard_normal((Dp.shape[0], 3))
    np.testing.assert_allclose(H.matvec(x), Dp @ x, rtol=1e-12, atol=1e-9 * np.abs(Dp).max())
    np.testing.assert_allclose(H.matvec(x, True), Dp.T @ x, rtol=1e-12, atol=1e-9 * np.abs(Dp).max())


def test_hinverse_accuracy_and_eps_limit():
    ct, bt, Dp = _plane_H(24, 20, 16, 2.0)
    N = Dp.shape[0]
    Xd = np.linalg.inv(Dp)
    prev = np.inf
    for eps in (1e-2, 1e-4, 1e-6, 1e-12):
        X = hm.inverse(hm.HM.from_dense(bt, Dp, 1e-15), eps).to_dense()
        res = np.linalg.norm(np.eye(N) - Dp @ X) / np.sqrt(N)
        assert res < 50 * eps and res < prev
        prev = res
    np.testing.assert_allclose(X, Xd, rtol=0, atol=1e-9 * np.abs(Xd).max())


def test_formatted_product_close_to_exact():
    """``C <- T_eps(C + alpha A B)`` deviates from the exact dense result
    by O(eps) relative to the operands."""
    ct, bt, Dp = _plane_H(22, 18, 16, 2.0)
    eps = 1e-6
    A = hm.inverse(hm.HM.from_dense(bt, Dp, 1e-15), eps)
    B = hm.HM.from_dense(bt, Dp @ Dp.T / np.abs(Dp).max(), eps)
    C = hm.HM.from_dense(bt, np.eye(Dp.shape[0]), eps)
    Ad, Bd, Cd = A.to_dense(), B.to_dense(), C.to_dense()
    hm.mul(-0.5, A, B, C, eps)
    ref = Cd - 0.5 * Ad @ Bd
    err = np.linalg.norm(C.to_dense() - ref) / np.linalg.norm(ref)
    assert err < 20 * eps, err
    # add with zero is a copy; H-add of exact sum
    Z = hm.HM.zeros(bt)
    hm.add(Z, 2.0, A, eps)
    np.testing.assert_allclose(Z.to_dense(), 2 * Ad, atol=20 * eps * np.abs(Ad).max())
