"""Pins of the oracle's counters (the stored-factor statistics, the
algorithmic bytes of one application and the setup flops by class) on
cases small enough to count by hand.

Cyclic-reduction structure used below (Sec. 4.1, planes eliminated at the
1-based odd positions): with nz = 3, level 0 eliminates planes 0 and 2 and
keeps plane 1, which is the top; with nz = 7, level 0 eliminates 0, 2, 4, 6,
level 1 (planes 1, 3, 5) eliminates 1 and 5, and plane 3 is the top.  A
2 x 2 plane with leaf size 4 is one cluster, so every H-matrix is a single
dense 4 x 4 leaf (16 entries) and a diagonal coupling has 4 entries."""
import numpy as np
import pytest

from oracle import assembly, hacr
from oracle import hmatrix as hm


def _hacr(nz, eps=1e-8):
    kap = np.exp(np.random.default_rng(3).standard_normal((nz + 2, 4, 4)))
    S = assembly.stencil7("poisson", 2, 2, nz, kappa=kap)
    return hacr.HACR(S, 2, 2, nz, eps=eps, eta=2.0, leaf=4)


def test_apply_bytes_hand_count_nz3():
    # one plane vector = 4 doubles = 32 B; a dense factor 16 entries; a diagonal coupling 32 B
    # forward: w_0 = Dinv_0 g_0 and w_2 = Dinv_2 g_2 (read g, write w, the factor);
    #          g_1 -= A_1 w_0 + C_1 w_2 (read and write g_1, two w, two diagonals)
    # top:     z_1 = Dinv_1 g_1
    # back:    rr = g_0 - C_0 z_1, z_0 = Dinv_0 rr; rr = g_2 - A_2 z_1, z_2 = Dinv_2 rr
    H = _hacr(3)
    v, d8 = 32, 16 * 8
    fwd = 2 * (2 * v + d8) + (2 * v + 2 * (v + 32))
    top = 2 * v + d8
    back = 2 * ((2 * v + v + 32) + (2 * v + d8))
    assert fwd + top + back == 1408
    assert H.apply_bytes(8) == 1408
    # FP32 factors: the dense factors at 4 bytes per entry, diagonals and vectors stay FP64
    assert H.apply_bytes(4) == 1408 - 5 * 16 * 4


def test_factor_list_and_stats_nz3_nz7():
    H3 = _hacr(3)
    # level 0: Dinv_0, Dinv_2, A_1, A_2 (A_0 absent), C_0, C_1 (C_2 absent); top Dinv_1
    assert len(H3.factor_list()) == 7
    H7 = _hacr(7)
    # level 0: 4 inverses + A_1..A_6 + C_0..C_5 = 16; level 1: Dinv_1, Dinv_5 and the
    # couplings A_3, A_5, C_1, C_3 (A_1 = -X A_0 and C_5 = -Y C_6 are absent) = 6; top 1
    fl = H7.factor_list()
    assert len(fl) == 23
    assert sum(1 for r, role, p, o in fl if r == 1 and role != "Dinv") == 4
    st = H7.stats()
    # 7 inverses + 4 level-1 couplings dense 4 x 4, 12 level-0 diagonals of 4
    assert st["entries"] == 11 * 16 + 12 * 4
    assert all(v == 0 for v in st["max_rank"].values())


def test_hm_stats_of_a_rank2_matrix():
    """Every admissible block of a rank-2 matrix has rank 2: the stored
    entries are the dense leaves' m n plus 2 (m + n) per low-rank leaf."""
    ct = hm.ClusterTree(8, 8, 8)
    bt = hm.BlockTree(ct, 2.0)
    rng = np.random.default_rng(5)
    F, G = rng.standard_normal((64, 2)), rng.standard_normal((64, 2))
    H = hm.HM.from_dense(bt, F @ G.T, 1e-12)
    e, mx, sm, nl = H.stats()
    dense = [(t, s) for (t, s), k in bt.kind.items() if k == "D"]
    low = [(t, s) for (t, s), k in bt.kind.items() if k == "L"]
    assert len(low) > 0 and nl == len(low) and mx == 2 and sm == 2 * len(low)
    assert e == sum(ct.size(t) * ct.size(s) for t, s in dense) + sum(2 * (ct.size(t) + ct.size(s)) for t, s in low)


def test_truncation_flops_hand_count():
    rng = np.random.default_rng(1)
    U = rng.standard_normal((10, 2)) @ rng.standard_normal((2, 3))   # 10 x 3 of rank 2
    V = rng.standard_normal((8, 3))
    hm.reset_flops()
    Uk, Vk = hm.truncate(U, V, 1e-10)
    assert Uk.shape[1] == 2
    f = hm.flops_snapshot()
    # QR of 10 x 3 and 8 x 3 with Q: 4 (10 + 8) 9 - 8 27 / 3; core 3 x 3 product and SVD;
    # rebuild of 10 x 2 and 8 x 2 from 3 columns
    assert f == {"qr": 576.0, "gemm": 54, "svd": 594, "rebuild": 216, "leaf_inverse": 0}
    hm.reset_flops()
    hm.truncate(rng.standard_normal((4, 5)), rng.standard_normal((3, 5)), 1e-10)
    # K = 5 >= min(4, 3): dense 4 x 3 sum of 5 outer products, then its thin SVD 14 4 9 + 8 27
    assert hm.flops_snapshot() == {"qr": 0, "gemm": 120, "svd": 720, "rebuild": 0, "leaf_inverse": 0}


def test_matvec_flops_hand_count():
    ct = hm.ClusterTree(4, 2, 4)   # 8 points: two clusters of 4 (x split)
    bt = hm.BlockTree(ct, 10.0)     # the off-diagonal blocks are admissible (dist 1, diam sqrt 2)
    H = hm.HM.from_dense(bt, np.arange(64.0).reshape(8, 8) % 7, 1e-14)
    e, mx, sm, nl = H.stats()
    hm.reset_flops()
    H.matvec(np.ones((8, 3)))
    # 2 dense 4 x 4 leaves and 2 low-rank leaves of (4 + 4) k entries, 3 columns: 2 x entries x 3
    assert hm.flops_snapshot()["gemm"] == 2 * e * 3


def test_setup_flops_by_class_nz3_nz7():
    # nz = 3: three 4 x 4 leaf inverses (2 m^3 = 128 each); level 0 only scales by diagonals
    H3 = _hacr(3)
    assert H3.setup_flops == {"gemm": 0, "qr": 0, "svd": 0, "rebuild": 0, "leaf_inverse": 3 * 128}
    # nz = 7: 4 + 2 + 1 inverses; level 1 forms X = A_3 Dinv_1, X C_1, Y = C_3 Dinv_5, Y A_5:
    # four dense 4 x 4 products of 2 4^3 = 128 flops
    H7 = _hacr(7)
    assert H7.setup_flops == {"gemm": 4 * 128, "qr": 0, "svd": 0, "rebuild": 0, "leaf_inverse": 7 * 128}


@pytest.mark.parametrize("nz", [3, 7])
def test_apply_bytes_counts_each_inverse_twice(nz):
    """Dense-only planes: the factor part of the count is twice every
    inverse below the top, the top once and every coupling once."""
    H = _hacr(nz)
    vec = 8 * 4
    factor = 0
    for r, role, p, obj in H.factor_list():
        e = obj.size * 8 if isinstance(obj, np.ndarray) else obj.stats()[0] * 8
        top = r == len(H.levels)
        factor += (2 if role == "Dinv" and not top else 1) * e
    vectors = H.apply_bytes(8) - factor
    assert vectors % vec == 0 and vectors > 0
