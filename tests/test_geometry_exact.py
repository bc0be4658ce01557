"""The library's plane geometry equals the oracle's, bit for bit (index
work): the H-order permutation of the bisection cluster tree (Sec. 3.1.2,
Sec. 4.2), the cluster and block-tree node counts, and every leaf of the
block tree with its admissibility under eq. admis, at the workload plane
sizes and a ragged one, for several eta.  The leaves stored dense although
admissible (only at large eta) must each hold an in-plane coupling of the
5-point operator.  Host only (the geometry needs no device)."""
import numpy as np
import pytest

from oracle import hmatrix as hm

import paper_1712_08872_amd as acr

SHAPES = [(127, 127), (63, 63), (47, 47), (45, 23), (31, 31)]


def _oracle_leaves(ct, bt):
    out = set()
    for (t, s), k in bt.kind.items():
        if k == "H":
            continue
        out.add((ct.lo[t], ct.lo[s], ct.size(t), ct.size(s), int(k == "L")))
    return out


def _has_coupling(perm, nx, r0, c0, m, n):
    """True if some row position in [r0, r0+m) and column position in
    [c0, c0+n) are grid neighbours (5-point stencil, in-plane)."""
    pos = np.empty_like(perm)
    pos[perm] = np.arange(perm.size)
    rows = perm[r0:r0 + m]
    x, y = rows % nx, rows // nx
    for dx, dy in ((-1, 0), (1, 0), (0, -1), (0, 1)):
        xx, yy = x + dx, y + dy
        ok = (xx >= 0) & (xx < nx) & (yy >= 0) & (yy < perm.size // nx)
        q = pos[(xx + nx * yy)[ok]]
        if np.any((q >= c0) & (q < c0 + n)):
            return True
    return False


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"{s[0]}x{s[1]}")
@pytest.mark.parametrize("eta", [1.0, 2.0, 4.0, 8.0, 256.0])
def test_geometry_equals_oracle(shape, eta):
    nx, ny = shape
    leaf = 32
    ct = hm.ClusterTree(nx, ny, leaf)
    bt = hm.BlockTree(ct, eta)
    info, perm, leaves = acr.acr_plane_geometry(nx, ny, eta=eta, leaf_size=leaf)
    assert np.array_equal(perm.astype(np.int64), ct.perm)
    assert info["clusters"] == len(ct.box)
    assert info["leaf_clusters"] == sum(c is None for c in ct.children)
    assert info["depth"] == max(ct.depth)
    assert info["block_nodes"] == len(bt.kind)
    ol = _oracle_leaves(ct, bt)
    mine = {tuple(int(v) for v in row[:5]) for row in leaves}
    assert len(mine) == info["leaves"] == len(leaves) == len(ol)
    assert mine == ol
    assert info["admissible"] == sum(k == "L" for k in bt.kind.values())
    assert info["lr_leaves"] + info["dense_leaves"] == info["leaves"]
    # low rank only where admissible; admissible but dense only around an in-plane coupling
    for r0, c0, m, n, adm, lr in leaves:
        assert lr <= adm
        if adm and not lr:
            assert _has_coupling(perm.astype(np.int64), nx, r0, c0, m, n), (r0, c0, m, n)
        if adm and lr:
            assert not _has_coupling(perm.astype(np.int64), nx, r0, c0, m, n), (r0, c0, m, n)


@pytest.mark.parametrize("leaf", [16, 64])
def test_geometry_other_leaf_sizes(leaf):
    nx, ny = 63, 40
    ct = hm.ClusterTree(nx, ny, leaf)
    bt = hm.BlockTree(ct, 2.0)
    info, perm, leaves = acr.acr_plane_geometry(nx, ny, eta=2.0, leaf_size=leaf)
    assert np.array_equal(perm.astype(np.int64), ct.perm)
    assert {tuple(int(v) for v in row[:5]) for row in leaves} == _oracle_leaves(ct, bt)


def test_dense_work_keeps_small_admissible_leaves_dense():
    info0, _, lv0 = acr.acr_plane_geometry(63, 63, eta=2.0, dense_work=0)
    info8, _, lv8 = acr.acr_plane_geometry(63, 63, eta=2.0, dense_work=8)
    assert np.array_equal(lv0[:, :5], lv8[:, :5])
    small = (lv0[:, 4] == 1) & (np.minimum(lv0[:, 2], lv0[:, 3]) <= 8)
    assert np.all(lv8[small, 5] == 0) and np.array_equal(lv8[~small, 5], lv0[~small, 5])


def test_leaves_cap_is_checked():
    import ctypes
    o = acr.default_options()
    info = acr.GeometryInfo()
    buf = (ctypes.c_int32 * 6)()
    st = acr.lib().acr_plane_geometry(31, 31, ctypes.byref(o), ctypes.byref(info), None, buf, 1)
    assert st == 1 and info.leaves > 1
