"""Test helper: the oracle's H-matrix cyclic reduction as the factor list
that acr_import_factors takes (leaves in the library's leaf order from
acr_plane_geometry, rows and columns in H-order)."""
import numpy as np

import paper_1712_08872_amd as acr

ROLE = {"Dinv": acr.FACTOR_DINV, "A": acr.FACTOR_A, "C": acr.FACTOR_C}


def leaf_blocks(h, ct, out=None):
    """(r0, c0) -> leaf node of an oracle H-matrix."""
    out = {} if out is None else out
    if h.kind == "H":
        for row in h.ch:
            for c in row:
                leaf_blocks(c, ct, out)
    else:
        out[(ct.lo[h.t], ct.lo[h.s])] = h
    return out


def encode(h, ct, leaves):
    """(ranks, data) of one H-matrix in the library's leaf order."""
    blocks = leaf_blocks(h, ct)
    ranks = np.zeros(len(leaves), dtype=np.int32)
    parts = []
    for l, (r0, c0, m, n, adm, lr) in enumerate(leaves):
        b = blocks[(int(r0), int(c0))]
        assert b.shape == (m, n)
        if lr:
            assert b.kind == "L"
            ranks[l] = b.U.shape[1]
            parts += [b.U.ravel(order="F"), b.V.ravel(order="F")]
        else:   # a dense leaf (an admissible one holding couplings is given densified)
            parts.append((b.D if b.kind == "D" else b.U @ b.V.T).ravel(order="F"))
    return ranks, np.concatenate(parts) if parts else np.zeros(0)


def oracle_factors(H, eta, leaf, dense_work=0):
    """The factor list of an oracle HACR object."""
    _, _, leaves = acr.acr_plane_geometry(H.nx, H.ny, eta=eta, leaf_size=leaf, dense_work=dense_work)
    out = []
    for r, role, p, obj in H.factor_list():
        f = dict(level=r, role=ROLE[role], plane=p)
        if isinstance(obj, np.ndarray):
            f.update(diag=True, data=obj)
        else:
            rk, data = encode(obj, H.ct, leaves)
            f.update(diag=False, ranks=rk, data=data)
        out.append(f)
    return out, leaves


def decode(f, leaves, B):
    """Dense H-ordered matrix of one encoded factor (the inverse of encode)."""
    if f["diag"]:
        return np.diag(f["data"])
    M = np.zeros((B, B))
    o = 0
    for l, (r0, c0, m, n, adm, lr) in enumerate(leaves):
        if lr:
            k = int(f["ranks"][l])
            U = f["data"][o:o + m * k].reshape((m, k), order="F")
            o += m * k
            V = f["data"][o:o + n * k].reshape((n, k), order="F")
            o += n * k
            M[r0:r0 + m, c0:c0 + n] = U @ V.T
        else:
            M[r0:r0 + m, c0:c0 + n] = f["data"][o:o + m * n].reshape((m, n), order="F")
            o += m * n
    assert o == f["data"].size
    return M
