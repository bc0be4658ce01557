"""H-matrices on one grid plane (oracle, FP64, plain recursive code).

Construction follows Sec. 3.1 and Sec. 4.2 of the paper:

* Cluster tree (Sec. 3.1.2, planar bisection of Sec. 4.2): the root is the
  whole ``nx x ny`` index box of a plane; a box with at most ``leaf``
  points (the paper's n_min) is a leaf; otherwise its longer side is split
  (ties split x) into ``floor(s/2)`` and the rest, lower coordinates
  first.  Depth-first leaf order defines the H-order permutation.
* Block cluster tree with the standard admissibility condition (eq.
  admis): ``(t, s)`` is admissible iff ``dist > 0`` and
  ``min(diam t, diam s) <= eta * dist``; diam and dist are Euclidean, of
  the bounding boxes in grid-index units.  Admissible blocks are low-rank
  leaves ``U V^T``; inadmissible blocks with a leaf cluster are dense
  leaves; the rest are split 2 x 2.  One block tree serves every
  H-matrix of a plane shape.
* Truncation ``T_eps`` (Sec. 3.1.5, Sec. 4.3): QR of ``U`` and of ``V``,
  SVD of ``R_U R_V^T``; singular values ``sigma_i > eps * sigma_1`` are
  kept (block-wise relative accuracy).  A zero block has rank 0.

Arithmetic (Hackbusch's formatted arithmetic on the common tree):
``mul(alpha, A, B, C)`` is ``C <- T_eps(C + alpha A B)`` by recursion over
the 2 x 2 children, products with a low-rank factor kept low rank,
dense x dense products dense, and every addition into a low-rank leaf
truncated.  ``inverse`` is the recursive 2 x 2 block inverse through the
Schur complement of the first diagonal child, with LU-based (partial
pivoting) inverses of the dense diagonal leaves.
"""
import numpy as np
import scipy.linalg as sla

# ------------------------------------------------------------- counters
# Algorithmic flops of the H-arithmetic by class (counters, not timings):
#   gemm          2 m n k for every product of an m x k and a k x n matrix;
#   qr            4 m K^2 - 4 K^3 / 3 for a Householder QR of an m x K
#                 factor with Q formed;
#   svd           22 K^3 for the SVD of a K x K core; 14 M n^2 + 8 n^3
#                 (M >= n) for the thin SVD of an M x n dense block;
#   rebuild       2 m K k for forming an m x k truncated factor from Q;
#   leaf_inverse  2 m^3 for the LU factorisation and inverse of an m x m leaf.
FLOPS = {"gemm": 0, "qr": 0, "svd": 0, "rebuild": 0, "leaf_inverse": 0}


def reset_flops():
    for k in FLOPS:
        FLOPS[k] = 0


def flops_snapshot():
    return dict(FLOPS)


def _svd_flops(m, n):
    M, q = max(m, n), min(m, n)
    return 14 * M * q * q + 8 * q ** 3


# ---------------------------------------------------------------- trees
class ClusterTree:
    """Binary bisection tree of the ``nx x ny`` plane."""

    def __init__(self, nx, ny, leaf=32):
        self.nx, self.ny, self.leaf = nx, ny, leaf
        self.box, self.children, self.lo, self.hi, self.depth = [], [], [], [], []
        self.perm = []           # H-order position -> natural in-plane index

        def rec(x0, x1, y0, y1, d):
            cid = len(self.box)
            self.box.append((x0, x1, y0, y1))
            self.children.append(None)
            self.depth.append(d)
            self.lo.append(len(self.perm))
            self.hi.append(None)
            sx, sy = x1 - x0, y1 - y0
            if sx * sy <= leaf:
                for y in range(y0, y1):
                    for x in range(x0, x1):
                        self.perm.append(x + nx * y)
            elif sx >= sy:
                m = x0 + sx // 2
                self.children[cid] = (rec(x0, m, y0, y1, d + 1), rec(m, x1, y0, y1, d + 1))
            else:
                m = y0 + sy // 2
                self.children[cid] = (rec(x0, x1, y0, m, d + 1), rec(x0, x1, m, y1, d + 1))
            self.hi[cid] = len(self.perm)
            return cid

        rec(0, nx, 0, ny, 0)
        self.perm = np.array(self.perm, dtype=np.int64)
        self.iperm = np.empty_like(self.perm)
        self.iperm[self.perm] = np.arange(len(self.perm))

    def size(self, c):
        return self.hi[c] - self.lo[c]

    def is_leaf(self, c):
        return self.children[c] is None

    def diam2(self, c):
        x0, x1, y0, y1 = self.box[c]
        return (x1 - 1 - x0) ** 2 + (y1 - 1 - y0) ** 2

    def dist2(self, a, b):
        ax0, ax1, ay0, ay1 = self.box[a]
        bx0, bx1, by0, by1 = self.box[b]
        dx = max(0, bx0 - (ax1 - 1), ax0 - (bx1 - 1))
        dy = max(0, by0 - (ay1 - 1), ay0 - (by1 - 1))
        return dx * dx + dy * dy

    def admissible(self, t, s, eta):
        d2 = self.dist2(t, s)
        return d2 > 0 and min(self.diam2(t), self.diam2(s)) <= eta * eta * d2


class BlockTree:
    """Block cluster tree: ``kind[(t,s)]`` in {'H', 'D', 'L'}."""

    def __init__(self, ct, eta):
        self.ct, self.eta = ct, eta
        self.kind, self.children = {}, {}

        def rec(t, s):
            if ct.admissible(t, s, eta):
                self.kind[(t, s)] = "L"
            elif ct.is_leaf(t) or ct.is_leaf(s):
                self.kind[(t, s)] = "D"
            else:
                self.kind[(t, s)] = "H"
                ch = [[None, None], [None, None]]
                for i, ti in enumerate(ct.children[t]):
                    for j, sj in enumerate(ct.children[s]):
                        ch[i][j] = (ti, sj)
                        rec(ti, sj)
                self.children[(t, s)] = ch

        rec(0, 0)

    def leaves(self, kind=None):
        return [b for b, k in self.kind.items() if k != "H" and (kind is None or k == kind)]


# ----------------------------------------------------------- truncation
def truncate(U, V, eps, max_rank=0):
    """``T_eps(U V^T)``: keep ``sigma_i > eps sigma_1``.

    The singular values come from QR of ``U`` and ``V`` and an SVD of
    ``R_U R_V^T``; when the concatenated rank is at least the smaller block
    dimension the block is formed and decomposed directly (same result,
    fewer factorizations).
    """
    m, n = U.shape[0], V.shape[0]
    K = U.shape[1]
    if K == 0:
        return np.zeros((m, 0)), np.zeros((n, 0))
    if K >= min(m, n):
        FLOPS["gemm"] += 2 * m * n * K
        return compress_dense(U @ V.T, eps, max_rank)
    Qu, Ru = sla.qr(U, mode="economic", check_finite=False)
    Qv, Rv = sla.qr(V, mode="economic", check_finite=False)
    FLOPS["qr"] += 4 * (m + n) * K * K - 8 * K ** 3 // 3
    W, s, Zt = sla.svd(Ru @ Rv.T, check_finite=False)
    FLOPS["gemm"] += 2 * K ** 3
    FLOPS["svd"] += 22 * K ** 3
    if s.size == 0 or s[0] == 0.0:
        return np.zeros((m, 0)), np.zeros((n, 0))
    k = int(np.count_nonzero(s > eps * s[0]))
    if max_rank:
        k = min(k, max_rank)
    FLOPS["rebuild"] += 2 * (m + n) * K * k
    return (Qu @ W[:, :k]) * s[:k], Qv @ Zt[:k].T


def compress_dense(M, eps, max_rank=0):
    """Best rank-k approximation of a dense block with ``sigma_i > eps sigma_1``."""
    FLOPS["svd"] += _svd_flops(*M.shape)
    W, s, Zt = sla.svd(M, full_matrices=False, check_finite=False)
    if s.size == 0 or s[0] == 0.0:
        return np.zeros((M.shape[0], 0)), np.zeros((M.shape[1], 0))
    k = int(np.count_nonzero(s > eps * s[0]))
    if max_rank:
        k = min(k, max_rank)
    return W[:, :k] * s[:k], Zt[:k].T


# ------------------------------------------------------------- H-matrix
class HM:
    """One node of an H-matrix on block ``(t, s)`` of a BlockTree."""

    __slots__ = ("bt", "t", "s", "kind", "D", "U", "V", "ch")

    def __init__(self, bt, t, s):
        self.bt, self.t, self.s = bt, t, s
        self.kind = bt.kind[(t, s)]
        self.D = self.U = self.V = self.ch = None

    @property
    def shape(self):
        ct = self.bt.ct
        return (ct.size(self.t), ct.size(self.s))

    # -- construction
    @staticmethod
    def zeros(bt, t=0, s=0):
        h = HM(bt, t, s)
        m, n = h.shape
        if h.kind == "D":
            h.D = np.zeros((m, n))
        elif h.kind == "L":
            h.U, h.V = np.zeros((m, 0)), np.zeros((n, 0))
        else:
            h.ch = [[HM.zeros(bt, *bt.children[(t, s)][i][j]) for j in range(2)] for i in range(2)]
        return h

    @staticmethod
    def from_dense(bt, M, eps, t=0, s=0):
        """H-approximation of a dense matrix given in H-order."""
        h = HM(bt, t, s)
        ct = bt.ct
        if h.kind == "H":
            h.ch = [[HM.from_dense(bt, M, eps, *bt.children[(t, s)][i][j]) for j in range(2)] for i in range(2)]
            return h
        blk = M[ct.lo[t]:ct.hi[t], ct.lo[s]:ct.hi[s]]
        if h.kind == "D":
            h.D = np.array(blk, dtype=np.float64)
        else:
            h.U, h.V = compress_dense(blk, eps)
        return h

    def copy(self):
        h = HM(self.bt, self.t, self.s)
        if self.kind == "D":
            h.D = self.D.copy()
        elif self.kind == "L":
            h.U, h.V = self.U.copy(), self.V.copy()
        else:
            h.ch = [[c.copy() for c in row] for row in self.ch]
        return h

    def scale(self, alpha, row=None, col=None):
        """In place ``diag(row) * alpha * H * diag(col)``; ``row``/``col``
        are vectors over this block's rows/columns in H-order."""
        if self.kind == "D":
            self.D *= alpha
            if row is not None:
                self.D *= row[:, None]
            if col is not None:
                self.D *= col[None, :]
        elif self.kind == "L":
            self.U = self.U * alpha
            if row is not None:
                self.U = self.U * row[:, None]
            if col is not None:
                self.V = self.V * col[:, None]
        else:
            ct = self.bt.ct
            for i in range(2):
                for j in range(2):
                    c = self.ch[i][j]
                    r0 = ct.lo[c.t] - ct.lo[self.t]
                    c0 = ct.lo[c.s] - ct.lo[self.s]
                    rr = None if row is None else row[r0:r0 + ct.size(c.t)]
                    cc = None if col is None else col[c0:c0 + ct.size(c.s)]
                    c.scale(alpha, rr, cc)
        return self

    # -- evaluation
    def to_dense(self):
        if self.kind == "D":
            return self.D.copy()
        if self.kind == "L":
            return self.U @ self.V.T
        m, n = self.shape
        out = np.empty((m, n))
        ct = self.bt.ct
        for row in self.ch:
            for c in row:
                r0 = ct.lo[c.t] - ct.lo[self.t]
                c0 = ct.lo[c.s] - ct.lo[self.s]
                out[r0:r0 + ct.size(c.t), c0:c0 + ct.size(c.s)] = c.to_dense()
        return out

    def matvec(self, X, transpose=False):
        """``H X`` (or ``H^T X``) for a dense ``X`` with one column per vector."""
        X = np.asarray(X, dtype=np.float64)
        ncol = X.shape[1] if X.ndim > 1 else 1
        if self.kind == "D":
            FLOPS["gemm"] += 2 * self.D.size * ncol
            return (self.D.T if transpose else self.D) @ X
        if self.kind == "L":
            FLOPS["gemm"] += 2 * (self.U.size + self.V.size) * ncol
            if transpose:
                return self.V @ (self.U.T @ X)
            return self.U @ (self.V.T @ X)
        m, n = self.shape
        if transpose:
            m, n = n, m
        out = np.zeros((m,) + X.shape[1:])
        ct = self.bt.ct
        for row in self.ch:
            for c in row:
                ro, co = ct.lo[c.t] - ct.lo[self.t], ct.lo[c.s] - ct.lo[self.s]
                rn, cn = ct.size(c.t), ct.size(c.s)
                if transpose:
                    out[co:co + cn] += c.matvec(X[ro:ro + rn], True)
                else:
                    out[ro:ro + rn] += c.matvec(X[co:co + cn])
        return out

    # -- statistics
    def stats(self):
        """(stored entries, max rank, sum of ranks, number of LR leaves)."""
        if self.kind == "D":
            return self.D.size, 0, 0, 0
        if self.kind == "L":
            k = self.U.shape[1]
            return self.U.size + self.V.size, k, k, 1
        e = mx = sm = nl = 0
        for row in self.ch:
            for c in row:
                a, b, cc, d = c.stats()
                e += a; mx = max(mx, b); sm += cc; nl += d
        return e, mx, sm, nl


# ------------------------------------------------------------ arithmetic
def _restrict(P, ct, t0, s0, t, s):
    """Restrict a product piece on (t0, s0) to the sub-block (t, s)."""
    r0, r1 = ct.lo[t] - ct.lo[t0], ct.hi[t] - ct.lo[t0]
    c0, c1 = ct.lo[s] - ct.lo[s0], ct.hi[s] - ct.lo[s0]
    if P[0] == "L":
        return ("L", P[1][r0:r1], P[2][c0:c1])
    return ("D", P[1][r0:r1, c0:c1])


def add_piece(C, alpha, P, eps, t0=None, s0=None):
    """``C <- T_eps(C + alpha P)`` where ``P`` is ``("L", U, V)`` or
    ``("D", M)`` given on block ``(t0, s0) ⊇ (C.t, C.s)``."""
    ct = C.bt.ct
    if t0 is None:
        t0, s0 = C.t, C.s
    if (t0, s0) != (C.t, C.s):
        P = _restrict(P, ct, t0, s0, C.t, C.s)
    if C.kind == "H":
        for row in C.ch:
            for c in row:
                add_piece(c, alpha, P, eps, C.t, C.s)
    elif C.kind == "D":
        if P[0] == "L":
            FLOPS["gemm"] += 2 * C.D.size * P[1].shape[1]
        C.D += alpha * (P[1] @ P[2].T if P[0] == "L" else P[1])
    else:
        if P[0] == "L":
            U = np.hstack([C.U, alpha * P[1]])
            V = np.hstack([C.V, P[2]])
        else:
            # exact low-rank form of a dense piece: (alpha P) I
            U = np.hstack([C.U, alpha * P[1]])
            V = np.hstack([C.V, np.eye(P[1].shape[1])])
        C.U, C.V = truncate(U, V, eps)


def add(C, alpha, X, eps):
    """``C <- T_eps(C + alpha X)`` for two H-matrices on the same block."""
    if C.kind == "H":
        for i in range(2):
            for j in range(2):
                add(C.ch[i][j], alpha, X.ch[i][j], eps)
    elif C.kind == "D":
        C.D += alpha * X.D
    else:
        C.U, C.V = truncate(np.hstack([C.U, alpha * X.U]), np.hstack([C.V, X.V]), eps)


def _product(A, B):
    """Exact product of two blocks with at least one leaf, as a piece."""
    if A.kind == "L":
        return ("L", A.U, B.matvec(A.V, transpose=True))
    if B.kind == "L":
        return ("L", A.matvec(B.U), B.V)
    if A.kind == "D" and B.kind == "D":
        FLOPS["gemm"] += 2 * A.D.shape[0] * A.D.shape[1] * B.D.shape[1]
        return ("D", A.D @ B.D)
    if A.kind == "D":
        return ("D", B.matvec(A.D.T, transpose=True).T)
    if B.kind == "D":
        return ("D", A.matvec(B.D))
    a, b = A.to_dense(), B.to_dense()
    FLOPS["gemm"] += 2 * a.shape[0] * a.shape[1] * b.shape[1]
    return ("D", a @ b)


def mul(alpha, A, B, C, eps):
    """Formatted product ``C <- T_eps(C + alpha A B)`` on matching blocks
    ``A:(t,r)``, ``B:(r,s)``, ``C:(t,s)``."""
    if A.kind == "H" and B.kind == "H" and C.kind == "H":
        for i in range(2):
            for j in range(2):
                for l in range(2):
                    mul(alpha, A.ch[i][l], B.ch[l][j], C.ch[i][j], eps)
        return
    add_piece(C, alpha, _product(A, B), eps)


def inverse(M, eps):
    """H-inverse of a diagonal block ``(t, t)`` by the recursive 2 x 2
    Schur-complement formula; returns a new HM, ``M`` is consumed."""
    if M.kind == "D":
        FLOPS["leaf_inverse"] += 2 * M.D.shape[0] ** 3
        lu, piv = sla.lu_factor(M.D)
        M.D = sla.lu_solve((lu, piv), np.eye(M.D.shape[0]))
        return M
    assert M.kind == "H"
    (M11, M12), (M21, M22) = M.ch
    bt = M.bt
    X11 = inverse(M11, eps)                       # X11 = M11^-1
    T12 = HM.zeros(bt, M12.t, M12.s)
    mul(1.0, X11, M12, T12, eps)                  # T12 = X11 M12
    T21 = HM.zeros(bt, M21.t, M21.s)
    mul(1.0, M21, X11, T21, eps)                  # T21 = M21 X11
    mul(-1.0, M21, T12, M22, eps)                 # S = M22 - M21 X11 M12
    X22 = inverse(M22, eps)                       # X22 = S^-1
    X12 = HM.zeros(bt, M12.t, M12.s)
    mul(-1.0, T12, X22, X12, eps)                 # X12 = -X11 M12 S^-1
    X21 = HM.zeros(bt, M21.t, M21.s)
    mul(-1.0, X22, T21, X21, eps)                 # X21 = -S^-1 M21 X11
    mul(-1.0, X12, T21, X11, eps)                 # X11 += X11 M12 S^-1 M21 X11
    M.ch = [[X11, X12], [X21, X22]]
    return M
