"""Accelerated cyclic reduction with H-matrix plane blocks (oracle, FP64).

Sec. 4.2 of the paper: the block cyclic reduction of ``dense_cr`` with every
formally dense plane block held as an H-matrix on the plane's bisection
tree, and every block operation replaced by its H-arithmetic counterpart
at accuracy eps (inverse, formatted product, truncated addition).  The
level-0 blocks are exact: ``D_k`` is the in-plane 5-point part converted
leaf by leaf, ``A_k`` and ``C_k`` are the diagonal z-couplings (vectors).

Stored factors, per level r: ``Dinv_i, A_i, C_i`` for eliminated ``i`` and
``A_j, C_j`` for kept ``j`` (the values at level r, before the update),
plus ``Dinv`` of the single top plane.  ``apply`` / ``apply_T`` are the
forward/backward sweeps of the dense reference, with H-matvecs.
"""
import numpy as np

from . import hmatrix as hm
from .assembly import plane_blocks
from .fem27 import plane_blocks27


def _coupling_matvec(cp, x, transpose=False):
    kind, val = cp
    if kind == "diag":
        return val * x
    return val.matvec(x, transpose)


class HACR:
    """H-matrix cyclic reduction preconditioner ``M^{-1} ~ A^{-1}``."""

    def __init__(self, S, nx, ny, nz, eps, eta=2.0, leaf=32):
        """``S``: a (7, N) stencil of the 7-point operators or a (27, N)
        stencil of the trilinear finite-element operator (``fem27``)."""
        self.nx, self.ny, self.nz, self.eps = nx, ny, nz, eps
        f0 = hm.flops_snapshot()
        self.ct = hm.ClusterTree(nx, ny, leaf)
        self.bt = hm.BlockTree(self.ct, eta)
        perm = self.ct.perm
        self.perm = perm
        if S.shape[0] == 27:
            # 27-point operator (Sec. 8): the z-couplings are 9-point in-plane matrices, held
            # as H-matrices from the start, so level 0 uses the formatted products too
            Dsp, Asp, Csp = plane_blocks27(S, nx, ny, nz)
            D = [self._from_sparse(d[perm][:, perm].tocsr()) for d in Dsp]
            A = [("H", self._from_sparse(a[perm][:, perm].tocsr())) if a is not None else None for a in Asp]
            C = [("H", self._from_sparse(c[perm][:, perm].tocsr())) if c is not None else None for c in Csp]
        else:
            Dsp, Av, Cv = plane_blocks(S, nx, ny, nz)
            D = [self._from_sparse(d[perm][:, perm].tocsr()) for d in Dsp]
            A = [("diag", a[perm]) if a is not None else None for a in Av]
            C = [("diag", c[perm]) if c is not None else None for c in Cv]
        self.levels = []
        P = list(range(nz))
        while True:
            if len(P) == 1:
                self.top = (P[0], hm.inverse(D[P[0]], eps))
                break
            E, K = P[0::2], P[1::2]
            lev = {"P": P, "E": E, "K": K, "Dinv": {}, "A": {}, "C": {}}
            for i in E:
                lev["Dinv"][i] = hm.inverse(D[i], eps)
            for p in P:
                lev["A"][p], lev["C"][p] = A[p], C[p]
            newD, newA, newC = {}, {}, {}
            for m, j in enumerate(K):
                pos = 2 * m + 1
                im, ip = P[pos - 1], (P[pos + 1] if pos + 1 < len(P) else None)
                Dj = D[j]
                X = self._left(A[j], lev["Dinv"][im])
                self._sub_prod(Dj, X, C[im])
                Aj = self._neg_prod(X, A[im])
                Cj = None
                if ip is not None:
                    Y = self._left(C[j], lev["Dinv"][ip])
                    self._sub_prod(Dj, Y, A[ip])
                    Cj = self._neg_prod(Y, C[ip])
                newD[j], newA[j], newC[j] = Dj, Aj, Cj
            for j in K:
                D[j], A[j], C[j] = newD[j], newA[j], newC[j]
            self.levels.append(lev)
            P = K
        #: algorithmic flops of the setup by class (counter, see hmatrix.FLOPS)
        self.setup_flops = {k: v - f0[k] for k, v in hm.flops_snapshot().items()}

    # ---- helpers
    def _from_sparse(self, Dp):
        bt, ct = self.bt, self.ct

        def rec(t, s):
            h = hm.HM(bt, t, s)
            if h.kind == "H":
                h.ch = [[rec(*bt.children[(t, s)][i][j]) for j in range(2)] for i in range(2)]
                return h
            blk = Dp[ct.lo[t]:ct.hi[t], ct.lo[s]:ct.hi[s]].toarray()
            if h.kind == "D":
                h.D = blk
            else:   # exact low-rank form of the couplings inside an admissible block
                h.U, h.V = hm.compress_dense(blk, 1e-15)
            return h
        return rec(0, 0)

    def _left(self, cp, Dinv):
        """``X = cp * Dinv`` (coupling times H-inverse)."""
        kind, val = cp
        if kind == "diag":
            return Dinv.copy().scale(1.0, row=val)
        X = hm.HM.zeros(self.bt)
        hm.mul(1.0, val, Dinv, X, self.eps)
        return X

    def _sub_prod(self, Dj, X, cp):
        """``Dj <- T_eps(Dj - X cp)``."""
        if cp is None:
            return
        kind, val = cp
        if kind == "diag":
            hm.add(Dj, -1.0, X.copy().scale(1.0, col=val), self.eps)
        else:
            hm.mul(-1.0, X, val, Dj, self.eps)

    def _neg_prod(self, X, cp):
        """``-X cp`` as a new coupling (None if ``cp`` is absent)."""
        if cp is None:
            return None
        kind, val = cp
        if kind == "diag":
            return ("H", X.copy().scale(-1.0, col=val))
        out = hm.HM.zeros(self.bt)
        hm.mul(-1.0, X, val, out, self.eps)
        return ("H", out)

    # ---- preconditioner
    def _planes(self, v):
        B = self.nx * self.ny
        return np.asarray(v, dtype=np.float64).reshape(self.nz, B)[:, self.perm].copy()

    def _unplanes(self, g):
        out = np.empty_like(g)
        out[:, self.perm] = g
        return out.reshape(-1)

    def apply(self, r):
        """``z = M^{-1} r`` (natural ordering in and out)."""
        g = self._planes(r)
        w = {}
        for lev in self.levels:
            for i in lev["E"]:
                w[i] = lev["Dinv"][i].matvec(g[i])
            P = lev["P"]
            for m, j in enumerate(lev["K"]):
                pos = 2 * m + 1
                g[j] -= _coupling_matvec(lev["A"][j], w[P[pos - 1]])
                if pos + 1 < len(P):
                    g[j] -= _coupling_matvec(lev["C"][j], w[P[pos + 1]])
        z = np.zeros_like(g)
        t, Dinv = self.top
        z[t] = Dinv.matvec(g[t])
        for lev in reversed(self.levels):
            P = lev["P"]
            for m, i in enumerate(lev["E"]):
                pos = 2 * m
                rr = g[i].copy()
                if pos > 0:
                    rr -= _coupling_matvec(lev["A"][i], z[P[pos - 1]])
                if pos + 1 < len(P):
                    rr -= _coupling_matvec(lev["C"][i], z[P[pos + 1]])
                z[i] = lev["Dinv"][i].matvec(rr)
        return self._unplanes(z)

    def apply_T(self, r):
        """``z = M^{-T} r``, the exact transpose of :meth:`apply`."""
        y = self._planes(r)
        for lev in self.levels:
            P = lev["P"]
            for m, i in enumerate(lev["E"]):
                pos = 2 * m
                v = lev["Dinv"][i].matvec(y[i], transpose=True)
                if pos > 0:
                    y[P[pos - 1]] -= _coupling_matvec(lev["A"][i], v, True)
                if pos + 1 < len(P):
                    y[P[pos + 1]] -= _coupling_matvec(lev["C"][i], v, True)
        z = np.zeros_like(y)
        t, Dinv = self.top
        z[t] = Dinv.matvec(y[t], transpose=True)
        for lev in reversed(self.levels):
            P = lev["P"]
            for m, i in enumerate(lev["E"]):
                pos = 2 * m
                rr = y[i].copy()
                if pos > 0:
                    rr -= _coupling_matvec(lev["C"][P[pos - 1]], z[P[pos - 1]], True)
                if pos + 1 < len(P):
                    rr -= _coupling_matvec(lev["A"][P[pos + 1]], z[P[pos + 1]], True)
                z[i] = lev["Dinv"][i].matvec(rr, transpose=True)
        return self._unplanes(z)

    # ---- statistics
    def factor_list(self):
        """Every stored factor as (level, role, plane, object)."""
        out = []
        for r, lev in enumerate(self.levels):
            for i in lev["E"]:
                out.append((r, "Dinv", i, lev["Dinv"][i]))
            for p in lev["P"]:
                for role in ("A", "C"):
                    cp = lev[role][p]
                    if cp is not None:
                        out.append((r, role, p, cp[1]))
        out.append((len(self.levels), "Dinv", self.top[0], self.top[1]))
        return out

    def apply_bytes(self, esz=8):
        """Algorithmic bytes of one :meth:`apply` (counter).

        Every step of the sweeps reads the stored factors it multiplies by
        (an H-matrix at its stored entries times ``esz`` bytes, a level-0
        diagonal coupling at 8 bytes per entry), the plane vectors it reads
        and the plane vector it updates, and writes one plane vector (plane
        vectors are FP64, ``8 nx ny`` bytes).  Per level, forward: each
        eliminated plane ``w_i = Dinv_i g_i``; each kept plane
        ``g_j -= A_j w + C_j w`` (reads g_j, the present couplings and their
        w, writes g_j).  Top: ``z = Dinv g``.  Backward, each eliminated
        plane: ``rr = g_i - A_i z - C_i z`` then ``z_i = Dinv_i rr``.
        """
        vec = 8 * self.nx * self.ny

        def fb(cp):
            if isinstance(cp, tuple):
                kind, val = cp
                return 8 * val.size if kind == "diag" else esz * val.stats()[0]
            return esz * cp.stats()[0]

        total = 0
        for lev in self.levels:
            P = lev["P"]
            for i in lev["E"]:
                total += 2 * vec + fb(lev["Dinv"][i])
            for m, j in enumerate(lev["K"]):
                pos = 2 * m + 1
                total += 2 * vec + vec + fb(lev["A"][j])
                if pos + 1 < len(P):
                    total += vec + fb(lev["C"][j])
        total += 2 * vec + fb(self.top[1])
        for lev in reversed(self.levels):
            P = lev["P"]
            for m, i in enumerate(lev["E"]):
                pos = 2 * m
                total += 2 * vec
                if pos > 0:
                    total += vec + fb(lev["A"][i])
                if pos + 1 < len(P):
                    total += vec + fb(lev["C"][i])
                total += 2 * vec + fb(lev["Dinv"][i])
        return total

    def stats(self):
        """Stored FP64 entries, per-level max and mean rank."""
        entries, per_level = 0, {}
        for r, role, p, obj in self.factor_list():
            if isinstance(obj, np.ndarray):
                entries += obj.size
                continue
            e, mx, sm, nl = obj.stats()
            entries += e
            d = per_level.setdefault(r, [0, 0, 0])
            d[0] = max(d[0], mx); d[1] += sm; d[2] += nl
        return {"entries": entries,
                "max_rank": {r: v[0] for r, v in per_level.items()},
                "mean_rank": {r: (v[1] / v[2] if v[2] else 0.0) for r, v in per_level.items()}}
