"""Exact block cyclic reduction with dense plane blocks (oracle, eps = 0).

Textbook block cyclic reduction (Sec. 4.1): a red/black permutation of the
block rows followed by block Gaussian elimination without pivoting,
recursively halving the number of planes until one is left, then forward
and backward substitution.  The paper defers the recurrences to its 2D
predecessor; they are written out here in the notation
``A_k u_{k-1} + D_k u_k + C_k u_{k+1} = f_k``:

* level r works on the ordered plane list ``P_r``; the planes at 1-based
  odd positions are eliminated (set E_r), the even ones kept (set K_r);
* for i in E_r: ``Dinv_i = D_i^{-1}``;
* for kept j with neighbours j-1, j+1 (both eliminated):
  ``X = A_j Dinv_{j-1}``, ``Y = C_j Dinv_{j+1}``,
  ``D_j <- D_j - X C_{j-1} - Y A_{j+1}``, ``A_j <- -X A_{j-1}``,
  ``C_j <- -Y C_{j+1}``; absent neighbours drop their terms;
* the level-r blocks are stored before they are updated.

``apply`` computes ``z = M^{-1} g`` with forward elimination, the top
solve and back substitution; ``apply_T`` is the exact transpose of that
linear map (eliminated planes' couplings transposed in the forward pass,
kept planes' couplings transposed in the backward pass).
"""
import numpy as np


def _dense(x, B):
    if x is None:
        return None
    if np.ndim(x) == 1:
        return np.diag(x)
    return x.toarray() if hasattr(x, "toarray") else np.array(x, dtype=np.float64)


class DenseCR:
    """Exact cyclic reduction of a block-tridiagonal matrix with dense blocks."""

    def __init__(self, D, A, C):
        nz = len(D)
        B = D[0].shape[0]
        self.B, self.nz = B, nz
        D = [_dense(d, B) for d in D]
        A = [_dense(a, B) for a in A]
        C = [_dense(c, B) for c in C]
        self.levels = []           # list of dicts per level
        P = list(range(nz))
        while True:
            if len(P) == 1:
                self.top = (P[0], np.linalg.inv(D[P[0]]))
                break
            E, K = P[0::2], P[1::2]
            lev = {"P": P, "E": E, "K": K, "Dinv": {}, "A": {}, "C": {}}
            for i in E:
                lev["Dinv"][i] = np.linalg.inv(D[i])
            for p in P:
                lev["A"][p] = A[p]
                lev["C"][p] = C[p]
            newD, newA, newC = {}, {}, {}
            for m, j in enumerate(K):
                pos = 2 * m + 1
                im, ip = P[pos - 1], (P[pos + 1] if pos + 1 < len(P) else None)
                Dj = D[j].copy()
                X = A[j] @ lev["Dinv"][im]
                Dj -= X @ C[im]
                Aj = -X @ A[im] if A[im] is not None else None
                Cj = None
                if ip is not None:
                    Y = C[j] @ lev["Dinv"][ip]
                    Dj -= Y @ A[ip]
                    Cj = -Y @ C[ip] if C[ip] is not None else None
                newD[j], newA[j], newC[j] = Dj, Aj, Cj
            for j in K:
                D[j], A[j], C[j] = newD[j], newA[j], newC[j]
            self.levels.append(lev)
            P = K
        self.reduced = None

    def apply(self, g):
        """``z = M^{-1} g`` (here ``M = A`` exactly)."""
        B = self.B
        g = np.array(g, dtype=np.float64).reshape(self.nz, B).copy()
        w = {}
        for lev in self.levels:
            for i in lev["E"]:
                w[i] = lev["Dinv"][i] @ g[i]
            P = lev["P"]
            for m, j in enumerate(lev["K"]):
                pos = 2 * m + 1
                im, ip = P[pos - 1], (P[pos + 1] if pos + 1 < len(P) else None)
                g[j] -= lev["A"][j] @ w[im]
                if ip is not None:
                    g[j] -= lev["C"][j] @ w[ip]
        z = np.zeros_like(g)
        t, Dinv = self.top
        z[t] = Dinv @ g[t]
        for lev in reversed(self.levels):
            P = lev["P"]
            for m, i in enumerate(lev["E"]):
                pos = 2 * m
                r = g[i].copy()
                if pos > 0:
                    r -= lev["A"][i] @ z[P[pos - 1]]
                if pos + 1 < len(P):
                    r -= lev["C"][i] @ z[P[pos + 1]]
                z[i] = lev["Dinv"][i] @ r
        return z.reshape(-1)

    def apply_T(self, g):
        """``z = M^{-T} g``, the exact transpose of :meth:`apply`."""
        B = self.B
        y = np.array(g, dtype=np.float64).reshape(self.nz, B).copy()
        for lev in self.levels:
            P = lev["P"]
            v = {}
            for m, i in enumerate(lev["E"]):
                v[i] = lev["Dinv"][i].T @ y[i]
            for m, i in enumerate(lev["E"]):
                pos = 2 * m
                if pos > 0:
                    y[P[pos - 1]] -= lev["A"][i].T @ v[i]
                if pos + 1 < len(P):
                    y[P[pos + 1]] -= lev["C"][i].T @ v[i]
        z = np.zeros_like(y)
        t, Dinv = self.top
        z[t] = Dinv.T @ y[t]
        for lev in reversed(self.levels):
            P = lev["P"]
            for m, i in enumerate(lev["E"]):
                pos = 2 * m
                r = y[i].copy()
                if pos > 0:
                    r -= lev["C"][P[pos - 1]].T @ z[P[pos - 1]]
                if pos + 1 < len(P):
                    r -= lev["A"][P[pos + 1]].T @ z[P[pos + 1]]
                z[i] = lev["Dinv"][i].T @ r
        return z.reshape(-1)
