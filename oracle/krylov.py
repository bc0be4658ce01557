"""Krylov solvers in FP64 (oracle).

The paper uses the conjugate gradient method (Hestenes-Stiefel) with the
2-norm of the relative residual down to 1e-8 for symmetric problems
(Sec. 5.3) and GMRES for the nonsymmetric and indefinite ones (Sec. 7,
Sec. 8).  Both start from ``x0`` (zero by default).

* ``pcg``: preconditioned CG with Fletcher-Reeves ``beta = r1'z1 / r0'z0``
  or, with ``flexible=True``, Polak-Ribiere ``beta = r1'(z1 - z0)/r0'z0``;
  stops when the recursive residual meets the tolerance and then checks
  the true residual (continuing if it does not).
* ``gmres``: right-preconditioned restarted GMRES(m) with modified
  Gram-Schmidt and Givens rotations; with right preconditioning the
  monitored residual is the true residual of ``A x = b``.
"""
import numpy as np


def pcg(Aop, b, Minv=None, tol=1e-8, maxit=1000, x0=None, flexible=False):
    """Return ``(x, info)``; ``info = {iters, relres, history, status}``."""
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    Minv = Minv or (lambda v: v.copy())
    r = b - Aop(x)
    hist = [np.linalg.norm(r) / nb]
    if hist[-1] <= tol:
        return x, {"iters": 0, "relres": hist[-1], "history": hist, "status": "ok"}
    z = Minv(r)
    p = z.copy()
    rz = r @ z
    it = 0
    while it < maxit:
        it += 1
        Ap = Aop(p)
        pAp = p @ Ap
        if pAp <= 0:
            return x, {"iters": it, "relres": hist[-1], "history": hist, "status": "breakdown"}
        alpha = rz / pAp
        x += alpha * p
        r -= alpha * Ap
        hist.append(np.linalg.norm(r) / nb)
        if hist[-1] <= tol:
            rt = np.linalg.norm(b - Aop(x)) / nb
            if rt <= tol:
                hist[-1] = rt
                return x, {"iters": it, "relres": rt, "history": hist, "status": "ok"}
            r = b - Aop(x)
        z1 = Minv(r)
        rz1 = r @ z1
        beta = (rz1 - r @ z) / rz if flexible else rz1 / rz
        p = z1 + beta * p
        z, rz = z1, rz1
    return x, {"iters": it, "relres": hist[-1], "history": hist, "status": "notconv"}


def gmres(Aop, b, Minv=None, restart=30, tol=1e-8, maxit=1000, x0=None):
    """Right-preconditioned GMRES(m); returns ``(x, info)``."""
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    Minv = Minv or (lambda v: v.copy())
    hist = []
    it = 0
    while True:
        r = b - Aop(x)
        beta = np.linalg.norm(r)
        hist.append(beta / nb)
        if beta / nb <= tol:
            return x, {"iters": it, "relres": beta / nb, "history": hist, "status": "ok"}
        if it >= maxit:
            return x, {"iters": it, "relres": beta / nb, "history": hist, "status": "notconv"}
        m = restart
        V = np.zeros((m + 1, b.size))
        Z = np.zeros((m, b.size))
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        while k < m and it < maxit:
            Z[k] = Minv(V[k])
            w = Aop(Z[k])
            for i in range(k + 1):               # modified Gram-Schmidt
                H[i, k] = w @ V[i]
                w = w - H[i, k] * V[i]
            H[k + 1, k] = np.linalg.norm(w)
            if H[k + 1, k] > 0:
                V[k + 1] = w / H[k + 1, k]
            for i in range(k):                   # previous rotations
                a, c = H[i, k], H[i + 1, k]
                H[i, k], H[i + 1, k] = cs[i] * a + sn[i] * c, -sn[i] * a + cs[i] * c
            den = np.hypot(H[k, k], H[k + 1, k])
            cs[k], sn[k] = (H[k, k] / den, H[k + 1, k] / den) if den > 0 else (1.0, 0.0)
            H[k, k], H[k + 1, k] = den, 0.0
            g[k], g[k + 1] = cs[k] * g[k], -sn[k] * g[k]
            it += 1
            k += 1
            hist.append(abs(g[k]) / nb)
            if abs(g[k]) / nb <= tol:
                break
        y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
        x = x + Z[:k].T @ y
