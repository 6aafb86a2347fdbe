"""Unrestarted GMRES from a zero initial guess (the Krylov method named for
eq. (iter)); Arnoldi with modified Gram-Schmidt, the small least-squares
problem solved with numpy at every step (plain, not incremental)."""
from __future__ import annotations

import numpy as np


def gmres(op, b: np.ndarray, tol: float, maxit: int):
    """Solve op(x) = b.  Stops when ||b - op(x)|| <= tol ||b|| (the residual
    of the Hessenberg least-squares problem, which equals the true residual
    in exact arithmetic).  Returns (x, iterations, relative residual history)."""
    bn = np.linalg.norm(b)
    if bn == 0:
        return np.zeros_like(b), 0, [0.0]
    V = [b / bn]
    H = np.zeros((maxit + 1, maxit), dtype=np.complex128)
    hist = [1.0]
    y = np.zeros(0, dtype=np.complex128)
    for j in range(maxit):
        w = op(V[j])
        for i in range(j + 1):
            H[i, j] = np.vdot(V[i], w)
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        e1 = np.zeros(j + 2, dtype=np.complex128)
        e1[0] = bn
        y, *_ = np.linalg.lstsq(H[:j + 2, :j + 1], e1, rcond=None)
        res = np.linalg.norm(H[:j + 2, :j + 1] @ y - e1) / bn
        hist.append(float(res))
        if res <= tol or H[j + 1, j] == 0:
            break
        V.append(w / H[j + 1, j])
    x = sum(y[i] * V[i] for i in range(len(y)))
    return x, len(y), hist
