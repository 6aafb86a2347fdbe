"""Mie series for plane-wave scattering by a sound-hard sphere (a textbook
closed form outside the paper, used to pin the one-obstacle solve of Sec. 3).

With incident u^i = exp(i k d.x) = sum_l (2l+1) i^l j_l(kr) P_l(cos g),
g the angle between x and d, the Neumann condition d(u^i + u)/dr = 0 at
r = a gives the outgoing scattered field
    u(x) = - sum_l (2l+1) i^l [j_l'(ka) / h_l'(ka)] h_l(k|x|) P_l(cos g),
with h_l = j_l + i y_l the spherical Hankel function of the first kind.
"""
from __future__ import annotations

import numpy as np
from scipy.special import eval_legendre, spherical_jn, spherical_yn


def sound_hard_sphere(k: float, a: float, d: np.ndarray, X: np.ndarray,
                      lmax: int | None = None) -> np.ndarray:
    d = np.asarray(d, float) / np.linalg.norm(d)
    r = np.linalg.norm(X, axis=1)
    cg = (X @ d) / r
    L = int(k * max(a, r.max()) + 40) if lmax is None else lmax
    u = np.zeros(X.shape[0], dtype=np.complex128)
    for l in range(L + 1):
        jp = spherical_jn(l, k * a, derivative=True)
        hp = jp + 1j * spherical_yn(l, k * a, derivative=True)
        h = spherical_jn(l, k * r) + 1j * spherical_yn(l, k * r)
        u += -(2 * l + 1) * (1j ** l) * (jp / hp) * h * eval_legendre(l, cg)
    return u
