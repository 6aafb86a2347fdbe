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


def penetrable_sphere(k: float, km: float, a: float, d: np.ndarray, X: np.ndarray,
                      lmax: int | None = None) -> np.ndarray:
    """Plane-wave scattering by a penetrable sphere of radius a with interior
    wavenumber km and equal densities: the transmission conditions of the
    paper (u^i + u = u^- and d/dr(u^i + u) = du^-/dr at r = a, u^i zero
    inside).  With u = sum_l (2l+1) i^l A_l h_l(k r) P_l(cos g) outside and
    u^- = sum_l (2l+1) i^l B_l j_l(km r) P_l(cos g) inside, the two
    conditions give per degree
        j_l(ka) + A_l h_l(ka) = B_l j_l(km a),
        k (j_l'(ka) + A_l h_l'(ka)) = km B_l j_l'(km a).
    Returns u at points with |x| > a and u^- at points with |x| < a."""
    d = np.asarray(d, float) / np.linalg.norm(d)
    r = np.linalg.norm(X, axis=1)
    cg = (X @ d) / r
    L = int(max(k, km) * max(a, r.max()) + 40) if lmax is None else lmax
    out = np.zeros(X.shape[0], dtype=np.complex128)
    inside = r < a
    for l in range(L + 1):
        j, jp = spherical_jn(l, k * a), spherical_jn(l, k * a, derivative=True)
        h = j + 1j * spherical_yn(l, k * a)
        hp = jp + 1j * spherical_yn(l, k * a, derivative=True)
        jm, jmp = spherical_jn(l, km * a), spherical_jn(l, km * a, derivative=True)
        # 2x2 system [[h, -jm], [k h', -km jm']] [A; B] = [-j; -k j']
        det = -h * km * jmp + jm * k * hp
        A = (j * km * jmp - jm * k * jp) / det
        B = (j * k * hp - h * k * jp) / det
        Pl = eval_legendre(l, cg)
        ho = spherical_jn(l, k * r) + 1j * spherical_yn(l, k * r)
        ji = spherical_jn(l, km * r)
        out += (2 * l + 1) * (1j ** l) * Pl * np.where(inside, B * ji, A * ho)
    return out
