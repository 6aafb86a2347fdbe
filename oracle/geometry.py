"""Generating curve, normals, collocation nodes and MFS sources (Sec. 3 and
Sec. 3.2 of the paper).

The body is the rotation about the z axis of a curve (rho(t), z(t)),
t in [0, pi], with z'(0) = z'(pi) = 0 (Sec. 3, start).  Two families:
  * polar: rho = r(t) sin t, z = r(t) cos t with r(t) = a (1 + eps cos j t);
  * the cup of Fig. 1(c): radius r(u) = 1 - a erf((u - pi/2)/a) and polar
    angle theta(u) = b - a + 2 (1 - (b - a)/pi) s_a(u - pi/2), with s_a the
    a-rounded absolute value s_a(x) = x erf(x/a) + (a/sqrt(pi)) e^{-x^2/a^2},
    rho = c r sin theta, z = c r cos theta, c = outer/(1 + a).
Both are traversed clockwise in the (rho, z) half plane (t = 0 at the top
pole for the polar family, at the inner bottom pole for the cup, which takes
u = pi - t), so that (-z', rho')/s is the outward normal and Z(t - i tau)
lies inside the body for tau > 0.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy.special import erf

from workloads import Body, CupShape, Shape


def radius(shape: Shape, t):
    """r(t) = a (1 + eps cos(j t)); t may be complex."""
    return shape.a * (1.0 + shape.eps * np.cos(shape.j * t))


def radius_dt(shape: Shape, t):
    return -shape.a * shape.eps * shape.j * np.sin(shape.j * t)


def cup_parts(sh: CupShape, t):
    """Cup radius r and polar angle theta (Fig. 1(c)) at u = pi - t, and the
    scale c; t may be complex (the formulas continue analytically)."""
    a, b = sh.half, sh.b
    x = (math.pi - t) - math.pi / 2
    r = 1.0 - a * erf(x / a)
    s_a = x * erf(x / a) + (a / math.sqrt(math.pi)) * np.exp(-(x / a) ** 2)
    th = b - a + 2.0 * (1.0 - (b - a) / math.pi) * s_a
    return r, th, sh.outer / (1.0 + a)


def curve_Z(shape, t):
    """The curve as one complex function Z(t) = rho(t) + i z(t):
    r(t) (sin t + i cos t) for the polar family, c r (sin theta + i cos theta)
    for the cup.  Evaluating it at complex t gives the complexified source
    points of Sec. 3.2, method (c)."""
    if isinstance(shape, CupShape):
        r, th, c = cup_parts(shape, t)
        return c * r * (np.sin(th) + 1j * np.cos(th))
    return radius(shape, t) * (np.sin(t) + 1j * np.cos(t))


@dataclass
class Geometry:
    """Collocation points with outward unit normals, and source points,
    all in the rho-z half plane."""
    rho: np.ndarray     # [M]
    z: np.ndarray       # [M]
    nrho: np.ndarray    # [M]
    nz: np.ndarray      # [M]
    srho: np.ndarray    # [N]
    sz: np.ndarray      # [N]
    t: np.ndarray       # [M] collocation parameters
    speed: np.ndarray   # [M] s(t)


def collocation_params(body: Body) -> np.ndarray:
    """Collocation parameters.  The paper only fixes M ~ 1.2 N (Sec. 3.3);
    this implementation uses the midpoint rule t_m = pi (m - 1/2)/M, or
    Gauss-Legendre nodes mapped to [0, pi] when asked for."""
    M = body.M
    if body.colloc == "gauss":
        x, _ = np.polynomial.legendre.leggauss(M)
        return math.pi * (x + 1.0) / 2.0
    if body.colloc == "mid":
        return math.pi * (np.arange(1, M + 1) - 0.5) / M
    raise ValueError(body.colloc)


def source_params(N: int) -> np.ndarray:
    """t_j = pi (j - 1/2)/N, j = 1..N (Sec. 3.2)."""
    return math.pi * (np.arange(1, N + 1) - 0.5) / N


def curve_points(sh, t: np.ndarray):
    """rho, z, outward unit normal (n = (-z', rho')/s for this orientation,
    Sec. 3) and speed s at real parameters t."""
    if isinstance(sh, CupShape):
        a = sh.half
        r, th, c = cup_parts(sh, t)
        x = (math.pi - t) - math.pi / 2
        # d/dt = -d/du:  dr/du = -(2/sqrt(pi)) e^{-x^2/a^2},  ds_a/dx = erf(x/a)
        r_t = (2.0 / math.sqrt(math.pi)) * np.exp(-(x / a) ** 2)
        th_t = -2.0 * (1.0 - (sh.b - a) / math.pi) * erf(x / a)
        rho, z = c * r * np.sin(th), c * r * np.cos(th)
        drho = c * (r_t * np.sin(th) + r * np.cos(th) * th_t)
        dz = c * (r_t * np.cos(th) - r * np.sin(th) * th_t)
        s = np.hypot(drho, dz)
        return rho, z, -dz / s, drho / s, s
    r = radius(sh, t)
    rp = radius_dt(sh, t)
    rho = r * np.sin(t)
    z = r * np.cos(t)
    drho = rp * np.sin(t) + r * np.cos(t)
    dz = rp * np.cos(t) - r * np.sin(t)
    s = np.hypot(drho, dz)
    return rho, z, -dz / s, drho / s, s


def build_geometry(body: Body) -> Geometry:
    """Collocation points with outward normals, and sources
    y_j = Z(t_j - i tau) (Sec. 3.2 (c), with the sign of tau chosen so that
    tau > 0 moves sources inside)."""
    sh = body.shape
    t = collocation_params(body)
    rho, z, nrho, nz, s = curve_points(sh, t)
    ts = source_params(body.N)
    Zs = curve_Z(sh, ts - 1j * body.tau)
    return Geometry(rho, z, nrho, nz, Zs.real.copy(), Zs.imag.copy(), t, s)


def surface_points(geom: Geometry, q: int):
    """The q x M surface points (rho_m cos phi_l, rho_m sin phi_l, z_m),
    phi_l = 2 pi l / q, and their unit normals; arrays [q, M, 3]."""
    ph = 2 * math.pi * np.arange(q) / q
    c, s = np.cos(ph)[:, None], np.sin(ph)[:, None]
    X = np.stack([geom.rho[None, :] * c, geom.rho[None, :] * s,
                  np.broadcast_to(geom.z, (q, geom.z.size))], axis=-1)
    Nn = np.stack([geom.nrho[None, :] * c, geom.nrho[None, :] * s,
                   np.broadcast_to(geom.nz, (q, geom.nz.size))], axis=-1)
    return X, Nn


def source_ring_points(geom: Geometry, q: int) -> np.ndarray:
    """Point sources y_j(phi_l), phi_l = 2 pi l / q; array [q, N, 3]."""
    ph = 2 * math.pi * np.arange(q) / q
    c, s = np.cos(ph)[:, None], np.sin(ph)[:, None]
    return np.stack([geom.srho[None, :] * c, geom.srho[None, :] * s,
                     np.broadcast_to(geom.sz, (q, geom.sz.size))], axis=-1)
