"""Pins of the oracle's cup body (Fig. 1(c) of the paper) and of a one-body
sound-hard cup solve: closed-form values of the parametrisation at the rim
and the poles, normals against finite differences and a point-in-polygon
test, complexified sources inside the body, and far-field reciprocity
u_inf(x; d) = u_inf(-d; -x) of the scattering solution (a property of the
exact solution for any sound-hard body).  CPU only."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import geometry, onebody

SH = W.CupShape(outer=0.35, half=0.2, b=math.pi / 6)


def outline(sh, n=20001):
    """Closed polygon of the generating curve (the axis closes it)."""
    Z = geometry.curve_Z(sh, np.linspace(0.0, math.pi, n))
    return Z.real, Z.imag


def inside(poly, px, py):
    """Even-odd ray casting in the +rho direction."""
    x, y = poly
    x2, y2 = np.roll(x, -1), np.roll(y, -1)
    c = np.zeros(np.shape(px), dtype=bool)
    for i in range(len(x)):
        cross = (y[i] > py) != (y2[i] > py)
        with np.errstate(divide="ignore", invalid="ignore"):
            xi = x[i] + (py - y[i]) * (x2[i] - x[i]) / (y2[i] - y[i])
        c ^= cross & (px < xi)
    return c


def test_cup_closed_form_points():
    """At t = pi/2 (the rim, x = 0): r = 1 and theta = b - a + 2 (1 - (b-a)/pi) a/sqrt(pi);
    t = 0 is the inner bottom pole (0, -c (1 - a)), t = pi the outer bottom
    pole (0, -c (1 + a)), c = outer/(1 + a)."""
    a, b = SH.half, SH.b
    c = SH.outer / (1 + a)
    th = b - a + 2 * (1 - (b - a) / math.pi) * a / math.sqrt(math.pi)
    Z = geometry.curve_Z(SH, np.array([0.0, math.pi / 2, math.pi]))
    assert abs(Z[1] - c * (math.sin(th) + 1j * math.cos(th))) < 1e-15
    assert abs(Z[0] - (-1j * c * (1 - a))) < 1e-15
    assert abs(Z[2] - (-1j * c * (1 + a))) < 1e-15
    # the enclosing radius is `outer`, reached at the outer pole only
    zz = geometry.curve_Z(SH, np.linspace(0, math.pi, 4001))
    assert np.max(np.abs(zz)) <= SH.outer * (1 + 1e-15)


def test_cup_normals_unit_outward_and_match_finite_differences():
    b = W.Body(SH, N=60, M=400, P=8, q=16, k=1.0, tau=0.05)
    t = geometry.collocation_params(b)
    rho, z, nrho, nz, s = geometry.curve_points(SH, t)
    assert np.max(np.abs(np.hypot(nrho, nz) - 1)) < 1e-14
    h = 1e-6
    Zp = (geometry.curve_Z(SH, t + h) - geometry.curve_Z(SH, t - h)) / (2 * h)
    assert np.max(np.abs(-Zp.imag / np.abs(Zp) - nrho)) < 1e-8
    assert np.max(np.abs(Zp.real / np.abs(Zp) - nz)) < 1e-8
    assert np.max(np.abs(np.abs(Zp) - s) / s) < 1e-8
    poly = outline(SH)
    d = 2e-3
    assert not inside(poly, rho + d * nrho, z + d * nz).any(), "a normal points into the body"
    assert inside(poly, rho - d * nrho, z - d * nz).all(), "a normal points out of the wrong side"


@pytest.mark.parametrize("N,tau", [(60, 0.05), (450, 0.05), (200, 0.1)])
def test_cup_sources_inside(N, tau):
    b = W.Body(SH, N=N, M=N + N // 5, P=8, q=16, k=1.0, tau=tau)
    g = geometry.build_geometry(b)
    assert (g.srho > 0).all()
    assert inside(outline(SH), g.srho, g.sz).all()


def far_field(body, geom, c, xhat):
    """u_inf(xhat) = (1/4 pi) sum_{j,l} sigma_jl e^{-i k xhat . y_jl}: the
    far-field pattern of the point-source form of the rings."""
    qs = 2 * body.P
    Y = geometry.source_ring_points(geom, qs).reshape(-1, 3)
    sig = onebody.point_strengths(c, qs).reshape(-1)
    return np.exp(-1j * body.k * (xhat @ Y.T)) @ sig / (4 * math.pi)


def wave_from(d):
    """Incidence along unit vector d in the convention d = (sin th cos ph, sin th sin ph, -cos th)."""
    return W.Wave(math.acos(-d[2]), math.atan2(d[1], d[0]))


def test_cup_far_field_reciprocity():
    """Sources 0.02-0.06 from the surface need q = 320 for the ring fill
    (Theorem 1: the smallest rate over the (collocation, source) pairs is
    0.122, and q >= P/2 + 37/0.122); the boundary residual is then ~5e-7."""
    b = W.Body(SH, N=120, M=144, P=32, q=320, k=6.0, tau=0.1)
    g = geometry.build_geometry(b)
    A = onebody.modal_blocks(b, g)
    pinv = onebody.ModalPinv(A)
    rng = np.random.default_rng(11)
    dirs = rng.standard_normal((4, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    sol = {}
    for i, d in enumerate(list(dirs) + list(-dirs)):
        w = wave_from(d)
        c = pinv.apply(onebody.rhs_modes(b, g, w))
        sol[i] = c
        if i == 0:
            eps1 = onebody.bc_residual(b, g, c, w, 37, 29, b.q)
            assert eps1 < 2e-6, f"boundary residual {eps1:.2e}: discretisation too coarse for the pin"
    n = len(dirs)
    worst, scale = 0.0, 0.0
    for i in range(n):
        for j in range(n):
            u1 = far_field(b, g, sol[i], dirs[j][None])[0]          # u_inf(d_j; d_i)
            u2 = far_field(b, g, sol[n + j], -dirs[i][None])[0]     # u_inf(-d_i; -d_j)
            worst = max(worst, abs(u1 - u2))
            scale = max(scale, abs(u1))
    assert worst < 1e-5 * scale, (worst, scale)
