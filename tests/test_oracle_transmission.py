"""Pins of the oracle's transmission problem (eqs. (helmi)-(neup1.4),
Sec. 3.4 and the end of Sec. 4.1): the penetrable-sphere Mie series checked
against its own interface conditions and the no-contrast case, the
free-space solve against that series outside and inside the sphere, and the
periodic solve against energy-flux balance, quasi-periodicity and the
transmission conditions at surface points that are not collocation points.
CPU only."""
import math

import numpy as np

import workloads as W
from oracle import geometry, kernel, mie, onebody, transmission as T


def _total(k, km, a, d, X):
    """Total field: u^i + u outside, u^- inside."""
    r = np.linalg.norm(X, axis=1)
    u = mie.penetrable_sphere(k, km, a, d, X)
    return np.where(r < a, u, u + np.exp(1j * k * (X @ d)))


def test_mie_penetrable_interface_conditions():
    """The total field and its radial derivative are continuous at r = a:
    the one-sided jumps at distance h, extrapolated to h = 0 (Richardson),
    vanish to the extrapolation error, while a wrong coefficient leaves an
    O(1) jump."""
    k, km, a = 2 * math.pi, 3 * math.pi, 0.5
    d = np.array([0.3, -0.4, 0.866]); d /= np.linalg.norm(d)
    rng = np.random.default_rng(3)
    e = rng.standard_normal((12, 3)); e /= np.linalg.norm(e, axis=1, keepdims=True)
    scale = np.max(np.abs(_total(k, km, a, d, e * (a + 1e-6))))

    def jump(h):
        return _total(k, km, a, d, e * (a + h)) - _total(k, km, a, d, e * (a - h))

    def djump(h):
        out = (_total(k, km, a, d, e * (a + 2 * h)) - _total(k, km, a, d, e * (a + h))) / h
        inn = (_total(k, km, a, d, e * (a - h)) - _total(k, km, a, d, e * (a - 2 * h))) / h
        return out - inn

    # the extrapolation error is O(h^2): 1.2e-9 and 3.7e-9 (relative) at h = 1e-5
    h = 1e-5
    assert np.max(np.abs(2 * jump(h / 2) - jump(h))) < 1e-8 * scale
    assert np.max(np.abs(2 * djump(h / 2) - djump(h))) < 3e-8 * k * scale


def test_mie_penetrable_without_contrast():
    """km = k: nothing scatters; u = 0 outside and u^- = u^i inside."""
    k = 5.0
    d = np.array([0.0, 0.6, -0.8])
    X = W.fibonacci_sphere(10, 0.3)
    assert np.max(np.abs(mie.penetrable_sphere(k, k, 0.5, d, X) - np.exp(1j * k * (X @ d)))) < 1e-13
    assert np.max(np.abs(mie.penetrable_sphere(k, k, 0.5, d, W.fibonacci_sphere(10, 0.9)))) < 1e-14


def test_transmission_sphere_matches_mie():
    pr = W.sphere_transmission()
    b = pr.body
    gi, go = T.geometries(b)
    A2 = T.transmission_blocks(b, pr.km, gi, go)
    w = pr.waves[0]
    c = onebody.solve_modes(A2, T.rhs_modes(b, gi, w))
    kv = W.wave_vector(b.k, w)
    uo = T.exterior_field(b, gi, c, pr.targets, pr.q_field)
    ui = T.interior_field(b, pr.km, go, c, pr.inner, pr.q_field)
    mo = mie.penetrable_sphere(b.k, pr.km, b.shape.a, kv, pr.targets)
    mi = mie.penetrable_sphere(b.k, pr.km, b.shape.a, kv, pr.inner)
    eo = np.linalg.norm(uo - mo) / np.linalg.norm(mo)
    ei = np.linalg.norm(ui - mi) / np.linalg.norm(mi)
    assert eo < 1e-10 and ei < 1e-10, (eo, ei)
    # the exterior sources of the interior field lie outside the sphere
    assert np.min(np.hypot(go.srho, go.sz)) > b.shape.a


def test_periodic_transmission_invariants():
    """Small periodic transmission solve: flux balance and quasi-periodicity
    (real k and km), and the two transmission conditions at 12 x 16 surface
    points between the collocation nodes, u^i + u - u^- and
    d(u^i + u - u^-)/dn, with u the full periodized exterior field (1.6e-6
    and 5.2e-6 at this coarse discretisation; a wrong sign or a dropped
    block leaves them of order one)."""
    pr = W.small_periodic_transmission(1)
    b, lat = pr.body, pr.lattice
    gi, go = T.geometries(b)
    A2 = T.transmission_blocks(b, pr.km, gi, go)
    ps = T.TransmissionPeriodicSolver(b, pr.km, lat, gi, go, A2)
    w = pr.waves[0]
    ps.set_wave(w)
    r = ps.solve(T.rhs_modes(b, gi, w), tol=1e-12)
    assert ps.eps_flux(r["a"], r["b"]) < 1e-6
    assert ps.eps_per(r["c"], r["d"], 2 * b.P) < 1e-6
    nt, nphi = 12, 16
    t = math.pi * (np.arange(nt) + 0.5) / nt
    rho, z, nrho, nz, _ = geometry.curve_points(b.shape, t)
    ph = 2 * math.pi * (np.arange(nphi) + 0.5) / nphi
    cph, sph = np.cos(ph)[:, None], np.sin(ph)[:, None]
    X = np.stack([rho[None] * cph, rho[None] * sph, np.broadcast_to(z, (nphi, nt))], -1).reshape(-1, 3)
    Nn = np.stack([nrho[None] * cph, nrho[None] * sph, np.broadcast_to(nz, (nphi, nt))], -1).reshape(-1, 3)
    u, g = ps.field_and_grad(r["c"], r["d"], X, b.q)
    Y = geometry.source_ring_points(go, b.q).reshape(-1, 3)
    sig = onebody.point_strengths(r["c"][:, b.N:], b.q).reshape(-1)
    um = kernel.G(pr.km, X[:, None, :], Y[None]) @ sig
    dum = kernel.dG_dnx(pr.km, X[:, None, :], Nn[:, None, :], Y[None]) @ sig
    kv = W.wave_vector(b.k, w)
    ui = np.exp(1j * (X @ kv))
    dui = 1j * (Nn @ kv) * ui
    e0 = np.sqrt(np.mean(np.abs(ui + u - um) ** 2))
    e1 = np.sqrt(np.mean(np.abs(dui + np.sum(g * Nn, 1) - dum) ** 2)) / b.k
    assert e0 < 1e-4 and e1 < 1e-4, (e0, e1)
