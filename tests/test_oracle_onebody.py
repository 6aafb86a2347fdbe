"""Pins of the oracle's one-obstacle part (Sec. 3 of the paper) against
closed forms, invariants, the paper's printed worked example and a textbook
special case.  CPU only."""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import geometry, kernel, mie, onebody

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------- kernel

def test_kernel_symmetric_and_helmholtz():
    """G(x,y) = G(y,x); G solves Delta G + k^2 G = 0 away from y (second
    differences, h = 1e-3, relative residual ~h^2)."""
    k = 7.0
    x = np.array([0.3, -0.2, 0.5]); y = np.array([-0.1, 0.25, 0.05])
    assert abs(kernel.G(k, x, y) - kernel.G(k, y, x)) < 1e-15
    h = 1e-3
    lap = -6 * kernel.G(k, x, y)
    for e in np.eye(3):
        lap += kernel.G(k, x + h * e, y) + kernel.G(k, x - h * e, y)
    lap /= h * h
    assert abs(lap + k * k * kernel.G(k, x, y)) < 1e-5 * abs(k * k * kernel.G(k, x, y))


def test_kernel_gradient_matches_finite_differences():
    k = 9.0
    x = np.array([0.4, 0.1, -0.3]); y = np.array([0.05, -0.2, 0.1])
    n = np.array([0.6, -0.64, 0.48])
    h = 1e-5
    fd = np.array([(kernel.G(k, x + h * e, y) - kernel.G(k, x - h * e, y)) / (2 * h)
                   for e in np.eye(3)])
    g = kernel.grad_x_G(k, x, y)
    assert np.max(np.abs(fd - g)) < 1e-8 * np.max(np.abs(g))
    assert abs(kernel.dG_dnx(k, x, n, y) - fd @ n) < 1e-8 * np.max(np.abs(g))


def test_outgoing_far_field_phase():
    """Along a ray, G(r d, 0) r e^{-ikr} is constant (outgoing, not
    incoming, radiation: eq. (somm))."""
    k = 5.0
    d = np.array([1.0, 2.0, 2.0]) / 3.0
    vals = [kernel.G(k, r * d, np.zeros(3)) * r * np.exp(-1j * k * r) for r in (3.0, 7.5, 20.0)]
    assert np.allclose(vals, 1 / (4 * math.pi), rtol=0, atol=1e-13)


# ----------------------------------------------------------- geometry

def test_sphere_geometry_closed_form():
    """For the sphere, normals are radial and sources Z(t_j - i tau) are a
    concentric shrink by e^{-tau} (0.7 for tau = ln(1/0.7))."""
    b = W.sphere_free_space().body
    g = geometry.build_geometry(b)
    assert np.allclose(g.nrho, g.rho / b.shape.a, atol=1e-14)
    assert np.allclose(g.nz, g.z / b.shape.a, atol=1e-14)
    assert np.allclose(np.hypot(g.srho, g.sz), 0.7 * b.shape.a, atol=1e-14)
    ts = math.pi * (np.arange(b.N) + 0.5) / b.N
    assert np.allclose(np.arctan2(g.srho, g.sz), ts, atol=1e-14)


def test_polar_normals_are_outward_unit_and_orthogonal():
    b = W.periodic_k10(1).body
    g = geometry.build_geometry(b)
    t = g.t
    h = 1e-6
    r1 = geometry.radius(b.shape, t + h); r0 = geometry.radius(b.shape, t - h)
    drho = (r1 * np.sin(t + h) - r0 * np.sin(t - h)) / (2 * h)
    dz = (r1 * np.cos(t + h) - r0 * np.cos(t - h)) / (2 * h)
    assert np.max(np.abs(g.nrho * drho + g.nz * dz)) < 1e-8
    assert np.allclose(np.hypot(g.nrho, g.nz), 1.0, atol=1e-14)
    assert np.all(g.nrho * g.rho + g.nz * g.z > 0)            # star-shaped: outward
    rs = np.hypot(g.srho, g.sz)
    th = np.arctan2(g.srho, g.sz)
    assert np.all(rs < b.shape.radius(th))                     # sources inside


# --------------------------------------------------------- modal fill

def _tiny_body(P=8, q=8):
    return W.Body(W.Shape(0.5, 0.15, 2), N=4, M=6, P=P, q=q, k=3.0, tau=0.3, colloc="mid")


def test_block_circulant_equivalence():
    """The un-FFT'd point matrix K between the P x M surface points and the
    P x N point sources satisfies (F (x) I) K (F^* (x) I) / P^2 =
    blockdiag(A'_n) with F[n, l] = e^{-2 pi i n l / P} (q = P)."""
    b = _tiny_body()
    g = geometry.build_geometry(b)
    P, M, N = b.P, b.M, b.N
    K = onebody.point_matrix_dGdn(b, g, P)
    F = np.exp(-2j * math.pi * np.outer(np.arange(P), np.arange(P)) / P)
    FI = np.kron(F, np.eye(M)); FJ = np.kron(F, np.eye(N))
    D = FI @ K @ FJ.conj().T / P ** 2
    A = onebody.modal_blocks(b, g, q=P)
    ref = np.zeros_like(D)
    for n in range(P):
        ref[n * M:(n + 1) * M, n * N:(n + 1) * N] = A[n]
    assert np.max(np.abs(D - ref)) < 1e-14 * np.max(np.abs(ref))


def test_modes_even_in_n():
    """A'_n = A'_{-n}: the integrand depends on the angle only via cos."""
    b = W.with_(_tiny_body(), P=12, q=40)
    g = geometry.build_geometry(b)
    A = onebody.modal_blocks(b, g)
    for n in range(1, b.P // 2):
        assert np.max(np.abs(A[n] - A[b.P - n])) < 1e-15 * np.max(np.abs(A))


def _ptr_value(k, tgt, src, q, n):
    """q-node trapezoid rule of eq. (ptr) for one element of A_n."""
    ph = 2 * math.pi * np.arange(q) / q
    x = np.array([tgt[0], 0.0, tgt[1]])
    y = np.stack([src[0] * np.cos(ph), src[0] * np.sin(ph), np.full(q, src[1])], 1)
    return np.mean(kernel.G(k, x, y) * np.exp(-1j * n * ph))


@pytest.mark.parametrize("tgt,rate", [((0.5, 0.49), 0.1489), ((0.6, 0.2), 0.5382)])
def test_theorem1_rate_on_paper_points(tgt, rate):
    """Fig. qconv / Thm. 1: k = 10, source (0.45, 0.44).  The trapezoid
    error decays like exp(-alpha q) with alpha = Im acos(1 + d^2/(2 rho rho')),
    0.1489 for the close target and 0.5382 for the far one.  The fitted
    slope of log(error) in q must agree to 10%."""
    k, src = 10.0, (0.45, 0.44)
    d2 = (tgt[0] - src[0]) ** 2 + (tgt[1] - src[1]) ** 2
    alpha = math.acosh(1 + d2 / (2 * tgt[0] * src[0]))
    assert abs(alpha - rate) < 1e-4
    for n in (0, 5):
        ref = _ptr_value(k, tgt, src, 2000, n)
        qs = np.arange(40, 160, 8) if rate < 0.3 else np.arange(16, 48, 4)
        err = np.array([abs(_ptr_value(k, tgt, src, int(q), n) - ref) for q in qs])
        slope = -np.polyfit(qs, np.log(err), 1)[0]
        assert abs(slope - alpha) < 0.1 * alpha, (n, slope, alpha)


def test_fill_converged_in_q_for_periodic_k10():
    """Sec. 3.1: the fixed q of the k = 10 periodic body converges the fill
    (doubling q changes entries by < 1e-12 absolute), checked on a sample
    of rows."""
    b = W.periodic_k10(1).body
    g = geometry.build_geometry(b)
    rows = np.array([0, 37, 119, 200, 239])
    a1 = onebody.ring_samples_dGdn(b, g, b.q, rows)
    a2 = onebody.ring_samples_dGdn(b, g, 2 * b.q, rows)
    bins = np.mod(onebody.mode_numbers(b.P), b.q)
    bins2 = np.mod(onebody.mode_numbers(b.P), 2 * b.q)
    f1 = (np.fft.fft(a1, axis=2) / b.q)[:, :, bins]
    f2 = (np.fft.fft(a2, axis=2) / (2 * b.q))[:, :, bins2]
    assert np.max(np.abs(f1 - f2)) < 1e-12


# ------------------------------------------------------- least squares

def test_pinv_solve_equals_normal_equations_and_lstsq():
    """Well-conditioned block (sources at half the radius, k = 1): truncated
    SVD = normal equations = LAPACK least squares."""
    b = W.Body(W.Shape(0.5), N=8, M=10, P=4, q=32, k=1.0, tau=math.log(2.0), colloc="mid")
    g = geometry.build_geometry(b)
    A = onebody.modal_blocks(b, g)
    rng = np.random.default_rng(5)
    f = rng.standard_normal(b.M) + 1j * rng.standard_normal(b.M)
    for n in range(b.P):
        An = A[n]
        x1 = onebody.pinv_solve(An, f)
        x2 = np.linalg.solve(An.conj().T @ An, An.conj().T @ f)
        x3, *_ = np.linalg.lstsq(An, f, rcond=None)
        assert np.linalg.norm(x1 - x3) < 1e-12 * np.linalg.norm(x3)
        assert np.linalg.norm(x1 - x2) < 1e-9 * np.linalg.norm(x3)


def test_modal_lsq_equals_dense_point_lsq():
    """The unitary DFT preserves the 2-norm, so the per-mode least squares
    equals dense least squares on the un-FFT'd matrix K (q = P), whose
    solution is the point-strength vector sigma of eq. (ptr)'s point form."""
    b = W.Body(W.Shape(0.5, 0.1, 2), N=6, M=9, P=6, q=6, k=2.0, tau=0.5, colloc="mid")
    g = geometry.build_geometry(b)
    A = onebody.modal_blocks(b, g)
    w = W.Wave(0.7, 1.1)
    fh = onebody.rhs_modes(b, g, w)
    c = np.stack([np.linalg.lstsq(A[n], fh[n], rcond=None)[0] for n in range(b.P)])
    K = onebody.point_matrix_dGdn(b, g, b.P)
    X, Nn = geometry.surface_points(g, b.P)
    kv = W.wave_vector(b.k, w)
    f = (-1j * (Nn @ kv) * np.exp(1j * (X @ kv))).reshape(-1)
    sig, *_ = np.linalg.lstsq(K, f, rcond=None)
    assert np.linalg.norm(sig - onebody.point_strengths(c, b.P).reshape(-1)) < 1e-10 * np.linalg.norm(sig)


def test_rhs_modes_of_axial_incidence():
    """For incidence along -z the data is axisymmetric: only mode 0 is
    non-zero, and it equals the ring value itself."""
    b = W.periodic_k10(1).body
    g = geometry.build_geometry(b)
    fh = onebody.rhs_modes(b, g, W.Wave(0.0, 0.3))
    ref = -1j * (-b.k * g.nz) * np.exp(-1j * b.k * g.z)
    assert np.max(np.abs(fh[0] - ref)) < 1e-13 * b.k
    assert np.max(np.abs(fh[1:])) < 1e-13 * b.k


# ------------------------------------------------------------------ Mie

def test_sphere_matches_mie_series():
    """Sound-hard sphere a = 0.5, k = 2 pi, 60 Gauss collocation nodes, 40
    sources at 0.7 a, P = 32, q = 128, oblique random incidence: the
    scattered field at 64 points on |x| = 2 agrees with the Mie series to
    better than 1e-9 relative, and the boundary error eps_1 < 1e-7."""
    pr = W.sphere_free_space()
    b = pr.body
    g = geometry.build_geometry(b)
    A = onebody.modal_blocks(b, g)
    fh = onebody.rhs_modes(b, g, pr.waves[0])
    c = onebody.solve_modes(A, fh)
    u = onebody.field(b, g, c, pr.targets, pr.q_field)
    um = mie.sound_hard_sphere(b.k, b.shape.a, W.wave_vector(b.k, pr.waves[0]), pr.targets)
    assert np.linalg.norm(u - um) / np.linalg.norm(um) < 1e-9
    assert onebody.bc_residual(b, g, c, pr.waves[0], 24, 24, b.q) < 1e-7


def test_mie_sign_convention_pins_point_form():
    """Flipping the sign of the mode exponent in the point-source form (a
    plausible mistake) breaks agreement with Mie at oblique incidence."""
    pr = W.sphere_free_space()
    b = pr.body
    g = geometry.build_geometry(b)
    A = onebody.modal_blocks(b, g)
    fh = onebody.rhs_modes(b, g, pr.waves[0])
    c = onebody.solve_modes(A, fh)
    cflip = c[np.mod(-onebody.mode_numbers(b.P), b.P)]     # c_n -> c_{-n}
    u = onebody.field(b, g, cflip, pr.targets, pr.q_field)
    um = mie.sound_hard_sphere(b.k, b.shape.a, W.wave_vector(b.k, pr.waves[0]), pr.targets)
    assert np.linalg.norm(u - um) / np.linalg.norm(um) > 1e-2


def test_mie_series_self_consistency():
    """The Mie field plus the incident wave has zero radial derivative on
    r = a (central differences)."""
    k, a = 4.0, 0.7
    d = np.array([0.3, -0.4, -np.sqrt(0.75)])
    pts = W.fibonacci_sphere(12, 1.0)
    h = 1e-5
    up = mie.sound_hard_sphere(k, a, d, pts * (a + h)) + np.exp(1j * k * (pts * (a + h)) @ d)
    um = mie.sound_hard_sphere(k, a, d, pts * (a - h)) + np.exp(1j * k * (pts * (a - h)) @ d)
    assert np.max(np.abs(up - um) / (2 * h)) < 1e-6 * k
