"""Transmission problem (eqs. (helmi)-(neup1.4), Sec. 3.4 and the end of
Sec. 4.1 of the paper), plainly.  Test infrastructure only: the tests, the
smoke check and the benchmark's CPU baseline call it; the product never
does.

The scattered field outside is the ring-source sum of Sec. 3 at wavenumber
k with sources inside the body (Z(t_j - i tau)); the field u^- inside is a
second ring-source sum at the interior wavenumber km with sources outside
(tau negated, Sec. 3.4).  Matching u - u^- = -u^i and du/dn - du^-/dn =
-du^i/dn mode by mode gives eq. (trans):
    [ A_n   -A^-_n  ] [eta_n  ]   [f_n ]
    [ A'_n  -A'^-_n ] [eta^-_n] = [f'_n],   f = -u^i,  f' = -du^i/dn,
A_n, A'_n the value and normal-derivative ring kernels (eqs. (ringkernel),
(ringkernelderiv)) by the trapezoid rule eq. (ptr).  Each per-mode block is
2M x 2N: rows [values; normal derivatives], columns [exterior; interior]
coefficients.

Periodic (end of Sec. 4.1): A_else acts on the exterior coefficients only
and gives both the value and the normal derivative of the eight phased
images at the surface nodes; B~ likewise holds the harmonics' values and
normal derivatives; C and Q are those of the Neumann case, C acting on the
exterior coefficients.  The interior field involves A_0 only.
"""
from __future__ import annotations

from dataclasses import replace

import numpy as np

from workloads import Body, Lattice, Wave, wave_vector
from . import kernel
from .geometry import Geometry, build_geometry, source_ring_points, surface_points
from .gmres import gmres
from .onebody import (ModalPinv, field_from_points, mode_numbers, point_strengths, ring_samples_dGdn,
                      ring_samples_G)
from .periodic import ELSE8, PeriodicSolver, harmonics, image_list


def geometries(body: Body):
    """Collocation points with the interior sources (exterior field) and
    with the exterior sources (interior field): the latter negate tau."""
    return build_geometry(body), build_geometry(replace(body, tau=-body.tau))


def _modes(samples: np.ndarray, P: int, q: int) -> np.ndarray:
    """[M, N, q] trapezoid samples -> [P, M, N] in FFT bin order (eq. (ptr))."""
    bins = np.mod(mode_numbers(P), q)
    return np.transpose((np.fft.fft(samples, axis=2) / q)[:, :, bins], (2, 0, 1))


def transmission_blocks(body: Body, km: float, g_in: Geometry, g_out: Geometry) -> np.ndarray:
    """Per-mode blocks of eq. (trans), [P, 2M, 2N]."""
    P, q, M, N = body.P, body.q, body.M, body.N
    A = _modes(ring_samples_G(body, g_in, q), P, q)
    Ad = _modes(ring_samples_dGdn(body, g_in, q), P, q)
    bm = replace(body, k=km)
    Am = _modes(ring_samples_G(bm, g_out, q), P, q)
    Amd = _modes(ring_samples_dGdn(bm, g_out, q), P, q)
    out = np.empty((P, 2 * M, 2 * N), dtype=np.complex128)
    out[:, :M, :N] = A
    out[:, :M, N:] = -Am
    out[:, M:, :N] = Ad
    out[:, M:, N:] = -Amd
    return out


def rhs_modes(body: Body, geom: Geometry, w: Wave) -> np.ndarray:
    """[f_hat; f_hat'] with f = -u^i and f' = -du^i/dn at the P x M surface
    points, each by eq. (fhatquad) (q = P).  Returns [P, 2M]."""
    kv = wave_vector(body.k, w)
    X, Nn = surface_points(geom, body.P)
    ui = np.exp(1j * (X @ kv))
    f = np.concatenate([-ui, -1j * (Nn @ kv) * ui], axis=1)     # [P, 2M]
    return np.fft.fft(f, axis=0) / body.P


def exterior_field(body: Body, g_in: Geometry, c: np.ndarray, X: np.ndarray, qs: int) -> np.ndarray:
    """Scattered field outside from the exterior coefficients c[:, :N]."""
    N = body.N
    return field_from_points(body.k, source_ring_points(g_in, qs), point_strengths(c[:, :N], qs), X)


def interior_field(body: Body, km: float, g_out: Geometry, c: np.ndarray, X: np.ndarray,
                   qs: int) -> np.ndarray:
    """Field u^- inside from the interior coefficients c[:, N:] at km."""
    N = body.N
    return field_from_points(km, source_ring_points(g_out, qs), point_strengths(c[:, N:], qs), X)


class TransmissionPeriodicSolver(PeriodicSolver):
    """eq. (iter) for the transmission case: unknowns eta~ in C^{2MP}
    (values then normal derivatives per mode), A_0 the blocks of eq. (trans)."""

    def __init__(self, body: Body, km: float, lat: Lattice, g_in: Geometry, g_out: Geometry,
                 A2: np.ndarray, rel_cutoff: float = 1e-10):
        self.km, self.g_out = km, g_out
        super().__init__(body, lat, g_in, A2, ModalPinv(A2, rel_cutoff), rel_cutoff)

    def btilde(self) -> np.ndarray:
        """B~[n, r, lm]: the harmonics' values (r < M) and normal derivatives
        (r >= M) on the surface rings, FFT / P.  [P, 2M, NH]."""
        P, M = self.P, self.body.M
        H, grad = harmonics(self.k, self.lat.p, self.Xs.reshape(-1, 3))
        dn = np.einsum("tic,tc->ti", grad, self.Ns.reshape(-1, 3))
        both = np.concatenate([H.reshape(P, M, -1), dn.reshape(P, M, -1)], axis=1)
        return np.fft.fft(both, axis=0) / P

    def aelse_point_matrix(self) -> np.ndarray:
        """K_else[(l', r), (l, j)]: the 8 phased images of the exterior point
        sources, value at surface node m (r = m) and normal derivative
        (r = M + m), q = P."""
        P, M = self.P, self.body.M
        X = self.Xs.reshape(-1, 3); Nn = self.Ns.reshape(-1, 3)
        Y = self.Ysrc.reshape(-1, 3)
        V = np.zeros((X.shape[0], Y.shape[0]), dtype=np.complex128)
        D = np.zeros_like(V)
        for (a, b), wgt, shift in image_list(self.lat, self.alpha, self.beta, ELSE8):
            for t0 in range(0, X.shape[0], 512):
                sl = slice(t0, t0 + 512)
                V[sl] += wgt * kernel.G(self.k, X[sl, None, :], Y[None, :, :] + shift)
                D[sl] += wgt * kernel.dG_dnx(self.k, X[sl, None, :], Nn[sl, None, :], Y[None, :, :] + shift)
        S = Y.shape[0]
        return np.concatenate([V.reshape(P, M, S), D.reshape(P, M, S)], axis=1).reshape(2 * P * M, S)

    def apply_aelse(self, c: np.ndarray) -> np.ndarray:
        N = self.body.N
        sig = point_strengths(c[:, :N], self.P).reshape(-1)
        g = (self.Kelse @ sig).reshape(self.P, 2 * self.body.M)
        return np.fft.fft(g, axis=0) / self.P

    def apply_c(self, c: np.ndarray) -> np.ndarray:
        N = self.body.N
        return self.Cpt @ point_strengths(c[:, :N], self.P).reshape(-1)

    def op(self, eta_t: np.ndarray) -> np.ndarray:
        P, M2 = self.P, 2 * self.body.M
        x = eta_t.reshape(P, M2)
        c = self.pinv.apply(x)
        out = x + self.apply_aelse(c) - self.apply_b(self.apply_qpinv(self.apply_c(c)))
        return out.reshape(-1)

    def solve(self, fh: np.ndarray, tol: float = 1e-12, maxit: int = 200):
        x, its, hist = gmres(self.op, fh.reshape(-1), tol, maxit)
        c = self.pinv.apply(x.reshape(self.P, 2 * self.body.M))
        xi = -self.apply_qpinv(self.apply_c(c))
        NH = (self.lat.p + 1) ** 2
        nrb = self.orders.m.size
        return dict(c=c, xi=xi, d=xi[:NH], a=xi[NH:NH + nrb], b=xi[NH + nrb:],
                    iters=its, hist=hist)

    def field_and_grad(self, c, d, X, qs, want_grad=True):
        """Exterior field in the cell (exterior coefficients and harmonics)."""
        return super().field_and_grad(c[:, :self.body.N], d, X, qs, want_grad)

    def interior(self, c: np.ndarray, X: np.ndarray, qs: int) -> np.ndarray:
        return interior_field(self.body, self.km, self.g_out, c, X, qs)
