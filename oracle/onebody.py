"""One-obstacle axisymmetric MFS (Sec. 3 of the paper), plainly.

Mode convention.  A mode-n coefficient c_nj multiplies the field
e^{+i n phi} A_n(rho, z; rho'_j, z'_j) (the ring kernel is even in the
angle, so A_n = A_{-n} and the block matrices do not depend on this sign;
it matters for the point-source form below).  Arrays over modes are stored
in FFT bin order: bin b holds mode n = b for b <= P/2 and n = b - P above.
"""
from __future__ import annotations

import math

import numpy as np

from workloads import Body, wave_vector, Wave
from . import kernel
from .geometry import Geometry, source_ring_points, surface_points


def mode_numbers(P: int) -> np.ndarray:
    """Mode n held in each FFT bin, n = -P/2+1..P/2 (Sec. 3, after eq. (fhat))."""
    b = np.arange(P)
    return np.where(b <= P // 2, b, b - P)


def ring_samples_dGdn(body: Body, geom: Geometry, q: int, m_index=None) -> np.ndarray:
    """g[m, j, l] = dG/dn_x((rho_m, 0, z_m); y_j(2 pi l / q)) for l = 0..q-1:
    the integrand of eq. (ringkernelderiv) at the trapezoid nodes."""
    mi = np.arange(body.M) if m_index is None else np.asarray(m_index)
    x = np.stack([geom.rho[mi], np.zeros(mi.size), geom.z[mi]], axis=-1)[:, None, None, :]
    nx = np.stack([geom.nrho[mi], np.zeros(mi.size), geom.nz[mi]], axis=-1)[:, None, None, :]
    y = np.transpose(source_ring_points(geom, q), (1, 0, 2))[None, :, :, :]   # [1, N, q, 3]
    return kernel.dG_dnx(body.k, x, nx, y)


def ring_samples_G(body: Body, geom: Geometry, q: int) -> np.ndarray:
    """Value kernel samples for eq. (ringkernel): G((rho_m,0,z_m); y_j(phi_l))."""
    x = np.stack([geom.rho, np.zeros(body.M), geom.z], axis=-1)[:, None, None, :]
    y = np.transpose(source_ring_points(geom, q), (1, 0, 2))[None, :, :, :]
    return kernel.G(body.k, x, y)


def modal_blocks(body: Body, geom: Geometry, q: int | None = None, chunk: int = 16) -> np.ndarray:
    """A'_n[m, j] = (1/q) sum_l dG/dn_x(x_m; y_j(phi_l)) e^{-i n phi_l}
    for the P modes (eq. (ptr) applied to eq. (ringkernelderiv)), computed as
    one length-q FFT per (m, j).  Returns [P, M, N] complex128, FFT bin order."""
    q = body.q if q is None else q
    P = body.P
    out = np.empty((P, body.M, body.N), dtype=np.complex128)
    bins = np.mod(mode_numbers(P), q)
    for m0 in range(0, body.M, chunk):
        mi = np.arange(m0, min(body.M, m0 + chunk))
        g = ring_samples_dGdn(body, geom, q, mi)            # [mc, N, q]
        gh = np.fft.fft(g, axis=2) / q
        out[:, mi, :] = np.transpose(gh[:, :, bins], (2, 0, 1))
    return out


def rhs_modes(body: Body, geom: Geometry, w: Wave) -> np.ndarray:
    """f = -du^i/dn at the P x M surface points (eq. (neu) with eq. (ui)),
    then f_hat_n = (1/P) sum_l f(phi_l) e^{-i n phi_l} (eq. (fhatquad), q = P).
    Returns [P, M] in FFT bin order."""
    kv = wave_vector(body.k, w)
    X, Nn = surface_points(geom, body.P)
    f = -1j * (Nn @ kv) * np.exp(1j * (X @ kv))          # [P, M]
    return np.fft.fft(f, axis=0) / body.P


def pinv_solve(A: np.ndarray, f: np.ndarray, rel_cutoff: float = 1e-10) -> np.ndarray:
    """Backward-stable truncated pseudo-inverse applied as V S^+ (U^* f), with
    singular values below rel_cutoff * s_max dropped (Sec. 4.2, practical
    word on pseudoinverses).  f may hold several right-hand sides as columns."""
    U, s, Vh = np.linalg.svd(A, full_matrices=False)
    keep = s > rel_cutoff * s[0]
    y = (U[:, keep].conj().T @ f)
    y = y / (s[keep][:, None] if y.ndim == 2 else s[keep])
    return Vh[keep].conj().T @ y


class ModalPinv:
    """Per-mode SVDs of the P blocks A'_n, kept to apply A_0^+ repeatedly."""

    def __init__(self, A: np.ndarray, rel_cutoff: float = 1e-10):
        self.fac = []
        self.rank = []
        for n in range(A.shape[0]):
            U, s, Vh = np.linalg.svd(A[n], full_matrices=False)
            keep = s > rel_cutoff * s[0]
            self.fac.append((U[:, keep], s[keep], Vh[keep]))
            self.rank.append(int(keep.sum()))

    def apply(self, x: np.ndarray) -> np.ndarray:
        """x [P, M] -> c [P, N], c_n = V_n S_n^+ (U_n^* x_n)."""
        out = []
        for n, (U, s, Vh) in enumerate(self.fac):
            out.append(Vh.conj().T @ ((U.conj().T @ x[n]) / s))
        return np.stack(out)


def solve_modes(A: np.ndarray, fh: np.ndarray, rel_cutoff: float = 1e-10) -> np.ndarray:
    """Solve eq. (linsys) mode by mode: c_n = A'_n^+ f_hat_n.  [P, N]."""
    return np.stack([pinv_solve(A[n], fh[n], rel_cutoff) for n in range(A.shape[0])])


def point_strengths(c: np.ndarray, qs: int) -> np.ndarray:
    """Point-source form of the ring sources: the trapezoid rule replaces
    each ring by qs point sources (Sec. 4.1, description of A_else) with
    sigma_jl = (1/qs) sum_n c_nj e^{+i n phi_l}.  c [P, N] -> sigma [qs, N]."""
    P = c.shape[0]
    assert qs >= P
    full = np.zeros((qs, c.shape[1]), dtype=np.complex128)
    full[np.mod(mode_numbers(P), qs)] = c
    return np.fft.ifft(full, axis=0)


def field_from_points(k: float, Y: np.ndarray, sigma: np.ndarray, X: np.ndarray,
                      chunk: int = 256) -> np.ndarray:
    """u(x) = sum_{j,l} G_k(x, y_jl) sigma_jl at targets X [T, 3].
    Y is [qs, N, 3], sigma [qs, N]."""
    Yf = Y.reshape(-1, 3)
    sf = sigma.reshape(-1)
    out = np.empty(X.shape[0], dtype=np.complex128)
    for t0 in range(0, X.shape[0], chunk):
        Xc = X[t0:t0 + chunk]
        out[t0:t0 + chunk] = kernel.G(k, Xc[:, None, :], Yf[None, :, :]) @ sf
    return out


def field(body: Body, geom: Geometry, c: np.ndarray, X: np.ndarray, qs: int) -> np.ndarray:
    """Scattered field of eq. (ubormfs) at free-space targets X, each ring
    kernel evaluated by the qs-node trapezoid rule."""
    Y = source_ring_points(geom, qs)
    return field_from_points(body.k, Y, point_strengths(c, qs), X)


def point_matrix_dGdn(body: Body, geom: Geometry, P: int) -> np.ndarray:
    """Dense un-FFT'd matrix K [(l', m), (l, j)] = dG/dn_x(x_{m l'}; y_{j l})
    between the P x M surface points and the P x N point sources (all at
    angles 2 pi l / P).  Used only as an independent check of the modal fill."""
    X, Nn = surface_points(geom, P)                          # [P, M, 3]
    Y = source_ring_points(geom, P)                          # [P, N, 3]
    K = kernel.dG_dnx(body.k, X[:, :, None, None, :], Nn[:, :, None, None, :],
                      Y[None, None, :, :, :])                # [P, M, P, N]
    return K.reshape(P * body.M, P * body.N)


def bc_residual(body: Body, geom: Geometry, c: np.ndarray, w: Wave, nt: int, nphi: int,
                qs: int) -> float:
    """epsilon_1 of Sec. 3.3: RMS over an nt x nphi grid on the surface
    (midpoints in t and in angle, so almost none are collocation points) of
    du/dn + du^i/dn, the error in the Neumann condition eq. (neu)."""
    from .geometry import curve_points
    kv = wave_vector(body.k, w)
    t = math.pi * (np.arange(nt) + 0.5) / nt
    rho, z, nrho, nz, _ = curve_points(body.shape, t)
    ph = 2 * math.pi * (np.arange(nphi) + 0.5) / nphi
    cph, sph = np.cos(ph)[:, None], np.sin(ph)[:, None]
    X = np.stack([rho[None] * cph, rho[None] * sph,
                  np.broadcast_to(z, (nphi, nt))], -1).reshape(-1, 3)
    Nn = np.stack([nrho[None] * cph, nrho[None] * sph,
                   np.broadcast_to(nz, (nphi, nt))], -1).reshape(-1, 3)
    Y = source_ring_points(geom, qs).reshape(-1, 3)
    sig = point_strengths(c, qs).reshape(-1)
    du = np.empty(X.shape[0], dtype=np.complex128)
    for t0 in range(0, X.shape[0], 128):
        du[t0:t0 + 128] = kernel.dG_dnx(body.k, X[t0:t0 + 128, None, :],
                                        Nn[t0:t0 + 128, None, :], Y[None]) @ sig
    dui = 1j * (Nn @ kv) * np.exp(1j * (X @ kv))
    return float(np.sqrt(np.mean(np.abs(du + dui) ** 2)))
