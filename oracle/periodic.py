"""Periodizing scheme (Sec. 4 of the paper), plainly.

Unit cell: x in [-e_x/2, e_x/2], y in [-e_y/2, e_y/2], z in [-z0, z0],
obstacle centred at the origin.  Walls L (x = -e_x/2), R (x = +e_x/2),
B (y = -e_y/2), F (y = +e_y/2), D (z = -z0), T (z = +z0), normals along
+x, +y, +z (Sec. 4, start).  Each wall pair carries an M1 x M1 product
Gauss grid (Sec. 4.1).

Representation in the cell (eq. (urep)):
    u = sum_{|a|,|b|<=1} alpha^a beta^b U0(x - a e1 - b e2) + sum_lm d_lm j_l(kr) Y_lm,
with U0 the field of the central copy's ring sources (eq. (Phinear)),
alpha = exp(i k_x e_x), beta = exp(i k_y e_y) (eq. (bloch), reading the
second as the y phase).  Rows of Q and C are ordered
[LR value, LR normal derivative, BF value, BF normal derivative,
 T value, T d/dz, D value, D d/dz], each block M1^2 rows (eq. (full)).
Columns of Q: the (p+1)^2 harmonics (index l^2 + l + m), then the
Rayleigh-Bloch amplitudes a_mn, then b_mn, in the order of rb_orders.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy.special import spherical_jn, sph_harm_y

from workloads import Body, Lattice, Wave, wave_vector
from . import kernel
from .geometry import Geometry, curve_points, source_ring_points, surface_points
from .gmres import gmres
from .onebody import ModalPinv, point_strengths

E1 = np.array([1.0, 0.0, 0.0])
E2 = np.array([0.0, 1.0, 0.0])


# ----------------------------------------------------------------- walls

@dataclass
class Walls:
    R: np.ndarray; L: np.ndarray     # [M1^2, 3] matched nodes
    F: np.ndarray; B: np.ndarray
    T: np.ndarray; D: np.ndarray
    wLR: np.ndarray; wBF: np.ndarray; wTD: np.ndarray  # Gauss area weights


def wall_nodes(lat: Lattice, M1: int | None = None) -> Walls:
    """M1 x M1 product Gauss nodes on each face (Sec. 4.1)."""
    M1 = lat.M1 if M1 is None else M1
    g, w = np.polynomial.legendre.leggauss(M1)
    hx, hy, hz = lat.ex / 2, lat.ey / 2, lat.z0

    def grid(u, v):
        U, V = np.meshgrid(u, v, indexing="ij")
        return U.ravel(), V.ravel()

    yy, zz = grid(g * hy, g * hz)
    R = np.stack([np.full_like(yy, hx), yy, zz], 1)
    L = np.stack([np.full_like(yy, -hx), yy, zz], 1)
    xx, zz2 = grid(g * hx, g * hz)
    F = np.stack([xx, np.full_like(xx, hy), zz2], 1)
    B = np.stack([xx, np.full_like(xx, -hy), zz2], 1)
    xx3, yy3 = grid(g * hx, g * hy)
    T = np.stack([xx3, yy3, np.full_like(xx3, hz)], 1)
    D = np.stack([xx3, yy3, np.full_like(xx3, -hz)], 1)
    W1, W2 = np.meshgrid(w, w, indexing="ij")
    ww = (W1 * W2).ravel()
    return Walls(R, L, F, B, T, D, ww * hy * hz, ww * hx * hz, ww * hx * hy)


# ------------------------------------------------------ Rayleigh-Bloch

@dataclass
class Orders:
    m: np.ndarray; n: np.ndarray
    kx: np.ndarray; ky: np.ndarray; kz: np.ndarray   # kz complex: +real or +imag


def rb_orders(k: float, kv: np.ndarray, lat: Lattice) -> Orders:
    """Bragg orders with kappa_x^2 + kappa_y^2 <= (pi N0)^2, where
    kappa_x = k_x + 2 pi m / e_x, kappa_y = k_y + 2 pi n / e_y and
    kappa_z = +sqrt(k^2 - kappa_x^2 - kappa_y^2) (positive real or positive
    imaginary), eqs. (rb1)-(rb2) and Sec. 4.  Ordered by m, then n."""
    cut = math.pi * lat.N0
    mlo = math.ceil((-cut - kv[0]) * lat.ex / (2 * math.pi))
    mhi = math.floor((cut - kv[0]) * lat.ex / (2 * math.pi))
    nlo = math.ceil((-cut - kv[1]) * lat.ey / (2 * math.pi))
    nhi = math.floor((cut - kv[1]) * lat.ey / (2 * math.pi))
    ms, ns = [], []
    for m in range(mlo, mhi + 1):
        for n in range(nlo, nhi + 1):
            kx = kv[0] + 2 * math.pi * m / lat.ex
            ky = kv[1] + 2 * math.pi * n / lat.ey
            if kx * kx + ky * ky <= cut * cut:
                ms.append(m); ns.append(n)
    m = np.array(ms); n = np.array(ns)
    kx = kv[0] + 2 * math.pi * m / lat.ex
    ky = kv[1] + 2 * math.pi * n / lat.ey
    kz = np.sqrt((k * k - kx * kx - ky * ky).astype(np.complex128))
    return Orders(m, n, kx, ky, kz)


# -------------------------------------------------- spherical harmonics

def lm_index(p: int):
    L = np.concatenate([[l] * (2 * l + 1) for l in range(p + 1)]).astype(int)
    Mv = np.concatenate([np.arange(-l, l + 1) for l in range(p + 1)]).astype(int)
    return L, Mv


def harmonics(k: float, p: int, X: np.ndarray):
    """H_lm(x) = j_l(k r) Y_lm(theta, phi) (orthonormal Y with the
    Condon-Shortley phase, origin at the obstacle centre; the regular
    auxiliary basis of eq. (urep)) and its Cartesian gradient by the chain
    rule in spherical coordinates.  Returns H [T, NH], grad [T, NH, 3].
    Targets must be off the z axis."""
    L, Mv = lm_index(p)
    r = np.linalg.norm(X, axis=1)
    th = np.arccos(np.clip(X[:, 2] / r, -1, 1))
    ph = np.mod(np.arctan2(X[:, 1], X[:, 0]), 2 * math.pi)
    st, ct, sp_, cp = np.sin(th), np.cos(th), np.sin(ph), np.cos(ph)
    assert np.all(st > 1e-12), "harmonic gradient needs targets off the axis"
    Y, dY = sph_harm_y(L[None, :], Mv[None, :], th[:, None], ph[:, None], diff_n=1)
    kr = k * r[:, None]
    jl = spherical_jn(L[None, :], kr)
    jlp = spherical_jn(L[None, :], kr, derivative=True)
    H = jl * Y
    dr = k * jlp * Y
    dth = jl * dY[..., 0] / r[:, None]
    dph = jl * dY[..., 1] / (r * st)[:, None]
    rhat = np.stack([st * cp, st * sp_, ct], 1)[:, None, :]
    that = np.stack([ct * cp, ct * sp_, -st], 1)[:, None, :]
    phat = np.stack([-sp_, cp, np.zeros_like(cp)], 1)[:, None, :]
    grad = dr[..., None] * rhat + dth[..., None] * that + dph[..., None] * phat
    return H, grad


# ---------------------------------------------------- near-field sums

def near_matrices(k: float, Y: np.ndarray, X: np.ndarray, images, want_grad=True):
    """Dense matrices of sum_img w_img G(x - a e1 - b e2, y) (and its
    x-gradient) for targets X [T, 3] and point sources Y [S, 3]; `images`
    is a list of ((a, b) shift in periods, complex weight, lattice)."""
    T, S = X.shape[0], Y.shape[0]
    Vm = np.zeros((T, S), dtype=np.complex128)
    Gm = np.zeros((T, S, 3), dtype=np.complex128) if want_grad else None
    for (a, b), wgt, shift in images:
        Xs = X - shift
        Vm += wgt * kernel.G(k, Xs[:, None, :], Y[None, :, :])
        if want_grad:
            Gm += wgt * kernel.grad_x_G(k, Xs[:, None, :], Y[None, :, :])
    return Vm, Gm


def image_list(lat: Lattice, alpha: complex, beta: complex, which):
    """((a, b), alpha^a beta^b, a e_x E1 + b e_y E2) for the requested shifts."""
    return [((a, b), alpha ** a * beta ** b, a * lat.ex * E1 + b * lat.ey * E2) for a, b in which]


def equilibrated_pinv_factors(Q: np.ndarray, cut: float):
    """Factors of Q's truncated pseudoinverse (Sec. 4.2: SVD, singular values
    below `cut` times the largest dropped), taken of Q with every column
    scaled to unit 2-norm.  The paper leaves the normalisation of the
    auxiliary basis open; with orthonormal Y_lm the columns of the high
    degrees are smaller than the low ones by more than the cutoff, so an
    unscaled relative cutoff would discard them whatever their use.  With
    Q D = U S V^* (D = diag(1/||q_j||)) the pseudoinverse is D V S^+ U^*;
    returned as (U_k, s_k, V_k^* D) for apply_qpinv."""
    dinv = 1.0 / np.linalg.norm(Q, axis=0)
    U, s, Vh = np.linalg.svd(Q * dinv[None, :], full_matrices=False)
    keep = s > cut * s[0]
    return U[:, keep], s[keep], Vh[keep] * dinv[None, :]


NEAR9 = [(a, b) for a in (-1, 0, 1) for b in (-1, 0, 1)]
ELSE8 = [ab for ab in NEAR9 if ab != (0, 0)]


# ------------------------------------------------------- the blocks

class PeriodicSolver:
    """Blocks of eq. (full) and the right-preconditioned system eq. (iter)
    for one obstacle, lattice and incident wave."""

    def __init__(self, body: Body, lat: Lattice, geom: Geometry, A: np.ndarray,
                 pinv: ModalPinv | None = None, rel_cutoff: float = 1e-10):
        self.body, self.lat, self.geom, self.A = body, lat, geom, A
        self.k = body.k
        self.P = body.P
        self.pinv = pinv if pinv is not None else ModalPinv(A, rel_cutoff)
        self.cut = rel_cutoff
        self.walls = wall_nodes(lat)
        self.Xs, self.Ns = surface_points(geom, self.P)          # [P, M, 3]
        self.Ysrc = source_ring_points(geom, self.P)              # [P, N, 3]
        self.Bt = self.btilde()

    # B~: harmonics -> Neumann data Fourier coefficients (Sec. 4.1)
    def btilde(self) -> np.ndarray:
        """B~[n, m, lm] = (1/P) sum_s dH_lm/dn(x_{m s}) e^{-i n phi_s} (the
        trapezoid rule of Sec. 4.1, taken on the normal derivative since the
        first block row enforces the Neumann condition).  [P, M, NH]."""
        P, M = self.P, self.body.M
        _, grad = harmonics(self.k, self.lat.p, self.Xs.reshape(-1, 3))
        dn = np.einsum("tic,tc->ti", grad, self.Ns.reshape(-1, 3))
        return np.fft.fft(dn.reshape(P, M, -1), axis=0) / P

    # per-incidence set-up
    def set_wave(self, w: Wave):
        lat = self.lat
        self.wave = w
        self.kv = wave_vector(self.k, w)
        self.alpha = np.exp(1j * self.kv[0] * lat.ex)
        self.beta = np.exp(1j * self.kv[1] * lat.ey)
        self.orders = rb_orders(self.k, self.kv, lat)
        self.Kelse = self.aelse_point_matrix()
        self.Cpt = self.c_point_matrix(cancel=True)
        self.Q = self.q_matrix()
        self.Qf = equilibrated_pinv_factors(self.Q, self.cut)

    def aelse_point_matrix(self) -> np.ndarray:
        """K_else[(l', m), (l, j)] = sum over the 8 non-central images of
        alpha^a beta^b dG/dn_x(x_{m l'}; y_{j l} + a e1 + b e2), q = P
        (eq. (A) and its description in Sec. 4.1)."""
        X = self.Xs.reshape(-1, 3); Nn = self.Ns.reshape(-1, 3)
        Y = self.Ysrc.reshape(-1, 3)
        K = np.zeros((X.shape[0], Y.shape[0]), dtype=np.complex128)
        for (a, b), wgt, shift in image_list(self.lat, self.alpha, self.beta, ELSE8):
            for t0 in range(0, X.shape[0], 512):
                sl = slice(t0, t0 + 512)
                K[sl] += wgt * kernel.dG_dnx(self.k, X[sl, None, :], Nn[sl, None, :],
                                             Y[None, :, :] + shift)
        return K

    def apply_aelse(self, c: np.ndarray) -> np.ndarray:
        """A_else eta: modes -> point strengths -> phased 8-image sum at the
        surface nodes -> FFT / P (Sec. 4.1).  c [P, N] -> [P, M]."""
        sig = point_strengths(c, self.P).reshape(-1)
        g = (self.Kelse @ sig).reshape(self.P, self.body.M)
        return np.fft.fft(g, axis=0) / self.P

    def _wall_rows(self, val_fn):
        """Assemble the 8 M1^2 rows from a function giving (value, gradient)
        of a field (or of a set of basis fields) at wall points, for the
        wall pair differences and the T/D Cauchy data."""
        W, al, be = self.walls, self.alpha, self.beta
        vR, gR = val_fn(W.R, "R"); vL, gL = val_fn(W.L, "L")
        vF, gF = val_fn(W.F, "F"); vB, gB = val_fn(W.B, "B")
        vT, gT = val_fn(W.T, "T"); vD, gD = val_fn(W.D, "D")
        return np.concatenate([vR - al * vL, gR[..., 0] - al * gL[..., 0],
                               vF - be * vB, gF[..., 1] - be * gB[..., 1],
                               vT, gT[..., 2], vD, gD[..., 2]], axis=0)

    def c_point_matrix(self, cancel: bool = True) -> np.ndarray:
        """C acting on the point strengths sigma (q = P) of the ring sources:
        wall discrepancies u_R - alpha u_L, d_x u_R - alpha d_x u_L,
        u_F - beta u_B, d_y u_F - beta d_y u_B, and Cauchy data u, u_z on T
        and D, of the 3x3 phased near sum (eq. (Phinear)).  With cancel=True
        only the distant images are kept on the side walls: the right-most
        three on L and the left-most three on R (likewise B/F), Sec. 4.1."""
        Y = self.Ysrc.reshape(-1, 3)
        lat, al, be = self.lat, self.alpha, self.beta
        if not cancel:
            imgs = image_list(lat, al, be, NEAR9)
            return self._wall_rows(lambda X, wall: near_matrices(self.k, Y, X, imgs))
        W = self.walls
        left3 = [(-1, b) for b in (-1, 0, 1)]
        right3 = [(1, b) for b in (-1, 0, 1)]
        back3 = [(a, -1) for a in (-1, 0, 1)]
        front3 = [(a, 1) for a in (-1, 0, 1)]
        vR, gR = near_matrices(self.k, Y, W.R, image_list(lat, al, be, left3))
        vL, gL = near_matrices(self.k, Y, W.L, image_list(lat, al, be, right3))
        vF, gF = near_matrices(self.k, Y, W.F, image_list(lat, al, be, back3))
        vB, gB = near_matrices(self.k, Y, W.B, image_list(lat, al, be, front3))
        imgs = image_list(lat, al, be, NEAR9)
        vT, gT = near_matrices(self.k, Y, W.T, imgs)
        vD, gD = near_matrices(self.k, Y, W.D, imgs)
        return np.concatenate([vR - al * vL, gR[..., 0] - al * gL[..., 0],
                               vF - be * vB, gF[..., 1] - be * gB[..., 1],
                               vT, gT[..., 2], vD, gD[..., 2]], axis=0)

    def apply_c(self, c: np.ndarray) -> np.ndarray:
        return self.Cpt @ point_strengths(c, self.P).reshape(-1)

    def q_matrix(self) -> np.ndarray:
        """Q = [S, -W] (Sec. 4.1): S holds the harmonics' wall discrepancies
        and T/D Cauchy data; W the Rayleigh-Bloch plane waves
        exp(i(kappa_x x + kappa_y y)) on T (value, i kappa_z times it for
        d/dz) for a_mn and on D (value, -i kappa_z times it) for b_mn,
        eqs. (T)-(nD)."""
        S = self._wall_rows(lambda X, wall: harmonics(self.k, self.lat.p, X))
        o = self.orders
        nr = self.walls.T.shape[0]
        nrb = o.m.size
        Wa = np.zeros((8 * nr, nrb), dtype=np.complex128)
        Wb = np.zeros((8 * nr, nrb), dtype=np.complex128)
        eT = np.exp(1j * (self.walls.T[:, :1] * o.kx[None] + self.walls.T[:, 1:2] * o.ky[None]))
        eD = np.exp(1j * (self.walls.D[:, :1] * o.kx[None] + self.walls.D[:, 1:2] * o.ky[None]))
        Wa[4 * nr:5 * nr] = eT
        Wa[5 * nr:6 * nr] = 1j * o.kz[None] * eT
        Wb[6 * nr:7 * nr] = eD
        Wb[7 * nr:8 * nr] = -1j * o.kz[None] * eD
        return np.concatenate([S, -Wa, -Wb], axis=1)

    def apply_qpinv(self, y: np.ndarray) -> np.ndarray:
        """Q^+ y = V S^+ (U^* y), truncation relative to s_max (Sec. 4.2)."""
        U, s, Vh = self.Qf
        return Vh.conj().T @ ((U.conj().T @ y) / s)

    def apply_b(self, xi: np.ndarray) -> np.ndarray:
        """B xi = B~ d (B is B~ padded with zeros), [P, M]."""
        NH = (self.lat.p + 1) ** 2
        return self.Bt @ xi[:NH]

    # eq. (iter)
    def op(self, eta_t: np.ndarray) -> np.ndarray:
        """(I + A_else A_0^+ - B Q^+ C A_0^+) eta~ on the flattened [P*M]."""
        P, M = self.P, self.body.M
        x = eta_t.reshape(P, M)
        c = self.pinv.apply(x)
        out = x + self.apply_aelse(c) - self.apply_b(self.apply_qpinv(self.apply_c(c)))
        return out.reshape(-1)

    def solve(self, fh: np.ndarray, tol: float = 1e-12, maxit: int = 200):
        """GMRES on eq. (iter), then eta = A_0^+ eta~ and xi = -Q^+ C eta
        (Sec. 4.2).  Returns a dict with c [P, N], d, a, b and the history."""
        x, its, hist = gmres(self.op, fh.reshape(-1), tol, maxit)
        c = self.pinv.apply(x.reshape(self.P, self.body.M))
        xi = -self.apply_qpinv(self.apply_c(c))
        NH = (self.lat.p + 1) ** 2
        nrb = self.orders.m.size
        return dict(c=c, xi=xi, d=xi[:NH], a=xi[NH:NH + nrb], b=xi[NH + nrb:],
                    iters=its, hist=hist)

    # evaluation and error metrics
    def field_and_grad(self, c: np.ndarray, d: np.ndarray, X: np.ndarray, qs: int,
                       want_grad: bool = True):
        """u (and grad u) at cell points X from eq. (urep): the 3x3 phased
        point-source sum of the ring sources (qs nodes) plus the harmonics."""
        Y = source_ring_points(self.geom, qs).reshape(-1, 3)
        sig = point_strengths(c, qs).reshape(-1)
        imgs = image_list(self.lat, self.alpha, self.beta, NEAR9)
        u = np.zeros(X.shape[0], dtype=np.complex128)
        g = np.zeros((X.shape[0], 3), dtype=np.complex128)
        for t0 in range(0, X.shape[0], 64):
            Xc = X[t0:t0 + 64]
            Vm, Gm = near_matrices(self.k, Y, Xc, imgs, want_grad)
            u[t0:t0 + 64] = Vm @ sig
            if want_grad:
                g[t0:t0 + 64] = np.einsum("tsc,s->tc", Gm, sig)
        H, gH = harmonics(self.k, self.lat.p, X)
        u += H @ d
        g += np.einsum("tic,i->tc", gH, d)
        return u, g

    def eps_flux(self, a: np.ndarray, b: np.ndarray) -> float:
        """|sum_{kappa_z > 0} kappa_z (|a|^2 + |b + e^{-i k_z z0} delta_00|^2)
        - kappa_z^{00}| with k_z the (negative) incident z wavenumber, i.e.
        the (0,0) transmitted amplitude referred to z = -z0 (Sec. 5)."""
        o = self.orders
        prop = (np.abs(o.kz.imag) < 1e-14) & (o.kz.real > 0)
        bb = b.copy()
        i00 = np.where((o.m == 0) & (o.n == 0))[0][0]
        bb[i00] += np.exp(-1j * self.kv[2] * self.lat.z0)
        kz = o.kz.real
        out = np.sum(kz[prop] * (np.abs(a[prop]) ** 2 + np.abs(bb[prop]) ** 2))
        return float(abs(out - kz[i00]))

    def eps_per(self, c, d, qs: int, M1t: int = 10) -> float:
        """RMS over an M1t x M1t Gauss grid on L/R and B/F of the value and
        (1/k) normal-derivative discrepancies of the full representation."""
        W = wall_nodes(self.lat, M1t)
        uR, gR = self.field_and_grad(c, d, W.R, qs)
        uL, gL = self.field_and_grad(c, d, W.L, qs)
        uF, gF = self.field_and_grad(c, d, W.F, qs)
        uB, gB = self.field_and_grad(c, d, W.B, qs)
        r = np.concatenate([uR - self.alpha * uL, (gR[:, 0] - self.alpha * gL[:, 0]) / self.k,
                            uF - self.beta * uB, (gF[:, 1] - self.beta * gB[:, 1]) / self.k])
        return float(np.sqrt(np.mean(np.abs(r) ** 2)))

    def eps_bc(self, c, d, qs: int, nt: int = 16, nphi: int = 16) -> float:
        """RMS over an nt x nphi surface grid of du/dn + du^i/dn; qs should
        be the fill's q since the central ring sources sit close to the
        surface (Thm. 1)."""
        t = math.pi * (np.arange(nt) + 0.5) / nt
        rho, z, nrho, nz, _ = curve_points(self.body.shape, t)
        ph = 2 * math.pi * (np.arange(nphi) + 0.5) / nphi
        cph, sph = np.cos(ph)[:, None], np.sin(ph)[:, None]
        X = np.stack([rho[None] * cph, rho[None] * sph, np.broadcast_to(z, (nphi, nt))], -1).reshape(-1, 3)
        Nn = np.stack([nrho[None] * cph, nrho[None] * sph, np.broadcast_to(nz, (nphi, nt))], -1).reshape(-1, 3)
        _, g = self.field_and_grad(c, d, X, qs)
        dui = 1j * (Nn @ self.kv) * np.exp(1j * (X @ self.kv))
        return float(np.sqrt(np.mean(np.abs(np.sum(g * Nn, 1) + dui) ** 2)))

    # independent dense route
    def dense_full_solve(self, fh: np.ndarray, rcond: float = 1e-12):
        """Assemble eq. (full) densely in mode space and solve it by dense
        least squares (an independent route to the Schur/GMRES answer; tiny
        sizes only).  Returns (c [P, N], xi)."""
        P, M, N = self.P, self.body.M, self.body.N
        F = np.exp(-2j * math.pi * np.outer(np.arange(P), np.arange(P)) / P)  # [bin, angle]
        Kr = self.Kelse.reshape(P, M, P, N)
        Aelse = np.einsum("bl,lmsj,cs->bmcj", F, Kr, F.conj()) / P ** 2
        A = Aelse.reshape(P * M, P * N).copy()
        for n in range(P):
            A[n * M:(n + 1) * M, n * N:(n + 1) * N] += self.A[n]
        NH = (self.lat.p + 1) ** 2
        NQ = self.Q.shape[1]
        Bfull = np.zeros((P * M, NQ), dtype=np.complex128)
        Bfull[:, :NH] = self.Bt.reshape(P * M, NH)
        # C on modes: sigma = (1/P) F^* c per source ring
        Cr = self.Cpt.reshape(-1, P, N)
        Cm = np.einsum("rsj,cs->rcj", Cr, F.conj()).reshape(-1, P * N) / P
        Full = np.block([[A, Bfull], [Cm, self.Q]])
        rhs = np.concatenate([fh.reshape(-1), np.zeros(Cm.shape[0], dtype=np.complex128)])
        sol, *_ = np.linalg.lstsq(Full, rhs, rcond=rcond)
        return sol[:P * N].reshape(P, N), sol[P * N:]
