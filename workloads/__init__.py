"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only *describes* problems: shape parameters, discretisation
sizes, lattice parameters, incident directions drawn from seeded generators
and test-point sets.  It holds none of the method's arithmetic (no kernel,
no quadrature, no geometry of the generating curve beyond the polar radius
used to keep test points outside the obstacle), so that the CPU oracle and
the GPU library can both consume it without sharing any computation.

Notation follows Liu & Barnett, "Efficient numerical solution of acoustic
scattering from doubly-periodic arrays of axisymmetric objects":
N sources per generating curve, M collocation points, P azimuthal modes
(n = -P/2+1..P/2), q trapezoid nodes for the ring-kernel fill, k wavenumber,
tau the complexification (source displacement) parameter (Sec. 3.2), and for
the periodizing scheme (Sec. 4) the lattice periods e_x, e_y, the cell
half-height z0, the spherical-harmonic degree p, the Rayleigh-Bloch cutoff
N0 and the wall Gauss order M1.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Tuple

import numpy as np


@dataclass(frozen=True)
class Shape:
    """Polar generating curve r(t) = a (1 + eps cos(j t)), t in [0, pi],
    rho = r sin t, z = r cos t (t = 0 is the top pole).  eps = 0 is a sphere."""
    a: float
    eps: float = 0.0
    j: int = 0

    def radius(self, theta):
        return self.a * (1.0 + self.eps * np.cos(self.j * np.asarray(theta)))


@dataclass(frozen=True)
class CupShape:
    """The "cup" body of the paper's Fig. 1(c): a spherical shell of mid radius
    1 and half-thickness `half` (in units of the mid radius) with a rounded
    opening of half-angle `b` about the +z axis, given parametrically by a
    radius r(t) and a polar angle theta(t) built from erf; scaled here so that
    the outer radius is `outer`.  Only the parameters live here; the curve is
    evaluated by the oracle and by the library, each in its own code."""
    outer: float = 0.35
    half: float = 0.2
    b: float = math.pi / 6

    def radius(self, theta):
        """Radius of the sphere that encloses the body (used only to keep test
        points outside it)."""
        return np.full(np.shape(theta), self.outer, dtype=float)


@dataclass(frozen=True)
class Body:
    """One axisymmetric obstacle and its one-body discretisation (Sec. 3)."""
    shape: "Shape | CupShape"
    N: int              # MFS sources on the generating curve
    M: int              # collocation points on the generating curve
    P: int              # azimuthal modes, even
    q: int              # trapezoid nodes for the ring-kernel fill, even, q >= P
    k: float            # wavenumber
    tau: float          # complexification parameter (> 0 puts sources inside)
    colloc: str = "mid"  # "mid": t_m = pi (m - 1/2)/M ; "gauss": Gauss-Legendre in t


@dataclass(frozen=True)
class Lattice:
    """Rectangular lattice and periodizer parameters (Sec. 4)."""
    ex: float
    ey: float
    z0: float
    p: int       # max spherical-harmonic degree
    N0: float    # Rayleigh-Bloch cutoff: kappa_x^2 + kappa_y^2 <= (pi N0)^2
    M1: int      # Gauss nodes per wall direction (even)


@dataclass(frozen=True)
class Wave:
    """Incident plane wave from above: k_vec = k (sin th cos ph, sin th sin ph, -cos th)."""
    theta: float
    phi: float


def wave_vector(k: float, w: Wave) -> np.ndarray:
    return k * np.array([math.sin(w.theta) * math.cos(w.phi),
                         math.sin(w.theta) * math.sin(w.phi),
                         -math.cos(w.theta)])


# ---------------------------------------------------------------- samplers

def _near_wood(k: float, lat: Lattice, w: Wave, rel: float = 1e-3) -> bool:
    """True if some Bragg order has |kappa_z| < rel*k (Wood anomaly nearby,
    Sec. 2 remark): such draws are rejected and redrawn."""
    kv = wave_vector(k, w)
    mmax = int(math.ceil((k + math.pi * lat.N0) * lat.ex / (2 * math.pi))) + 1
    nmax = int(math.ceil((k + math.pi * lat.N0) * lat.ey / (2 * math.pi))) + 1
    m = np.arange(-mmax, mmax + 1)[:, None]
    n = np.arange(-nmax, nmax + 1)[None, :]
    kx = kv[0] + 2 * math.pi * m / lat.ex
    ky = kv[1] + 2 * math.pi * n / lat.ey
    kz2 = k * k - kx * kx - ky * ky
    return bool(np.min(np.abs(kz2)) < (rel * k) ** 2)


def sample_waves(k: float, lat: Lattice | None, count: int, seed: int,
                 theta_max: float = math.pi / 2) -> List[Wave]:
    """Incidences with theta ~ U[0, theta_max), phi ~ U[0, 2 pi), drawn in that
    order from numpy's PCG64 stream; near-Wood draws are redrawn."""
    rng = np.random.default_rng(seed)
    out: List[Wave] = []
    while len(out) < count:
        th = float(rng.uniform(0.0, theta_max))
        ph = float(rng.uniform(0.0, 2 * math.pi))
        w = Wave(th, ph)
        if lat is not None and _near_wood(k, lat, w):
            continue
        out.append(w)
    return out


def sample_direction_sphere(seed: int) -> Wave:
    """One direction uniform on S^2, expressed in the (theta, phi) convention
    of :class:`Wave` (theta in [0, pi])."""
    rng = np.random.default_rng(seed)
    u, v = rng.uniform(size=2)
    return Wave(float(math.acos(1.0 - 2.0 * u)), float(2 * math.pi * v))


def fibonacci_sphere(n: int, radius: float) -> np.ndarray:
    """n quasi-uniform points on a sphere (golden-angle spiral), shape [n, 3]."""
    i = np.arange(n) + 0.5
    z = 1.0 - 2.0 * i / n
    r = np.sqrt(1.0 - z * z)
    g = math.pi * (3.0 - math.sqrt(5.0))
    return radius * np.stack([r * np.cos(g * i), r * np.sin(g * i), z], axis=1)


def cell_grid(lat: Lattice, shape: Shape, n: int = 4, clearance: float = 0.1,
              zfrac: float = 0.9) -> np.ndarray:
    """n^3 cell-centred grid points in the unit cell (|z| <= zfrac*z0), keeping
    only those whose radius exceeds the polar radius of the obstacle by at
    least `clearance` (outside the obstacle and away from its surface)."""
    xs = (np.arange(n) + 0.5) / n - 0.5
    X, Y, Z = np.meshgrid(xs * lat.ex, xs * lat.ey, xs * 2 * zfrac * lat.z0, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    r = np.linalg.norm(pts, axis=1)
    th = np.arccos(np.clip(pts[:, 2] / np.maximum(r, 1e-300), -1, 1))
    keep = r > shape.radius(th) + clearance
    return pts[keep]


# ------------------------------------------------------------ named configs

@dataclass(frozen=True)
class Problem:
    name: str
    body: Body
    lattice: Lattice | None
    waves: Tuple[Wave, ...]
    targets: np.ndarray = field(compare=False, repr=False, default=None)
    q_field: int = 0      # trapezoid nodes used when evaluating u at targets
    gmres_tol: float = 1e-12
    maxit: int = 200
    km: float = 0.0       # 0: sound-hard; > 0: transmission with this interior wavenumber
    inner: np.ndarray = field(compare=False, repr=False, default=None)   # test points inside


def sphere_free_space() -> Problem:
    """Sound-hard sphere a = 0.5 in free space, k = 2 pi; 60 Gauss collocation
    nodes, 40 sources on the curve shrunk by 0.7 (tau = ln(1/0.7)), P = 32,
    q = 128; one random direction (seed 1); 64 test points on |x| = 2."""
    b = Body(Shape(0.5), N=40, M=60, P=32, q=128, k=2 * math.pi,
             tau=math.log(1 / 0.7), colloc="gauss")
    return Problem("sphere_free_space", b, None, (sample_direction_sphere(1),),
                   fibonacci_sphere(64, 2.0), q_field=128)


def periodic_k10(nwaves: int = 8) -> Problem:
    """Unit square lattice, k = 10, r = 0.3 (1 + 0.1 cos 3t); N = 200,
    M = 240 (midpoint), tau = 0.1, P = 64, q = 400; periodizer z0 = 0.8,
    p = 30, N0 = 14, M1 = 24 (the smallest Q found by convergence with
    eps_flux and eps_per ~1e-11, a tenth of the 1e-10 target, with Q's
    columns equilibrated); incidences from seed 2."""
    shape = Shape(0.3, 0.1, 3)
    b = Body(shape, N=200, M=240, P=64, q=400, k=10.0, tau=0.1, colloc="mid")
    lat = Lattice(1.0, 1.0, 0.8, p=30, N0=14, M1=24)
    waves = tuple(sample_waves(b.k, lat, nwaves, seed=2))
    return Problem("periodic_k10", b, lat, waves, cell_grid(lat, shape), q_field=256,
                   gmres_tol=1e-10)


def cup_free_space() -> Problem:
    """The cup of Fig. 1(c) (outer radius 0.35) in free space, k = 6, N = 120,
    M = 144, P = 32, tau = 0.1, q = 320 (Theorem 1 rate 0.122); one random
    direction (seed 12); 32 test points on |x| = 1."""
    b = Body(CupShape(), N=120, M=144, P=32, q=320, k=6.0, tau=0.1, colloc="mid")
    return Problem("cup_free_space", b, None, (sample_direction_sphere(12),),
                   fibonacci_sphere(32, 1.0), q_field=320)


def small_periodic_cup(nwaves: int = 2) -> Problem:
    """A small periodic cup case that the oracle solves in seconds: unit
    lattice, the cup of Fig. 1(c) scaled to outer radius 0.35, k = 6,
    N = 60, M = 72, P = 16, tau = 0.1, q = 320 (Theorem 1: the smallest rate
    over the (collocation, source) pairs is 0.13, q >= P/2 + 37/0.13);
    z0 = 0.6, p = 12, N0 = 8, M1 = 14; incidences from seed 9."""
    shape = CupShape()
    b = Body(shape, N=60, M=72, P=16, q=320, k=6.0, tau=0.1, colloc="mid")
    lat = Lattice(1.0, 1.0, 0.6, p=12, N0=8, M1=14)
    waves = tuple(sample_waves(b.k, lat, nwaves, seed=9))
    return Problem("small_periodic_cup", b, lat, waves, cell_grid(lat, shape, n=3), q_field=320)


def cup_periodic_large(nwaves: int = 8) -> Problem:
    """The large configuration: sound-hard cups of Fig. 1(c) (outer radius
    0.35) on the unit square lattice at k = 2 pi 13 (13 wavelengths per
    period); N = 450, M = 540 (midpoint), P = 144 (NP = 64800), tau = 0.05,
    q = 540 (Theorem 1: the smallest rate over the (collocation, source)
    pairs is 0.0829, q >= P/2 + 37/0.0829); periodizer z0 = 0.55, p = 90
    (k times the cell-corner radius 0.89 is 73), N0 = 40, M1 = 56 (about
    3.6 Gauss nodes per wavelength on the walls), chosen by convergence of
    eps_flux and eps_per on the worst incidence (7e-11 and 2e-10);
    incidences from seed 5; GMRES to 1e-10."""
    shape = CupShape()
    b = Body(shape, N=450, M=540, P=144, q=540, k=2 * math.pi * 13, tau=0.05, colloc="mid")
    lat = Lattice(1.0, 1.0, 0.55, p=90, N0=40, M1=56)
    waves = tuple(sample_waves(b.k, lat, nwaves, seed=5))
    return Problem("cup_periodic_large", b, lat, waves, cell_grid(lat, shape), q_field=540,
                   gmres_tol=1e-10)


def sphere_transmission() -> Problem:
    """Penetrable sphere a = 0.5 in free space, k = 2 pi, interior
    wavenumber km = 1.5 k; discretisation of the free-space sphere (60 Gauss
    collocation nodes, N = 40, tau = ln(1/0.7) so the exterior field's
    sources sit at 0.35 and the interior field's at 0.714), P = 32, q = 128;
    one random direction (seed 1); 32 test points on |x| = 2 and 16 inside
    on |x| = 0.25."""
    b = Body(Shape(0.5), N=40, M=60, P=32, q=128, k=2 * math.pi, tau=math.log(1 / 0.7), colloc="gauss")
    return Problem("sphere_transmission", b, None, (sample_direction_sphere(1),), fibonacci_sphere(32, 2.0),
                   q_field=128, km=1.5 * 2 * math.pi, inner=fibonacci_sphere(16, 0.25))


def small_periodic_transmission(nwaves: int = 2) -> Problem:
    """The small periodic body (r = 0.3 (1 + 0.1 cos 3t), N = 40, M = 48,
    P = 24, q = 160, tau = 0.2, unit lattice, z0 = 0.6, p = 24, N0 = 10,
    M1 = 20) as a transmission obstacle with k = 5 and km = 1.5 k;
    incidences from seed 7."""
    pr = small_periodic(nwaves=nwaves)
    return replace(pr, name="small_periodic_transmission", km=1.5 * pr.body.k)


def cup_periodic_large_transmission(nwaves: int = 8) -> Problem:
    """The large configuration's transmission variant: the same cups,
    lattice and discretisation with interior wavenumber km = 1.5 k (the
    doubled sets: 2M x 2N = 1080 x 900 per mode; the exterior sources of the
    interior field need q >= 485 by Theorem 1, under the q = 540 taken)."""
    pr = cup_periodic_large(nwaves)
    return replace(pr, name="cup_periodic_large_transmission", km=1.5 * pr.body.k)


def serving_stream(count: int, seed_dirs: int = 4, seed_arrivals: int = 40):
    """Request stream of the serving configuration against the k = 10
    operator: incidences theta ~ U[0, pi/2), phi ~ U[0, 2 pi) from seed 4
    (near-Wood draws redrawn), and unit-rate exponential inter-arrival gaps
    from seed 40 (scale them by 1/rate for a Poisson stream of that rate)."""
    pr = periodic_k10(1)
    waves = sample_waves(pr.body.k, pr.lattice, count, seed=seed_dirs)
    gaps = np.random.default_rng(seed_arrivals).exponential(1.0, size=count)
    return waves, gaps


def even_5smooth_at_least(x: float) -> int:
    """Smallest even 2^a 3^b 5^c >= x (a length the angle FFTs factor well)."""
    n = max(2, int(math.ceil(x)))
    while True:
        if n % 2 == 0:
            r = n
            for f in (2, 3, 5):
                while r % f == 0:
                    r //= f
            if r == 1:
                return n
        n += 1


def batch_obstacles(count: int = 256, seed: int = 3) -> List[Body]:
    """Batched-build configuration: `count` independent obstacles, each drawn
    in this order from seed 3: a ~ U[0.2, 0.4], eps ~ U[0, 0.15],
    j ~ U{2..5}, N ~ U{100..600}, P ~ U{32, 64, 96, 128, 160},
    k ~ U[5, 30]; M = ceil(1.2 N), midpoint collocation, tau = 0.1, and
    q the smallest even 5-smooth length >= max(P, P/2 + 370) (the fill
    convergence of the k = 10 body at tau = 0.1 with the margin of P/2
    for the highest mode)."""
    rng = np.random.default_rng(seed)
    out: List[Body] = []
    for _ in range(count):
        a = float(rng.uniform(0.2, 0.4))
        eps = float(rng.uniform(0.0, 0.15))
        j = int(rng.integers(2, 6))
        N = int(rng.integers(100, 601))
        P = int(rng.choice([32, 64, 96, 128, 160]))
        k = float(rng.uniform(5.0, 30.0))
        M = int(math.ceil(1.2 * N))
        q = even_5smooth_at_least(max(P, P / 2 + 370))
        out.append(Body(Shape(a, eps, j), N=N, M=M, P=P, q=q, k=k, tau=0.1, colloc="mid"))
    return out


def tiny_free_space() -> Problem:
    """A small sphere case for fast CPU tests: a = 0.5, k = 2, N = 16,
    M = 20 (Gauss), P = 8, q = 48."""
    b = Body(Shape(0.5), N=16, M=20, P=8, q=48, k=2.0, tau=math.log(1 / 0.6), colloc="gauss")
    return Problem("tiny_free_space", b, None, (sample_direction_sphere(11),),
                   fibonacci_sphere(16, 2.0), q_field=48)


def small_periodic(nwaves: int = 2, k: float = 5.0) -> Problem:
    """A small periodic case that the oracle solves in seconds: unit lattice,
    r = 0.3 (1 + 0.1 cos 3t), N = 40, M = 48, P = 24, q = 160, tau = 0.2,
    z0 = 0.6, p = 24, N0 = 10, M1 = 20."""
    shape = Shape(0.3, 0.1, 3)
    b = Body(shape, N=40, M=48, P=24, q=160, k=k, tau=0.2, colloc="mid")
    lat = Lattice(1.0, 1.0, 0.6, p=24, N0=10, M1=20)
    waves = tuple(sample_waves(b.k, lat, nwaves, seed=7))
    return Problem("small_periodic", b, lat, waves, cell_grid(lat, shape, n=3), q_field=64)


def with_(obj, **kw):
    """dataclasses.replace shorthand for deriving variants of a config."""
    return replace(obj, **kw)
