// Host-side geometry of the method: the polar and cup generating curves
// (Sec. 3, Fig. 1) with their normals and complexified MFS sources
// (Sec. 3.2), Gauss-Legendre
// nodes (collocation in t, wall grids of Sec. 4.1), the unit-cell walls and
// the Rayleigh-Bloch orders of eqs. (rb1)-(rb2).
#include "geometry.hpp"

#include "common.hpp"

#include <cmath>
#include <complex>

namespace mfs {

using cplx = std::complex<double>;

void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
  // Newton iteration on P_n from the Chebyshev-like initial guess
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int l = 2; l <= n; ++l) {
        const double p2 = ((2.0 * l - 1.0) * z * p1 - (l - 1.0) * p0) / l;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1.0; }
      const double dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) {
        // final derivative for the weight
        double q0 = 1.0, q1 = z;
        for (int l = 2; l <= n; ++l) {
          const double q2 = ((2.0 * l - 1.0) * z * q1 - (l - 1.0) * q0) / l;
          q0 = q1;
          q1 = q2;
        }
        const double dq = n * (z * q1 - q0) / (z * z - 1.0);
        w[i] = 2.0 / ((1.0 - z * z) * dq * dq);
        break;
      }
    }
    x[i] = z;
  }
  // ascending order
  for (int i = 0; i < n / 2; ++i) {
    std::swap(x[i], x[n - 1 - i]);
    std::swap(w[i], w[n - 1 - i]);
  }
}

static cplx radius(const mfs_polar_spec &s, cplx t) { return s.a * (1.0 + s.eps * std::cos((double)s.j * t)); }

void polar_geometry(const mfs_polar_spec &s, double *rho, double *z, double *nrho, double *nz,
                    double *srho, double *sz) {
  std::vector<double> t(s.M);
  if (s.colloc == 1) {
    std::vector<double> x, w;
    gauss_legendre(s.M, x, w);
    for (int m = 0; m < s.M; ++m) t[m] = kPi * (x[m] + 1.0) / 2.0;
  } else {
    for (int m = 0; m < s.M; ++m) t[m] = kPi * (m + 0.5) / s.M;
  }
  for (int m = 0; m < s.M; ++m) {
    const double tt = t[m];
    const double r = s.a * (1.0 + s.eps * std::cos(s.j * tt));
    const double rp = -s.a * s.eps * s.j * std::sin(s.j * tt);
    rho[m] = r * std::sin(tt);
    z[m] = r * std::cos(tt);
    const double dr = rp * std::sin(tt) + r * std::cos(tt);
    const double dz = rp * std::cos(tt) - r * std::sin(tt);
    const double sp = std::hypot(dr, dz);
    nrho[m] = -dz / sp;   // outward for this orientation (t = 0 at the top pole)
    nz[m] = dr / sp;
  }
  for (int j = 0; j < s.N; ++j) {
    // Z(t) = rho + i z = r(t) (sin t + i cos t), continued to t_j - i tau
    const cplx tc(kPi * (j + 0.5) / s.N, -s.tau);
    const cplx Z = radius(s, tc) * (std::sin(tc) + cplx(0.0, 1.0) * std::cos(tc));
    srho[j] = Z.real();
    sz[j] = Z.imag();
  }
}

// sin(w)/w
static double sinc(double w) {
  if (std::fabs(w) < 1e-4) return 1.0 - w * w / 6.0 + w * w * w * w / 120.0;
  return std::sin(w) / w;
}

// erf(x + iy) by the series of Abramowitz & Stegun 7.1.29:
//   erf(x) + e^{-x^2}/(2 pi x) [(1 - cos 2xy) + i sin 2xy]
//   + (2/pi) e^{-x^2} sum_{n >= 1} e^{-n^2/4}/(n^2 + 4x^2) (f_n + i g_n),
//   f_n = 2x - 2x cosh(ny) cos(2xy) + n sinh(ny) sin(2xy),
//   g_n = 2x cosh(ny) sin(2xy) + n sinh(ny) cos(2xy),
// whose error is about 1e-16 of |erf| for the |y| <= 1 used here.  The
// second term is written with sinc so that x = 0 needs no special case.
static cplx erf_complex(cplx z) {
  const double x = z.real(), y = z.imag();
  const double ex = std::exp(-x * x);
  const double xy = x * y;
  const double s1 = sinc(xy);
  double re = std::erf(x) + ex * x * y * y * s1 * s1 / kPi;
  double im = ex * y * sinc(2.0 * xy) / kPi;
  const double c2 = std::cos(2.0 * xy), s2 = std::sin(2.0 * xy);
  double sr = 0.0, si = 0.0;
  for (int n = 1; n <= 40; ++n) {
    const double w = std::exp(-0.25 * n * n) / (n * n + 4.0 * x * x);
    const double ch = std::cosh(n * y), sh = std::sinh(n * y);
    sr += w * (2.0 * x - 2.0 * x * ch * c2 + n * sh * s2);
    si += w * (2.0 * x * ch * s2 + n * sh * c2);
  }
  re += 2.0 / kPi * ex * sr;
  im += 2.0 / kPi * ex * si;
  return {re, im};
}

// Cup of Fig. 1(c) at u = pi - t (x = u - pi/2 = pi/2 - t): radius
// r = 1 - a erf(x/a), polar angle theta = b - a + kap s_a(x) with
// kap = 2 (1 - (b - a)/pi) and s_a(x) = x erf(x/a) + (a/sqrt(pi)) e^{-x^2/a^2}.
void cup_geometry(const mfs_cup_spec &s, double *rho, double *z, double *nrho, double *nz, double *srho,
                  double *sz) {
  const double a = s.half, b = s.b, c = s.outer / (1.0 + a);
  const double kap = 2.0 * (1.0 - (b - a) / kPi);
  const double rsp = 1.0 / std::sqrt(kPi);
  std::vector<double> t(s.M);
  if (s.colloc == 1) {
    std::vector<double> x, w;
    gauss_legendre(s.M, x, w);
    for (int m = 0; m < s.M; ++m) t[m] = kPi * (x[m] + 1.0) / 2.0;
  } else {
    for (int m = 0; m < s.M; ++m) t[m] = kPi * (m + 0.5) / s.M;
  }
  for (int m = 0; m < s.M; ++m) {
    const double x = 0.5 * kPi - t[m];
    const double e = std::erf(x / a), g = std::exp(-(x / a) * (x / a));
    const double r = 1.0 - a * e;
    const double th = b - a + kap * (x * e + a * rsp * g);
    const double r_t = 2.0 * rsp * g;   // dr/dt (dx/dt = -1)
    const double th_t = -kap * e;       // dtheta/dt
    rho[m] = c * r * std::sin(th);
    z[m] = c * r * std::cos(th);
    const double dr = c * (r_t * std::sin(th) + r * std::cos(th) * th_t);
    const double dz = c * (r_t * std::cos(th) - r * std::sin(th) * th_t);
    const double sp = std::hypot(dr, dz);
    nrho[m] = -dz / sp;   // outward: the curve runs clockwise in the (rho, z) half plane
    nz[m] = dr / sp;
  }
  for (int j = 0; j < s.N; ++j) {
    // Z = c r (sin theta + i cos theta) continued to t_j - i tau
    const cplx x(0.5 * kPi - kPi * (j + 0.5) / s.N, s.tau);
    const cplx e = erf_complex(x / a);
    const cplx r = 1.0 - a * e;
    const cplx th = b - a + kap * (x * e + a * rsp * std::exp(-(x / a) * (x / a)));
    const cplx Z = c * r * (std::sin(th) + cplx(0.0, 1.0) * std::cos(th));
    srho[j] = Z.real();
    sz[j] = Z.imag();
  }
}

void wall_nodes(const mfs_lattice &lat, std::vector<double> &soa) {
  const int M1 = lat.M1, n = M1 * M1;
  std::vector<double> g, w;
  gauss_legendre(M1, g, w);
  const double hx = lat.ex / 2, hy = lat.ey / 2, hz = lat.z0;
  soa.assign((size_t)18 * n, 0.0);   // walls R L F B T D, each x y z [n]
  auto put = [&](int wall, int i, double x, double y, double z) {
    soa[(size_t)(3 * wall) * n + i] = x;
    soa[(size_t)(3 * wall + 1) * n + i] = y;
    soa[(size_t)(3 * wall + 2) * n + i] = z;
  };
  for (int a = 0; a < M1; ++a)
    for (int b = 0; b < M1; ++b) {
      const int i = a * M1 + b;
      put(0, i, hx, g[a] * hy, g[b] * hz);
      put(1, i, -hx, g[a] * hy, g[b] * hz);
      put(2, i, g[a] * hx, hy, g[b] * hz);
      put(3, i, g[a] * hx, -hy, g[b] * hz);
      put(4, i, g[a] * hx, g[b] * hy, hz);
      put(5, i, g[a] * hx, g[b] * hy, -hz);
    }
}

void rb_orders(double k, const double kv[3], const mfs_lattice &lat, std::vector<RBOrder> &out) {
  out.clear();
  const double cut = kPi * lat.N0;
  const int mlo = (int)std::ceil((-cut - kv[0]) * lat.ex / (2 * kPi));
  const int mhi = (int)std::floor((cut - kv[0]) * lat.ex / (2 * kPi));
  const int nlo = (int)std::ceil((-cut - kv[1]) * lat.ey / (2 * kPi));
  const int nhi = (int)std::floor((cut - kv[1]) * lat.ey / (2 * kPi));
  for (int m = mlo; m <= mhi; ++m)
    for (int n = nlo; n <= nhi; ++n) {
      const double kx = kv[0] + 2 * kPi * m / lat.ex;
      const double ky = kv[1] + 2 * kPi * n / lat.ey;
      if (kx * kx + ky * ky <= cut * cut) {
        RBOrder o;
        o.m = m;
        o.n = n;
        o.kx = kx;
        o.ky = ky;
        const double kz2 = k * k - kx * kx - ky * ky;
        o.kz = kz2 >= 0.0 ? cplx(std::sqrt(kz2), 0.0) : cplx(0.0, std::sqrt(-kz2));
        out.push_back(o);
      }
    }
}

}  // namespace mfs
