// Auxiliary spherical-harmonic basis H_lm = j_l(kr) Y_lm (eq. (urep)) and the
// Rayleigh-Bloch plane waves (eqs. (T)-(nD)): the per-incidence fill of
// Q = [S, -W] (Sec. 4.1), the Neumann data of the harmonics on the surface
// rings (the B~ block) and the harmonic part of the field at test points.
//
// Y_lm are orthonormal with the Condon-Shortley phase, Y_l^{-m} =
// (-1)^m conj(Y_l^m), origin at the obstacle centre.  Normalised associated
// Legendre functions by the standard stable recurrences
//   P_0^0 = 1/sqrt(4 pi),  P_m^m = -sqrt((2m+1)/(2m)) sin(th) P_{m-1}^{m-1},
//   P_{m+1}^m = sqrt(2m+3) cos(th) P_m^m,
//   P_l^m = a_lm (cos(th) P_{l-1}^m - b_lm P_{l-2}^m),
//   a_lm = sqrt((4l^2-1)/(l^2-m^2)), b_lm = sqrt(((l-1)^2-m^2)/(4(l-1)^2-1)),
// their theta derivative
//   dP_l^m/dth = (l cos(th) P_l^m - sqrt((2l+1)/(2l-1)) sqrt(l^2-m^2) P_{l-1}^m) / sin(th),
// and spherical Bessel functions by Miller's backward recurrence normalised
// with j_0 = sin x / x or j_1 = sin x / x^2 - cos x / x.  Cartesian gradients
// follow from grad H = dH/dr r^ + (1/r) dH/dth th^ + (1/(r sin th)) dH/dph ph^,
// so targets must lie off the z axis (wall nodes with M1 even, surface
// rings with rho > 0).
#include "internal.hpp"

namespace mfs {
namespace {

constexpr int MAXP = 96;

__device__ void sph_bessel(int p, double x, double *j, double *jp) {
  const int L = p + 32 + (int)x;
  double fnext = 0.0, f = 1e-200;
  for (int l = L; l >= 1; --l) {
    const double fprev = (2.0 * l + 1.0) / x * f - fnext;   // f_{l-1}
    fnext = f;
    f = fprev;
    if (l - 1 <= p) j[l - 1] = f;
    if (l <= p) j[l] = fnext;
    if (fabs(f) > 1e250) {
      f *= 1e-250;
      fnext *= 1e-250;
      for (int i = l - 1; i <= p; ++i)
        if (i >= 0) j[i] *= 1e-250;
    }
  }
  double s, c;
  sincos(x, &s, &c);
  const double j0 = s / x;
  const double j1 = s / (x * x) - c / x;
  double scale;
  if (fabs(j0) >= fabs(j1)) scale = j0 / j[0];
  else scale = j1 / j[1];
  for (int l = 0; l <= p; ++l) j[l] *= scale;
  jp[0] = -j[1];
  for (int l = 1; l <= p; ++l) jp[l] = j[l - 1] - (l + 1.0) / x * j[l];
}

// Spherical coordinates of a point and the frame vectors.
struct Sph {
  double r, ct, st, cp, sp;
};
__device__ inline Sph sph_of(double x, double y, double z) {
  Sph o;
  const double rho = sqrt(x * x + y * y);
  o.r = sqrt(rho * rho + z * z);
  o.ct = z / o.r;
  o.st = rho / o.r;
  o.cp = rho > 0.0 ? x / rho : 1.0;
  o.sp = rho > 0.0 ? y / rho : 0.0;
  return o;
}

// Visit every (l, m >= 0): calls f(l, m, P_l^m, dP_l^m/dth).
template <class F>
__device__ inline void legendre_visit(int p, double ct, double st, F f) {
  double pmm = 0.28209479177387814;   // 1/sqrt(4 pi)
  for (int m = 0; m <= p; ++m) {
    if (m > 0) pmm = -sqrt((2.0 * m + 1.0) / (2.0 * m)) * st * pmm;
    double p2 = 0.0, p1 = pmm;   // P_{l-2}, P_{l-1}
    // l = m
    {
      const double dth = (m * ct * pmm) / st;
      f(m, m, pmm, dth);
    }
    for (int l = m + 1; l <= p; ++l) {
      double pl;
      if (l == m + 1) pl = sqrt(2.0 * m + 3.0) * ct * pmm;
      else {
        const double a = sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)m * m));
        const double b = sqrt(((l - 1.0) * (l - 1.0) - (double)m * m) / (4.0 * (l - 1.0) * (l - 1.0) - 1.0));
        pl = a * (ct * p1 - b * p2);
      }
      const double dth = (l * ct * pl - sqrt((2.0 * l + 1.0) / (2.0 * l - 1.0)) *
                                            sqrt((double)l * l - (double)m * m) * p1) / st;
      f(l, m, pl, dth);
      p2 = p1;
      p1 = pl;
    }
  }
}

// Value and Cartesian gradient of H_lm for m >= 0 and its m < 0 partner,
// given j, jp, P, dP/dth at a point.
struct HVal {
  double2 h, gx, gy, gz;
};
__device__ inline void harm_pair(int l, int m, double P, double dP, const double *j,
                                 const double *jp, double k, const Sph &s, HVal &pos, HVal &neg) {
  // e^{i m phi} by angle addition on (cp, sp)
  const double phi = atan2(s.sp, s.cp);
  double sm, cm;
  sincos(m * phi, &sm, &cm);
  const double2 e = cz(cm, sm);
  const double jl = j[l];
  const double dr = k * jp[l] * P;           // d/dr of the real radial-polar part
  const double dth = jl * dP / s.r;          // (1/r) d/dth
  const double dph = jl * P / (s.r * s.st);  // times (i m e) below
  // r^, th^, ph^
  const double rx = s.st * s.cp, ry = s.st * s.sp, rz = s.ct;
  const double tx = s.ct * s.cp, ty = s.ct * s.sp, tz = -s.st;
  const double px = -s.sp, py = s.cp;
  const double ax = dr * rx + dth * tx, ay = dr * ry + dth * ty, az = dr * rz + dth * tz;
  // grad = e * (a) + i m e * dph * ph^
  const double2 ime = cz(-m * e.y * dph, m * e.x * dph);
  pos.h = cscale(e, jl * P);
  pos.gx = cadd(cscale(e, ax), cscale(ime, px));
  pos.gy = cadd(cscale(e, ay), cscale(ime, py));
  pos.gz = cscale(e, az);
  // Y_l^{-m} = (-1)^m conj(Y_l^m); the radial factor is real
  const double sg = (m & 1) ? -1.0 : 1.0;
  neg.h = cscale(cconj(pos.h), sg);
  neg.gx = cscale(cconj(pos.gx), sg);
  neg.gy = cscale(cconj(pos.gy), sg);
  neg.gz = cscale(cconj(pos.gz), sg);
}

__device__ inline int lm_col(int l, int m) { return l * l + l + m; }

// One thread per (unit, node): units LR, FB (pairs of walls) and T, D; each
// writes two rows of Q: value and normal-derivative (discrepancy or Cauchy).
__global__ __launch_bounds__(64) void qfill_s_kernel(const QFillArgs *__restrict__ args) {
  const QFillArgs a = args[blockIdx.y];   // one incidence per grid row
  const int M1sq = a.M1 * a.M1;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 4 * M1sq) return;
  const int unit = idx / M1sq, i = idx % M1sq;
  double j1[MAXP + 1], jp1[MAXP + 1], j2[MAXP + 1], jp2[MAXP + 1];
  // walls SoA: R L F B T D
  auto wall = [&](int w, int c) { return a.wall[(size_t)(3 * w + c) * M1sq + i]; };
  int w1, w2;
  double2 ph;
  int comp;   // gradient component of the normal
  if (unit == 0) { w1 = 0; w2 = 1; ph = a.alpha; comp = 0; }
  else if (unit == 1) { w1 = 2; w2 = 3; ph = a.beta; comp = 1; }
  else if (unit == 2) { w1 = 4; w2 = -1; ph = cz(0.0, 0.0); comp = 2; }
  else { w1 = 5; w2 = -1; ph = cz(0.0, 0.0); comp = 2; }
  const Sph s1 = sph_of(wall(w1, 0), wall(w1, 1), wall(w1, 2));
  sph_bessel(a.p, a.k * s1.r, j1, jp1);
  Sph s2 = s1;
  if (w2 >= 0) {
    s2 = sph_of(wall(w2, 0), wall(w2, 1), wall(w2, 2));
    sph_bessel(a.p, a.k * s2.r, j2, jp2);
  }
  const int rowv = (2 * unit) * M1sq + i, rowd = (2 * unit + 1) * M1sq + i;
  auto put = [&](int col, const HVal &h1, const HVal *h2) {
    double2 v = h1.h;
    double2 g = comp == 0 ? h1.gx : (comp == 1 ? h1.gy : h1.gz);
    if (h2) {
      v = csub(v, cmul(ph, h2->h));
      const double2 g2 = comp == 0 ? h2->gx : (comp == 1 ? h2->gy : h2->gz);
      g = csub(g, cmul(ph, g2));
    }
    a.Q[(size_t)col * a.ldq + rowv] = v;
    a.Q[(size_t)col * a.ldq + rowd] = g;
  };
  if (w2 < 0) {
    legendre_visit(a.p, s1.ct, s1.st, [&](int l, int m, double P, double dP) {
      HVal hp, hn;
      harm_pair(l, m, P, dP, j1, jp1, a.k, s1, hp, hn);
      put(lm_col(l, m), hp, nullptr);
      if (m > 0) put(lm_col(l, -m), hn, nullptr);
    });
  } else {
    // both points share l, m; evaluate the second point's Legendre functions
    // in the same order by a second pass that adds into Q
    legendre_visit(a.p, s1.ct, s1.st, [&](int l, int m, double P, double dP) {
      HVal hp, hn;
      harm_pair(l, m, P, dP, j1, jp1, a.k, s1, hp, hn);
      put(lm_col(l, m), hp, nullptr);
      if (m > 0) put(lm_col(l, -m), hn, nullptr);
    });
    legendre_visit(a.p, s2.ct, s2.st, [&](int l, int m, double P, double dP) {
      HVal hp, hn;
      harm_pair(l, m, P, dP, j2, jp2, a.k, s2, hp, hn);
      auto sub = [&](int col, const HVal &h2) {
        const double2 g2 = comp == 0 ? h2.gx : (comp == 1 ? h2.gy : h2.gz);
        double2 *qv = &a.Q[(size_t)col * a.ldq + rowv];
        double2 *qd = &a.Q[(size_t)col * a.ldq + rowd];
        *qv = csub(*qv, cmul(ph, h2.h));
        *qd = csub(*qd, cmul(ph, g2));
      };
      sub(lm_col(l, m), hp);
      if (m > 0) sub(lm_col(l, -m), hn);
    });
  }
}

// -W blocks: rows of T (value, d/dz) for the a_mn columns and of D for b_mn.
__global__ void qfill_w_kernel(const QFillArgs *__restrict__ args) {
  const QFillArgs a = args[blockIdx.y];   // one incidence per grid row
  const int M1sq = a.M1 * a.M1;
  const int NH = (a.p + 1) * (a.p + 1);
  const long total = (long)4 * M1sq * a.nrb;
  for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    const int o = (int)(idx / (4 * M1sq));
    const int rr = (int)(idx % (4 * M1sq));
    const int blk = rr / M1sq, i = rr % M1sq;     // 0 T val, 1 T dz, 2 D val, 3 D dz
    const int w = blk < 2 ? 4 : 5;
    const double x = a.wall[(size_t)(3 * w) * M1sq + i], y = a.wall[(size_t)(3 * w + 1) * M1sq + i];
    double s, c;
    sincos(a.kx[o] * x + a.ky[o] * y, &s, &c);
    const double2 e = cz(c, s);
    const double2 ikz = cz(-a.kz[o].y, a.kz[o].x);     // i kappa_z
    double2 v;
    if (blk == 0 || blk == 2) v = cz(-e.x, -e.y);
    else if (blk == 1) v = cscale(cmul(ikz, e), -1.0);
    else v = cmul(ikz, e);
    const int row = (4 + blk) * M1sq + i;
    const int col = NH + (blk < 2 ? 0 : a.nrb) + o;
    a.Q[(size_t)col * a.ldq + row] = v;
  }
}

__global__ void zero_kernel(double2 *p, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    p[i] = cz(0.0, 0.0);
}

// dH_lm/dn at (rho_i, 0, z_i) with normal (nrho_i, 0, nz_i): out[lm][i].
__global__ __launch_bounds__(64) void bfill_kernel(int M, int p, double k, const double *rho,
                                                   const double *z, const double *nrho,
                                                   const double *nz, double2 *out, int value) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  double j[MAXP + 1], jp[MAXP + 1];
  const Sph s = sph_of(rho[i], 0.0, z[i]);
  sph_bessel(p, k * s.r, j, jp);
  const double nr = nrho[i], nzz = nz[i];
  legendre_visit(p, s.ct, s.st, [&](int l, int m, double P, double dP) {
    const double dr = k * jp[l] * P, dth = j[l] * dP / s.r;
    // d/drho = st d/dr + ct/r d/dth ; d/dz = ct d/dr - st/r d/dth  (phi = 0)
    const double v = value ? j[l] * P : nr * (s.st * dr + s.ct * dth) + nzz * (s.ct * dr - s.st * dth);
    out[(size_t)lm_col(l, m) * M + i] = cz(v, 0.0);
    if (m > 0) out[(size_t)lm_col(l, -m) * M + i] = cz((m & 1) ? -v : v, 0.0);
  });
}

// out[r][b][i] -= sum over (l, mm) with mm = b (mod P) of B[lm][i] d[r][lm];
// out[r][b][i] at (r P + b) ldo + i
__global__ void bapply_kernel(int nrhs, int P, int M, int p, const double2 *__restrict__ B,
                              const double2 *__restrict__ d, int ldd, double2 *__restrict__ out, int ldo) {
  const long total = (long)nrhs * P * M;
  for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    const int i = (int)(idx % M);
    const int b = (int)((idx / M) % P);
    const int r = (int)(idx / ((long)M * P));
    double2 acc = cz(0.0, 0.0);
    // modes mm congruent to b with |mm| <= p
    int mm0 = b;
    while (mm0 - P >= -p) mm0 -= P;   // smallest candidate >= -p
    for (int mm = mm0; mm <= p; mm += P) {
      const int am = mm < 0 ? -mm : mm;
      for (int l = am; l <= p; ++l) {
        const int col = lm_col(l, mm);
        cfma(acc, B[(size_t)col * M + i], d[(size_t)r * ldd + col]);
      }
    }
    const size_t o = ((size_t)r * P + b) * ldo + i;
    out[o] = csub(out[o], acc);
  }
}

// u[r][t] += sum_lm H_lm(x_t) d[r][lm]
__global__ __launch_bounds__(64) void harm_field_kernel(int nrhs, int nt, const double *xyz, int p,
                                                        double k, const double2 *d, int ldd,
                                                        double2 *out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  double j[MAXP + 1], jp[MAXP + 1];
  const Sph s = sph_of(xyz[3 * t], xyz[3 * t + 1], xyz[3 * t + 2]);
  sph_bessel(p, k * s.r, j, jp);
  const double phi = atan2(s.sp, s.cp);
  for (int r = 0; r < nrhs; ++r) {
    double2 acc = cz(0.0, 0.0);
    legendre_visit(p, s.ct, s.st, [&](int l, int m, double P, double dP) {
      double sm, cm;
      sincos(m * phi, &sm, &cm);
      const double2 hv = cz(j[l] * P * cm, j[l] * P * sm);
      cfma(acc, hv, d[(size_t)r * ldd + lm_col(l, m)]);
      if (m > 0) {
        const double sg = (m & 1) ? -1.0 : 1.0;
        cfma(acc, cscale(cconj(hv), sg), d[(size_t)r * ldd + lm_col(l, -m)]);
      }
    });
    out[(size_t)r * nt + t] = cadd(out[(size_t)r * nt + t], acc);
  }
}

}  // namespace

void launch_qfill(const std::vector<QFillArgs> &h, hipStream_t s) {
  const int W = (int)h.size();
  if (W == 0) return;
  const int M1sq = h[0].M1 * h[0].M1;
  int nrbmax = 0;
  for (const auto &a : h) {
    MFS_REQUIRE(a.p <= MAXP, "harmonic degree p exceeds 96");
    MFS_REQUIRE(a.M1 == h[0].M1 && a.p == h[0].p, "one wall grid and degree per batch");
    nrbmax = std::max(nrbmax, a.nrb);
    const long n = (long)a.ldq * ((a.p + 1) * (a.p + 1) + 2 * a.nrb);
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)std::min<long>(4096, (n + 255) / 256)), dim3(256), 0, s,
                       a.Q, n);
  }
  DevBuf args(h.size() * sizeof(QFillArgs));
  HIP_CHECK(hipMemcpyAsync(args.p, h.data(), h.size() * sizeof(QFillArgs), hipMemcpyHostToDevice, s));
  // every incidence in one grid: the harmonics of a wall node are a long
  // serial evaluation per thread, so the incidences side by side fill the chip
  hipLaunchKernelGGL(qfill_s_kernel, dim3(cdiv(4 * M1sq, 64), W), dim3(64), 0, s, args.as<QFillArgs>());
  const long nw = (long)4 * M1sq * nrbmax;
  if (nw > 0)
    hipLaunchKernelGGL(qfill_w_kernel, dim3((unsigned)std::min<long>(4096, (nw + 255) / 256), W), dim3(256), 0, s,
                       args.as<QFillArgs>());
  HIP_CHECK(hipGetLastError());
  HIP_CHECK(hipStreamSynchronize(s));   // the argument array is released on return
}

void launch_bfill(int M, int p, double k, const double *rho, const double *z, const double *nrho,
                  const double *nz, double2 *out, hipStream_t s, int value) {
  MFS_REQUIRE(p <= MAXP, "harmonic degree p exceeds 96");
  hipLaunchKernelGGL(bfill_kernel, dim3(cdiv(M, 64)), dim3(64), 0, s, M, p, k, rho, z, nrho, nz, out, value);
  HIP_CHECK(hipGetLastError());
}

void launch_bapply(int nrhs, int P, int M, int p, const double2 *B, const double2 *d, int ldd,
                   double2 *out, hipStream_t s, int ldo) {
  const long n = (long)nrhs * P * M;
  if (ldo <= 0) ldo = M;
  hipLaunchKernelGGL(bapply_kernel, dim3((unsigned)std::min<long>(2048, (n + 255) / 256)), dim3(256), 0, s,
                     nrhs, P, M, p, B, d, ldd, out, ldo);
  HIP_CHECK(hipGetLastError());
}

void launch_harm_field(int nrhs, int nt, const double *xyz, int p, double k, const double2 *d,
                       int ldd, double2 *out, hipStream_t s) {
  MFS_REQUIRE(p <= MAXP, "harmonic degree p exceeds 96");
  hipLaunchKernelGGL(harm_field_kernel, dim3(cdiv(nt, 64)), dim3(64), 0, s, nrhs, nt, xyz, p, k, d, ldd,
                     out);
  HIP_CHECK(hipGetLastError());
}

}  // namespace mfs
