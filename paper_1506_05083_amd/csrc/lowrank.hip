// Low-rank image blocks of A_else (eq. (A); Sec. 6 names the compression of
// these neighbour interactions as the way on to larger periods).
//
// For a body whose stored near field does not fit in HBM the surface sums
// of A_else otherwise evaluate every (target, source, image) kernel value at
// every GMRES iteration.  The blocks K_e[t][s] = dG/dn_t(x_t - e, y_s) of
// the eight neighbour images are numerically of low rank (the images lie a
// gap away from the body), and they do not depend on the incident wave
// (the Bloch phases weight whole images), so they are factored once per
// lattice and applied as matrix products:
//
//   build (per class of images that a lattice rotation carries into each
//   other, one representative e):
//     Omega: S x ell complex Gaussian (counter-based hash, Box-Muller);
//     Y = K_e Omega            lr_sketch_kernel: kernel values generated in
//                              registers, Omega staged through LDS, FP64
//                              matrix cores (the randomised range finder);
//     Y = Q R                  the library's blocked Householder QR; ell is
//                              grown until the last |R_ii| / max |R_ii| is
//                              below 1e-13, then cut where it first falls
//                              below 1e-13 (plus 16 columns);
//     U = Q[:, :ell]           the QR's U formation from the identity;
//     X = U^H K_e              lr_project_kernel: kernel values generated in
//                              registers, U staged through LDS;
//   apply (every iteration, all right-hand sides of the batch):
//     Z[r][rot] = X sigma_r(R^rot .)      lr_stage1_kernel (slices of the
//                                          sources, partial sums),
//     Y[r][rot] = w_r(R^rot e) sum Z      lr_reduce_kernel,
//     out_r(t) = sum_rot (U Y[r][rot])(R^-rot t)
//                                          lr_stage2_kernel (the nrot target
//                                          tiles of one rotation orbit per
//                                          workgroup: U read once).
// Both passes of the build cost 8 T S ell flops each on the matrix cores;
// the apply streams U and X once (16 (T + S) ell bytes per class).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <vector>

#include "internal.hpp"

namespace mfs {

void launch_zero(double2 *p, long n, hipStream_t s);
// U = Q [I; 0] from the QR's reflectors (qr.hip)
void qr_form_u(const MatDesc *descs, const std::vector<MatDesc> &h, int maxrank, hipStream_t s, bool from_identity,
               int nb);

namespace {

constexpr int LC = 128;   // columns of a build workgroup's tile (8 blocks of 16)
constexpr int LK = 16;    // contraction indices per LDS stage of the build

struct LrGeom {
  const double *tgt;   // SoA x y z nx ny nz, [npad] each
  int npad;
  const double *src;   // SoA x y z, [S] each
  int T, S;
  double k;
};

// dG/dn_t (x_t - (sx, sy, 0), y_s): the derivative along the target's unit
// normal of e^{ikR} / (4 pi R)
__device__ inline double2 lr_kernel(double dx, double dy, double dz, double nx, double ny, double nz, double k) {
  const double R2 = fma(dx, dx, fma(dy, dy, dz * dz));
  const double iR = rsqrt(R2);
  double sn, cs;
  sincos(k * (R2 * iR), &sn, &cs);
  const double f = fma(nx, dx, fma(ny, dy, nz * dz)) * iR * iR * (0.25 / kPi);
  return cz(f * fma(-cs, iR, -sn * k), f * fma(cs, k, -sn * iR));
}

__device__ inline unsigned long long mix64(unsigned long long x) {   // SplitMix64 finaliser
  x += 0x9e3779b97f4a7c15ULL;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ULL;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebULL;
  return x ^ (x >> 31);
}

// Omega[s][c] (row length ldo), complex Gaussian by Box-Muller on two
// hashed uniforms; columns c >= ell are zero
__global__ void lr_omega_kernel(double2 *__restrict__ om, int S, int ell, int ldo, unsigned long long seed) {
  const long total = (long)S * ldo;
  for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
    const int c = (int)(idx % ldo);
    if (c >= ell) { om[idx] = cz(0.0, 0.0); continue; }
    const unsigned long long h1 = mix64(seed ^ (2ULL * (unsigned long long)idx));
    const unsigned long long h2 = mix64(seed ^ (2ULL * (unsigned long long)idx + 1ULL));
    const double u1 = ((double)(h1 >> 11) + 1.0) * 0x1.0p-53;   // (0, 1]
    const double u2 = (double)(h2 >> 11) * 0x1.0p-53;
    const double r = sqrt(-2.0 * log(u1));
    double sn, cs;
    sincos(2.0 * kPi * u2, &sn, &cs);
    om[idx] = cz(r * cs, r * sn);
  }
}

// Y[c][t] (column-major, ld ldy) = sum_s K_e[t][s] Omega[s][c]; computed as
// D[c][t] = sum_s Omega^T[c][s] K^T[s][t] so that a lane group stores 16
// consecutive targets of one column.  Workgroup: 64 targets (16 a wave) x
// 128 columns; the lane (l16, k4) evaluates K at target l16 and source k4 of
// each 4-source step.
__global__ __launch_bounds__(256) void lr_sketch_kernel(LrGeom g, double sx, double sy,
                                                        const double2 *__restrict__ om, int ldo,
                                                        double2 *__restrict__ Y, int ldy, int ell) {
  __shared__ double2 Os[LK][LC + 1];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int l16 = lane & 15, k4 = lane >> 4;
  const int c0 = blockIdx.y * LC;
  const int t = blockIdx.x * 64 + 16 * wv + l16;
  const bool tin = t < g.T;
  const int tt = tin ? t : 0;
  const double tx = g.tgt[tt] - sx, ty = g.tgt[g.npad + tt] - sy, tz = g.tgt[2 * g.npad + tt];
  const double nx = g.tgt[3 * g.npad + tt], ny = g.tgt[4 * g.npad + tt], nz = g.tgt[5 * g.npad + tt];
  dx4 re[LC / 16], im[LC / 16];
#pragma unroll
  for (int u = 0; u < LC / 16; ++u) {
    re[u] = dx4{0.0, 0.0, 0.0, 0.0};
    im[u] = re[u];
  }
  for (int s0 = 0; s0 < g.S; s0 += LK) {
#pragma unroll
    for (int u = 0; u < LK * LC / 256; ++u) {
      const int idx = tid + 256 * u, r = idx / LC, c = idx % LC;
      const int s = s0 + r;
      Os[r][c] = s < g.S ? om[(size_t)s * ldo + c0 + c] : cz(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < LK; kk += 4) {
      const int s = s0 + kk + k4;
      const int sc = s < g.S ? s : 0;
      double2 kv = lr_kernel(tx - g.src[sc], ty - g.src[g.S + sc], tz - g.src[2 * g.S + sc], nx, ny, nz, g.k);
      kv = csel(tin && s < g.S, kv, cz(0.0, 0.0));
#pragma unroll
      for (int u = 0; u < LC / 16; ++u) {
        const double2 o = Os[kk + k4][16 * u + l16];
        re[u] = mfma_f64(o.x, kv.x, re[u]);
        re[u] = mfma_f64(-o.y, kv.y, re[u]);
        im[u] = mfma_f64(o.x, kv.y, im[u]);
        im[u] = mfma_f64(o.y, kv.x, im[u]);
      }
    }
    __syncthreads();
  }
  if (!tin) return;
  // lane (l16, k4) holds D[c = 16 u + k4 + 4 v][t] in element v
#pragma unroll
  for (int u = 0; u < LC / 16; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int c = c0 + 16 * u + k4 + 4 * v;
      if (c < ell) Y[(size_t)c * ldy + t] = cz(re[u][v], im[u][v]);
    }
}

// X[s][i] (row length ldx) = sum_t conj(U[t][i]) K_e[t][s]; computed as
// D[s][i] = sum_t K^T[s][t] conj(U)[t][i] so that a lane group stores 16
// consecutive i of one source.  Workgroup: 64 sources (16 a wave) x 128
// columns of U; the lane (l16, k4) evaluates K at source l16 and target k4
// of each 4-target step.
__global__ __launch_bounds__(256) void lr_project_kernel(LrGeom g, double sx, double sy,
                                                         const double2 *__restrict__ U, int ldu, int ell,
                                                         double2 *__restrict__ X, int ldx) {
  __shared__ double2 Us[LK][LC + 1];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int l16 = lane & 15, k4 = lane >> 4;
  const int i0 = blockIdx.y * LC;
  const int s = blockIdx.x * 64 + 16 * wv + l16;
  const bool sin_ = s < g.S;
  const int sc = sin_ ? s : 0;
  const double yx = g.src[sc] + sx, yy = g.src[g.S + sc] + sy, yz = g.src[2 * g.S + sc];
  dx4 re[LC / 16], im[LC / 16];
#pragma unroll
  for (int u = 0; u < LC / 16; ++u) {
    re[u] = dx4{0.0, 0.0, 0.0, 0.0};
    im[u] = re[u];
  }
  for (int t0 = 0; t0 < g.T; t0 += LK) {
#pragma unroll
    for (int u = 0; u < LK * LC / 256; ++u) {
      const int idx = tid + 256 * u, r = idx % LK, i = i0 + idx / LK;
      const int t = t0 + r;
      Us[r][idx / LK] = (t < g.T && i < ell) ? U[(size_t)i * ldu + t] : cz(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < LK; kk += 4) {
      const int t = t0 + kk + k4;
      const int tc = t < g.T ? t : 0;
      double2 kv = lr_kernel(g.tgt[tc] - yx, g.tgt[g.npad + tc] - yy, g.tgt[2 * g.npad + tc] - yz,
                             g.tgt[3 * g.npad + tc], g.tgt[4 * g.npad + tc], g.tgt[5 * g.npad + tc], g.k);
      kv = csel(sin_ && t < g.T, kv, cz(0.0, 0.0));
#pragma unroll
      for (int u = 0; u < LC / 16; ++u) {
        const double2 w = Us[kk + k4][16 * u + l16];
        // kv * conj(w)
        re[u] = mfma_f64(kv.x, w.x, re[u]);
        re[u] = mfma_f64(kv.y, w.y, re[u]);
        im[u] = mfma_f64(kv.y, w.x, im[u]);
        im[u] = mfma_f64(-kv.x, w.y, im[u]);
      }
    }
    __syncthreads();
  }
  // lane (l16, k4) holds D[s = 16 wv + k4 + 4 v][i = 16 u + l16] in element v
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int sr = blockIdx.x * 64 + 16 * wv + k4 + 4 * v;
    if (sr >= g.S) continue;
#pragma unroll
    for (int u = 0; u < LC / 16; ++u) {
      const int i = i0 + 16 * u + l16;
      if (i < ell) X[(size_t)sr * ldx + i] = cz(re[u][v], im[u][v]);
    }
  }
}

// first ell columns of the identity, ldu rows each
__global__ void lr_identity_kernel(double2 *__restrict__ U, int ldu, int ell) {
  const int c = blockIdx.y;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < ldu; r += gridDim.x * blockDim.x)
    U[(size_t)c * ldu + r] = cz(r == c ? 1.0 : 0.0, 0.0);
  (void)ell;
}

__global__ void lr_diag_kernel(const double2 *__restrict__ A, int lda, int n, double *__restrict__ d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const double2 v = A[(size_t)i * lda + i];
    d[i] = sqrt(v.x * v.x + v.y * v.y);
  }
}

constexpr int LR_SLICE = 2048;   // sources per workgroup of the first apply stage
constexpr int LR_R = 16;         // right-hand-side columns of the apply (nrhs <= 16)

// Zp[slice][rot][i][r] = sum over the slice's sources s of X[s][i] sigma[r][R^rot s]
// (one wave: 16 rows i, all rotations)
template <int NROT>
__global__ __launch_bounds__(64) void lr_stage1_kernel(const double2 *__restrict__ X, int ldx, int ell, int S,
                                                       int shiftS, const double2 *__restrict__ sigma, int nrhs,
                                                       double2 *__restrict__ Zp) {
  const int lane = threadIdx.x, l16 = lane & 15, k4 = lane >> 4;
  const int i0 = blockIdx.x * 16, slice = blockIdx.y;
  const int sb = slice * LR_SLICE, se = min(S, sb + LR_SLICE);
  const bool rin = l16 < nrhs;
  const double2 *sg = sigma + (size_t)(rin ? l16 : 0) * S;
  dx4 re[NROT], im[NROT];
#pragma unroll
  for (int r = 0; r < NROT; ++r) {
    re[r] = dx4{0.0, 0.0, 0.0, 0.0};
    im[r] = re[r];
  }
  for (int s0 = sb; s0 < se; s0 += 4) {
    const int s = s0 + k4;
    const bool ok = s < se;
    const int sc = ok ? s : 0;
    const double2 a = ld_or0(X, (size_t)sc * ldx + i0 + l16, ok && i0 + l16 < ell);
#pragma unroll
    for (int r = 0; r < NROT; ++r) {
      int sr = sc + r * shiftS;
      sr = sr >= S ? sr - S : sr;
      const double2 b = ld_or0(sg, sr, ok && rin);
      re[r] = mfma_f64(a.x, b.x, re[r]);
      re[r] = mfma_f64(-a.y, b.y, re[r]);
      im[r] = mfma_f64(a.x, b.y, im[r]);
      im[r] = mfma_f64(a.y, b.x, im[r]);
    }
  }
  // lane (l16, k4) holds D[i = k4 + 4 v][r = l16]
#pragma unroll
  for (int r = 0; r < NROT; ++r)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + k4 + 4 * v;
      Zp[(((size_t)slice * NROT + r) * ell + i) * LR_R + l16] = cz(re[r][v], im[r][v]);
    }
}

// Yc[rot][i][r] = w[img(rot)][r] sum over slices of Zp (zero for r >= nrhs)
__global__ void lr_reduce_kernel(const double2 *__restrict__ Zp, int nslice, int nrot, int ell, int nrhs,
                                 const double2 *__restrict__ w, int4 img, double2 *__restrict__ Yc) {
  const int n = nrot * ell * LR_R;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  const int r = idx % LR_R, rot = idx / (ell * LR_R);
  if (r >= nrhs) { Yc[idx] = cz(0.0, 0.0); return; }
  double2 acc = cz(0.0, 0.0);
  for (int sl = 0; sl < nslice; ++sl) acc = cadd(acc, Zp[(size_t)sl * n + idx]);
  const int im = rot == 0 ? img.x : rot == 1 ? img.y : rot == 2 ? img.z : img.w;
  Yc[idx] = cmul(w[(size_t)im * nrhs + r], acc);
}

// out[r][t0 + row + o shiftT] (+)= sum_rot sum_i U[t0 + row + ((o - rot) mod NROT) shiftT][i] Yc[rot][i][r]
// for the 16 rows of the orbit tile t0 (rows past shiftT masked); the four
// waves split the columns i and are summed through LDS.  accumulate: add to
// out (a later class) instead of storing.
template <int NROT>
__global__ __launch_bounds__(256) void lr_stage2_kernel(const double2 *__restrict__ U, int ldu, int ell, int T,
                                                        int shiftT, const double2 *__restrict__ Yc, int nrhs,
                                                        double2 *__restrict__ out, size_t ldo, int accumulate) {
  __shared__ dx4 red[3][NROT][2][64];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int l16 = lane & 15, k4 = lane >> 4;
  const int t0 = blockIdx.x * 16;
  const bool rowin = t0 + l16 < shiftT;
  const int row = rowin ? t0 + l16 : 0;
  dx4 re[NROT], im[NROT];
#pragma unroll
  for (int o = 0; o < NROT; ++o) {
    re[o] = dx4{0.0, 0.0, 0.0, 0.0};
    im[o] = re[o];
  }
  const int per = ell / 4;   // a multiple of 4 (ell is a multiple of 16)
  for (int i0 = wv * per; i0 < (wv + 1) * per; i0 += 4) {
    const int i = i0 + k4;
    double2 a[NROT];
#pragma unroll
    for (int q = 0; q < NROT; ++q) {
      int t = row + q * shiftT;
      t = t >= T ? t - T : t;
      a[q] = ld_or0(U, (size_t)i * ldu + t, rowin);
    }
#pragma unroll
    for (int rot = 0; rot < NROT; ++rot) {
      const double2 b = Yc[((size_t)rot * ell + i) * LR_R + l16];
#pragma unroll
      for (int o = 0; o < NROT; ++o) {
        const double2 x = a[(o - rot + NROT) % NROT];
        re[o] = mfma_f64(x.x, b.x, re[o]);
        re[o] = mfma_f64(-x.y, b.y, re[o]);
        im[o] = mfma_f64(x.x, b.y, im[o]);
        im[o] = mfma_f64(x.y, b.x, im[o]);
      }
    }
  }
  if (wv > 0) {
#pragma unroll
    for (int o = 0; o < NROT; ++o) {
      red[wv - 1][o][0][lane] = re[o];
      red[wv - 1][o][1][lane] = im[o];
    }
  }
  __syncthreads();
  if (wv != 0) return;
#pragma unroll
  for (int o = 0; o < NROT; ++o)
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      re[o] += red[w][o][0][lane];
      im[o] += red[w][o][1][lane];
    }
  // lane (l16, k4) holds D[row = k4 + 4 v][r = l16]
  if (l16 >= nrhs) return;
#pragma unroll
  for (int o = 0; o < NROT; ++o)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int rr = t0 + k4 + 4 * v;
      if (rr >= shiftT) continue;
      double2 *p = out + (size_t)l16 * ldo + rr + (size_t)o * shiftT;
      const double2 val = cz(re[o][v], im[o][v]);
      *p = accumulate ? cadd(*p, val) : val;
    }
}

}  // namespace

std::shared_ptr<NearLowRank> build_near_lowrank(const BodyData &b, const NsumPlan &psurf, double ex, double ey,
                                                hipStream_t s) {
  MFS_REQUIRE(!b.trans() && psurf.groups.size() == 1 && psurf.groups[0].t0 == 0 && psurf.groups[0].nimg == 8,
              "low-rank near field: sound-hard surface plan expected");
  auto lr = std::make_shared<NearLowRank>();
  lr->P = b.P; lr->M = b.M; lr->N = b.N;
  lr->T = b.P * b.M;
  lr->S = b.P * b.N;
  lr->ex = ex; lr->ey = ey; lr->k = b.k;
  // MFS_LOWRANK_HALFTURN=1 takes the half-turn form on a square lattice too
  const char *ht = std::getenv("MFS_LOWRANK_HALFTURN");
  const bool square = std::fabs(ex - ey) <= 1e-12 * std::max(ex, ey) && b.P % 4 == 0 && !(ht && std::atoi(ht));
  lr->nrot = square ? 4 : 2;
  lr->ncls = square ? 2 : 4;
  lr->shiftT = (b.P / lr->nrot) * b.M;
  lr->shiftS = (b.P / lr->nrot) * b.N;
  const int reps[4][2] = {{1, 0}, {1, 1}, {0, 1}, {1, -1}};
  const int creps2[4][2] = {{1, 0}, {0, 1}, {1, 1}, {1, -1}};
  const NsumGroup &grp = psurf.groups[0];
  for (int c = 0; c < lr->ncls; ++c) {
    auto &C = lr->cls[c];
    C.a = square ? reps[c][0] : creps2[c][0];
    C.b = square ? reps[c][1] : creps2[c][1];
    int a = C.a, bb = C.b;
    for (int r = 0; r < lr->nrot; ++r) {
      int found = -1;
      for (int im = 0; im < grp.nimg; ++im)
        if (grp.ia[im] == a && grp.ib[im] == bb) found = im;
      MFS_REQUIRE(found >= 0, "low-rank near field: image missing from the surface plan");
      C.img[r] = found;
      if (lr->nrot == 4) { const int na = -bb, nb = a; a = na; bb = nb; }   // rotation by +pi/2
      else { a = -a; bb = -bb; }                                           // half-turn
    }
  }
  const int T = lr->T, S = lr->S;
  const int ldy = round_up(T, 16);
  // rank of the widest class: start from (k r)^2 (the body seen from an
  // image subtends about that many wavelength-sized patches), grow if short
  double rmax = 0.0;
  for (int m = 0; m < b.M; ++m) rmax = std::max(rmax, std::hypot(b.h_rho[m], b.h_z[m]));
  const int cap = std::max(16, std::min(T, S) / 16 * 16);
  int ell0 = round_up((int)(1.1 * (b.k * rmax) * (b.k * rmax)) + 64, 64);
  if (const char *e = std::getenv("MFS_LOWRANK_ELL")) ell0 = round_up(std::max(16, std::atoi(e)), 16);
  LrGeom g{psurf.tgt.as<double>(), psurf.ntarget_pad, b.src_P.as<double>(), T, S, b.k};
  hipEvent_t e0, e1;
  HIP_CHECK(hipEventCreate(&e0));
  HIP_CHECK(hipEventCreate(&e1));
  HIP_CHECK(hipEventRecord(e0, s));
  DevBuf flags(2 * sizeof(int));
  for (int c = 0; c < lr->ncls; ++c) {
    auto &C = lr->cls[c];
    const double sx = C.a * ex, sy = C.b * ey;
    int ell = std::min(cap, ell0);
    for (;;) {
      const int ldo = round_up(ell, LC);
      if (device_free_bytes() < ((size_t)S * ldo + 2 * (size_t)ldy * ell + (size_t)S * ell) * sizeof(double2) +
                                    ((size_t)2 << 30)) {
        progress("low-rank near field: class (%d, %d) at width %d does not fit; sums stay on the fly", C.a, C.b,
                 ell);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return nullptr;
      }
      DevBuf om((size_t)S * ldo * sizeof(double2)), Y((size_t)ldy * ell * sizeof(double2));
      hipLaunchKernelGGL(lr_omega_kernel, dim3(2048), dim3(256), 0, s, om.as<double2>(), S, ell, ldo,
                         0x5eed0000ULL + 7919ULL * (unsigned long long)c + (unsigned long long)ell);
      hipLaunchKernelGGL(lr_sketch_kernel, dim3(cdiv(T, 64), ldo / LC), dim3(256), 0, s, g, sx, sy,
                         om.as<double2>(), ldo, Y.as<double2>(), ldy, ell);
      HIP_CHECK(hipGetLastError());
      om.release();
      // Y = Q R (panels of 16)
      const int npan = cdiv(ell, 16);
      DevBuf tau((size_t)ell * sizeof(double2)), Tf((size_t)npan * 16 * 16 * sizeof(double2));
      MatDesc d{};
      d.a = Y.as<double2>(); d.m = T; d.n = ell; d.lda = ldy;
      d.tau = tau.as<double2>(); d.T = Tf.as<double2>();
      d.rank = flags.as<int>(); d.flag = flags.as<int>() + 1;
      std::vector<MatDesc> hd{d};
      DevBuf dd(sizeof(MatDesc));
      HIP_CHECK(hipMemcpyAsync(dd.p, &hd[0], sizeof(MatDesc), hipMemcpyHostToDevice, s));
      qr_factor(dd.as<MatDesc>(), hd, s, 16);
      DevBuf dg((size_t)ell * sizeof(double));
      hipLaunchKernelGGL(lr_diag_kernel, dim3(cdiv(ell, 256)), dim3(256), 0, s, Y.as<double2>(), ldy, ell,
                         dg.as<double>());
      std::vector<double> diag(ell);
      HIP_CHECK(hipMemcpyAsync(diag.data(), dg.p, ell * sizeof(double), hipMemcpyDeviceToHost, s));
      HIP_CHECK(hipStreamSynchronize(s));
      const double dmax = *std::max_element(diag.begin(), diag.end());
      const double tail = dmax > 0.0 ? diag[ell - 1] / dmax : 0.0;
      if (tail > 1e-13 && ell < cap) {   // the sketch still sees directions above the noise: widen
        const int next = std::min(cap, round_up(ell + ell / 2, 64));
        progress("low-rank near field: class (%d, %d) width %d short (tail %.1e); widening to %d", C.a, C.b, ell,
                 tail, next);
        ell = next;
        continue;
      }
      // keep the columns up to where |R_ii| falls below 1e-13 of the largest
      // (the sketch's own rounding floor is about 2e-14 at S = 64800)
      int keep = ell;
      for (int i = 0; i < ell; ++i)
        if (diag[i] < 1e-13 * dmax) { keep = i; break; }
      keep = std::min(ell, round_up(std::max(keep, 1) + 16, 16));
      C.ell = keep;
      C.ldu = ldy;
      C.tail = keep < ell ? diag[keep] / dmax : tail;
      C.U.alloc((size_t)ldy * keep * sizeof(double2));
      hipLaunchKernelGGL(lr_identity_kernel, dim3(cdiv(ldy, 256), keep), dim3(256), 0, s, C.U.as<double2>(), ldy,
                         keep);
      hd[0].u = C.U.as<double2>();
      hd[0].ldu = ldy;
      HIP_CHECK(hipMemcpyAsync(dd.p, &hd[0], sizeof(MatDesc), hipMemcpyHostToDevice, s));
      HIP_CHECK(hipMemcpyAsync(flags.p, &keep, sizeof(int), hipMemcpyHostToDevice, s));
      qr_form_u(dd.as<MatDesc>(), hd, keep, s, true, 16);
      C.X.alloc((size_t)S * keep * sizeof(double2));
      hipLaunchKernelGGL(lr_project_kernel, dim3(cdiv(S, 64), cdiv(keep, LC)), dim3(256), 0, s, g, sx, sy,
                         C.U.as<double2>(), ldy, keep, C.X.as<double2>(), keep);
      HIP_CHECK(hipGetLastError());
      HIP_CHECK(hipStreamSynchronize(s));   // the host copies above go out of scope
      lr->bytes += ((size_t)ldy + S) * keep * sizeof(double2);
      progress("low-rank near field: class (%d, %d) x %d rotations: rank %d of sketch %d (|R| tail %.1e)", C.a,
               C.b, lr->nrot, keep, ell, C.tail);
      break;
    }
  }
  HIP_CHECK(hipEventRecord(e1, s));
  HIP_CHECK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
  lr->build_ms = ms;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return lr;
}

size_t lowrank_work_bytes(const NearLowRank &lr, int nrhs) {
  (void)nrhs;
  int ellmax = 0;
  for (int c = 0; c < lr.ncls; ++c) ellmax = std::max(ellmax, lr.cls[c].ell);
  const int nslice = cdiv(lr.S, LR_SLICE);
  return ((size_t)nslice * lr.nrot * ellmax * LR_R + (size_t)lr.nrot * ellmax * LR_R) * sizeof(double2);
}

void lowrank_apply(const NearLowRank &lr, int nrhs, const double2 *sigma, const double2 *w, double2 *out,
                   size_t ldo, void *work, hipStream_t s) {
  MFS_REQUIRE(nrhs >= 1 && nrhs <= LR_R, "low-rank near field: 1..16 right-hand sides");
  const int nslice = cdiv(lr.S, LR_SLICE);
  for (int c = 0; c < lr.ncls; ++c) {
    const auto &C = lr.cls[c];
    double2 *Zp = static_cast<double2 *>(work);
    double2 *Yc = Zp + (size_t)nslice * lr.nrot * C.ell * LR_R;
    const int4 img = make_int4(C.img[0], C.img[1], C.img[2], C.img[3]);
    if (lr.nrot == 4) {
      hipLaunchKernelGGL(lr_stage1_kernel<4>, dim3(C.ell / 16, nslice), dim3(64), 0, s, C.X.as<double2>(), C.ell,
                         C.ell, lr.S, lr.shiftS, sigma, nrhs, Zp);
    } else {
      hipLaunchKernelGGL(lr_stage1_kernel<2>, dim3(C.ell / 16, nslice), dim3(64), 0, s, C.X.as<double2>(), C.ell,
                         C.ell, lr.S, lr.shiftS, sigma, nrhs, Zp);
    }
    const int n = lr.nrot * C.ell * LR_R;
    hipLaunchKernelGGL(lr_reduce_kernel, dim3(cdiv(n, 256)), dim3(256), 0, s, Zp, nslice, lr.nrot, C.ell, nrhs, w,
                       img, Yc);
    if (lr.nrot == 4)
      hipLaunchKernelGGL(lr_stage2_kernel<4>, dim3(cdiv(lr.shiftT, 16)), dim3(256), 0, s, C.U.as<double2>(), C.ldu,
                         C.ell, lr.T, lr.shiftT, Yc, nrhs, out, ldo, c > 0 ? 1 : 0);
    else
      hipLaunchKernelGGL(lr_stage2_kernel<2>, dim3(cdiv(lr.shiftT, 16)), dim3(256), 0, s, C.U.as<double2>(), C.ldu,
                         C.ell, lr.T, lr.shiftT, Yc, nrhs, out, ldo, c > 0 ? 1 : 0);
    HIP_CHECK(hipGetLastError());
  }
}

}  // namespace mfs
