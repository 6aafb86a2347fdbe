// Column-pivoted QR of batched square triangles with the pivots chosen on a
// random sketch (the rank-revealing step of the truncated pseudoinverses,
// Sec. 4.2), after Martinsson, Quintana-Orti, Heavner and van de Geijn,
// "Householder QR factorization with randomization for column pivoting
// (HQRRP)", SIAM J. Sci. Comput. 39 (2017), and Duersch and Gu, "Randomized
// QR with column pivoting", SIAM J. Sci. Comput. 39 (2017).
//
// Y = Omega A (Omega: L x m, independent standard normal entries, L = QB +
// 8 rows) stands in for A in the choice of pivots.  For each block of QB
// columns: an ordinary column-pivoted QR of the sketch of the remaining
// columns (L rows, QB steps) names QB columns; they are swapped to the
// front of the remaining block in A and in Y (and in the pivot record); the
// block is factored by the unpivoted blocked Householder QR, whose trailing
// update is one matrix-core pass over the rest of A; the sketch of the rest
// follows from Y2 <- Y2 - Y1 R11^{-1} R12 (the sketch of the updated
// trailing block under the rotated Omega Q, which is again Gaussian), so A
// is read once per block for the update and never per column.
//
// The result has the form the other pivoted QRs leave: R above the
// diagonal, Householder vectors below it with tau (LAPACK's zlarfg
// convention), the compact-WY T of every 32-column panel, and piv (the
// original column at each position).  The pivots differ from those of the
// deterministic QRCP; what the callers use them for (the graded Jacobi's
// ordering, the complete orthogonal decomposition's cut at the trailing
// Frobenius norm of the R it produced) does not depend on the exact order.
#include <cmath>
#include <cstdint>
#include <vector>

#include "internal.hpp"

namespace mfs {
namespace {

constexpr int QB = 32;          // columns a block (the QR's panel width and the T factors')
constexpr int SL = QB + 8;      // rows of the sketch
constexpr int SRC = 32;         // rows of A a chunk in the sketch product

__device__ inline uint64_t mix64(uint64_t z) {   // splitmix64 finaliser
  z += 0x9e3779b97f4a7c15ULL;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

// om[i * ldo + r] ~ N(0, 1): Box-Muller on two 53-bit uniforms of a hash of (i, r)
__global__ void omega_kernel(double *__restrict__ om, int ldo, int m) {
  const long n = (long)SL * ldo;
  for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += (long)gridDim.x * blockDim.x) {
    const int i = (int)(idx / ldo), r = (int)(idx % ldo);
    double v = 0.0;
    if (r < m) {
      const uint64_t h1 = mix64(((uint64_t)i << 32) ^ (uint64_t)r), h2 = mix64(h1 ^ 0x5851f42d4c957f2dULL);
      const double u1 = ((h1 >> 11) + 1.0) * 0x1.0p-53, u2 = (h2 >> 11) * 0x1.0p-53;   // u1 in (0, 1]
      v = sqrt(-2.0 * log(u1)) * cospi(2.0 * u2);
    }
    om[idx] = v;
  }
}

// Y[c][i] = sum_r om[i][r] A[r][c] for i < SL, c < n (Y column-major, SL rows)
__global__ __launch_bounds__(256) void sketch_kernel(const MatDesc *__restrict__ ad, const double *__restrict__ om,
                                                     int ldo, double2 *__restrict__ Y, size_t ystride) {
  const MatDesc a = ad[blockIdx.y];
  const int c0 = blockIdx.x * 64;
  if (c0 >= a.n) return;
  const int tid = threadIdx.x, cc = tid & 63, g = tid >> 6;
  __shared__ double2 As[SRC][65];
  __shared__ double Os[SL][SRC + 1];
  double2 acc[SL / 4];
#pragma unroll
  for (int t = 0; t < SL / 4; ++t) acc[t] = cz(0.0, 0.0);
  for (int r0 = 0; r0 < a.m; r0 += SRC) {
    for (int e = tid; e < SRC * 64; e += 256) {
      const int rr = e % SRC, q = e / SRC, r = r0 + rr, c = c0 + q;
      As[rr][q] = (r < a.m && c < a.n) ? a.a[(size_t)c * a.lda + r] : cz(0.0, 0.0);
    }
    for (int e = tid; e < SL * SRC; e += 256) {
      const int rr = e % SRC, i = e / SRC, r = r0 + rr;
      Os[i][rr] = r < a.m ? om[(size_t)i * ldo + r] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int rr = 0; rr < SRC; ++rr) {
      const double2 x = As[rr][cc];
#pragma unroll
      for (int t = 0; t < SL / 4; ++t) {
        const double o = Os[g + 4 * t][rr];
        acc[t].x = fma(o, x.x, acc[t].x);
        acc[t].y = fma(o, x.y, acc[t].y);
      }
    }
    __syncthreads();
  }
  const int c = c0 + cc;
  if (c < a.n) {
    double2 *y = Y + blockIdx.y * ystride + (size_t)c * SL;
#pragma unroll
    for (int t = 0; t < SL / 4; ++t) y[g + 4 * t] = acc[t];
  }
}

// The sketch of the remaining columns [K0, n) as a matrix of its own
// (yt, SL x (n - K0)), its column norms and an identity pivot record.
__global__ __launch_bounds__(256) void ycopy_kernel(const MatDesc *__restrict__ ad, int K0,
                                                    const double2 *__restrict__ Y, size_t ystride,
                                                    double2 *__restrict__ yt, double *__restrict__ ytn,
                                                    int *__restrict__ ytp, int ld) {
  const MatDesc a = ad[blockIdx.y];
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (K0 + j >= a.n) return;
  const int lane = threadIdx.x & 63;
  const double2 x = lane < SL ? Y[blockIdx.y * ystride + (size_t)(K0 + j) * SL + lane] : cz(0.0, 0.0);
  if (lane < SL) yt[blockIdx.y * ystride + (size_t)j * SL + lane] = x;
  const double s = wave_sum(cabs2(x));
  if (lane == 0) {
    ytn[(size_t)blockIdx.y * ld + j] = sqrt(s);
    ytp[(size_t)blockIdx.y * ld + j] = j;
  }
}

// One wave a matrix: the swaps (i, sw[i]) that bring the chosen columns
// ytp[0..nb) (positions relative to K0, before any swap) to positions
// 0..nb in order, applied to the global pivot record as they are found.
// Only positions 0..nb and the chosen ones past nb ever move: entry e of
// (tpos, tcol) says position tpos[e] holds original column tcol[e] (e < nb:
// position e; e = nb + j: chosen column j if it lies past nb, else unused).
__global__ __launch_bounds__(64) void swaplist_kernel(const MatDesc *__restrict__ ad, int K0,
                                                      const int *__restrict__ ytp, int ld, int *__restrict__ sw,
                                                      int *__restrict__ piv) {
  const int w = blockIdx.x;
  const MatDesc a = ad[w];
  const int nb = min(QB, a.n - K0);
  if (nb <= 0) return;
  const int lane = threadIdx.x;
  const int *ch = ytp + (size_t)w * ld;
  __shared__ int tpos[2 * QB], tcol[2 * QB];
  if (lane < nb) {
    tpos[lane] = lane;
    tcol[lane] = lane;
  } else if (lane < 2 * nb) {
    const int c = ch[lane - nb];
    tpos[lane] = c >= nb ? c : -1;
    tcol[lane] = c;
  } else if (lane < 2 * QB) {
    tpos[lane] = -1;
  }
  __syncthreads();
  int *pv = piv + (size_t)w * ld + K0;
  for (int i = 0; i < nb; ++i) {
    const int c = ch[i];
    const bool hit = lane < 2 * QB && tpos[lane] >= 0 && tcol[lane] == c;
    const unsigned long long m = __ballot(hit);
    const int e = __ffsll((long long)m) - 1;   // every chosen column is tracked
    const int p = tpos[e];
    if (lane == 0) {
      sw[w * QB + i] = p;
      if (p != i) {
        tcol[e] = tcol[i];
        tcol[i] = c;
        const int t = pv[i];
        pv[i] = pv[p];
        pv[p] = t;
      }
    }
    __syncthreads();
  }
}

// The swaps of swaplist_kernel applied to every row of columns K0.. of the
// matrices d (one thread a row, the swaps in order)
__global__ __launch_bounds__(256) void colswap_kernel(const MatDesc *__restrict__ dd, const MatDesc *__restrict__ ad,
                                                      int K0, const int *__restrict__ sw) {
  const MatDesc d = dd[blockIdx.y];
  const int nb = min(QB, ad[blockIdx.y].n - K0);
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (nb <= 0 || r >= d.m) return;
  const int *s = sw + blockIdx.y * QB;
  for (int i = 0; i < nb; ++i) {
    const int p = s[i];
    if (p != i) {
      double2 *ci = d.a + (size_t)(K0 + i) * d.lda + r, *cp = d.a + (size_t)(K0 + p) * d.lda + r;
      const double2 t = *ci;
      *ci = *cp;
      *cp = t;
    }
  }
}

// Y[:, K0 + nb ..] -= (Y1 R11^{-1}) R12 after the block's QR: Z = Y1 R11^{-1}
// by forward substitution in every workgroup (a column of Z whose pivot
// R11[j][j] is below 1e-14 |R11[0][0]| is dropped: the block's remaining
// columns are then negligible and the sketch only ranks them), then 64
// columns of Y2 a workgroup.
__global__ __launch_bounds__(256) void sketch_update_kernel(const MatDesc *__restrict__ ad, int K0,
                                                            double2 *__restrict__ Y, size_t ystride) {
  const MatDesc a = ad[blockIdx.y];
  const int nb = min(QB, a.n - K0);
  const int c0 = K0 + nb + blockIdx.x * 64;
  if (nb <= 0 || c0 >= a.n) return;
  const int tid = threadIdx.x;
  __shared__ double2 R11[QB][QB + 1];
  __shared__ double2 Z[SL][QB + 1];
  __shared__ double2 R12[QB][65];
  double2 *y = Y + blockIdx.y * ystride;
  for (int e = tid; e < QB * QB; e += 256) {
    const int i = e % QB, j = e / QB;
    R11[i][j] = (i < nb && j < nb && i <= j) ? a.a[(size_t)(K0 + j) * a.lda + K0 + i] : cz(0.0, 0.0);
  }
  for (int e = tid; e < QB * 64; e += 256) {
    const int i = e % QB, q = e / QB, c = c0 + q;
    R12[i][q] = (i < nb && c < a.n) ? a.a[(size_t)c * a.lda + K0 + i] : cz(0.0, 0.0);
  }
  __syncthreads();
  if (tid < SL) {
    const double tiny = 1e-14 * sqrt(cabs2(R11[0][0]));
    for (int j = 0; j < nb; ++j) {
      double2 z = y[(size_t)(K0 + j) * SL + tid];
      for (int t = 0; t < j; ++t) z = csub(z, cmul(Z[tid][t], R11[t][j]));
      const double2 dj = R11[j][j];
      const double dd = cabs2(dj);
      Z[tid][j] = sqrt(dd) > tiny ? cz((z.x * dj.x + z.y * dj.y) / dd, (z.y * dj.x - z.x * dj.y) / dd)
                                  : cz(0.0, 0.0);
    }
  }
  __syncthreads();
  const int q = tid & 63, g = tid >> 6, c = c0 + q;
  if (c < a.n) {
    for (int i = g; i < SL; i += 4) {
      double2 acc = cz(0.0, 0.0);
      for (int j = 0; j < nb; ++j) cfma(acc, Z[i][j], R12[j][q]);
      double2 *yc = y + (size_t)c * SL + i;
      *yc = csub(*yc, acc);
    }
  }
}

}  // namespace

void qrcp_sketched(const MatDesc *descs, const std::vector<MatDesc> &h, int *piv, int ld, hipStream_t s) {
  const int W = (int)h.size();
  int nmax = 0, mmax = 0;
  for (const auto &d : h) {
    nmax = std::max(nmax, d.n);
    mmax = std::max(mmax, d.m);
  }
  if (W == 0 || nmax == 0) return;
  MFS_REQUIRE(ld >= nmax, "sketched QRCP: pivot stride below the widest matrix");
  const size_t ystride = (size_t)SL * nmax;
  const int ldo = round_up(mmax, 64);
  DevBuf om((size_t)SL * ldo * sizeof(double)), Y(W * ystride * sizeof(double2)),
      yt(W * ystride * sizeof(double2)), ytau((size_t)W * QB * sizeof(double2)),
      ytn((size_t)W * ld * sizeof(double)), ytp((size_t)W * ld * sizeof(int)), sw((size_t)W * QB * sizeof(int)),
      ydesc(W * sizeof(MatDesc)), tdesc;
  // descriptors: the sketch (SL x n) and, per block, its remaining columns
  std::vector<MatDesc> hy(W);
  for (int w = 0; w < W; ++w) {
    MatDesc d{};
    d.a = Y.as<double2>() + w * ystride;
    d.m = SL; d.n = h[w].n; d.lda = SL;
    hy[w] = d;
  }
  HIP_CHECK(hipMemcpyAsync(ydesc.p, hy.data(), W * sizeof(MatDesc), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(omega_kernel, dim3(256), dim3(256), 0, s, om.as<double>(), ldo, mmax);
  hipLaunchKernelGGL(sketch_kernel, dim3(cdiv(nmax, 64), W), dim3(256), 0, s, descs, om.as<double>(), ldo,
                     Y.as<double2>(), ystride);
  HIP_CHECK(hipGetLastError());
  // the remaining columns' sketch of every block as a matrix of its own
  const int nblk = cdiv(nmax, QB);
  std::vector<MatDesc> ht((size_t)nblk * W);
  for (int b = 0; b < nblk; ++b)
    for (int w = 0; w < W; ++w) {
      MatDesc d{};
      d.a = yt.as<double2>() + w * ystride;
      d.m = SL; d.n = std::max(0, h[w].n - b * QB); d.lda = SL;
      d.tau = ytau.as<double2>() + (size_t)w * QB;
      ht[(size_t)b * W + w] = d;
    }
  tdesc.alloc(ht.size() * sizeof(MatDesc));
  HIP_CHECK(hipMemcpyAsync(tdesc.p, ht.data(), ht.size() * sizeof(MatDesc), hipMemcpyHostToDevice, s));
  QRPanels32 qr(descs, h);
  for (int K0 = 0; K0 < nmax; K0 += QB) {
    const MatDesc *td = tdesc.as<MatDesc>() + (size_t)(K0 / QB) * W;
    hipLaunchKernelGGL(ycopy_kernel, dim3(cdiv(nmax - K0, 4), W), dim3(256), 0, s, descs, K0, Y.as<double2>(),
                       ystride, yt.as<double2>(), ytn.as<double>(), ytp.as<int>(), ld);
    const int steps = std::min(QB, nmax - K0);
    for (int k = 0; k < steps; ++k) launch_qrcp_step(td, W, nmax - K0, k, ytn.as<double>(), ytp.as<int>(), ld, s);
    hipLaunchKernelGGL(swaplist_kernel, dim3(W), dim3(64), 0, s, descs, K0, ytp.as<int>(), ld, sw.as<int>(), piv);
    hipLaunchKernelGGL(colswap_kernel, dim3(cdiv(mmax, 256), W), dim3(256), 0, s, descs, descs, K0, sw.as<int>());
    hipLaunchKernelGGL(colswap_kernel, dim3(1, W), dim3(64), 0, s, ydesc.as<MatDesc>(), descs, K0, sw.as<int>());
    HIP_CHECK(hipGetLastError());
    qr.panel(K0, s);
    if (K0 + QB < nmax)
      hipLaunchKernelGGL(sketch_update_kernel, dim3(cdiv(nmax - K0 - QB, 64), W), dim3(256), 0, s, descs, K0,
                         Y.as<double2>(), ystride);
    HIP_CHECK(hipGetLastError());
  }
  HIP_CHECK(hipStreamSynchronize(s));   // the host descriptor copies above are gone on return
}

}  // namespace mfs
