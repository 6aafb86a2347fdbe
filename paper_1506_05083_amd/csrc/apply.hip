// Solution-operator apply A^+ x = W (U^H x), W = V S^+ (Sec. 4.2: the
// pseudoinverse is never formed, the two factors are applied in turn).
//
// Mode 0 (one-body operator): the distinct block of mode d serves bins d and
// P-d (A'_{-n} = A'_n), so every block multiplies 2 nrhs columns at once (one
// for d = 0 and d = P/2): a small batched GEMM whose cost is reading U and W
// from HBM once per call.  Mode 1 (periodizing matrix Q): one matrix per
// right-hand side.
//
// stage 1: Y[mat][c][i] = sum_m conj(U[m][i]) x_c[m], 16 rows of Y a
//          workgroup, 48-row chunks of U and X staged through LDS;
// stage 2: out_c[jj] = sum_i W[jj][i] Y[c][i], 16 output rows a workgroup,
//          64-column chunks of W and Y staged through LDS.
// (Small blocks, e.g. 33 modes of 240 x 200: many narrow workgroups and few
// chunks, so that the call is not a chain of dependent load latencies.)
// Mode 1 has a single right-hand side per matrix, so both stages are
// matrix-vector products bound by streaming U and W from HBM: stage 1 gives
// every column of U its own wave (a dot product with x), stage 2 gives every
// 64 output rows eight waves that split the sum over i and meet in LDS.
#include "internal.hpp"

namespace mfs {
namespace {

constexpr int MAXC = 32;  // columns per call (2 * nrhs for mode 0)
constexpr int S1I = 16;   // stage 1: columns of U a workgroup
constexpr int KC1 = 48;   // stage 1: rows of U and x a chunk
constexpr int S2R = 16;   // stage 2: output rows a workgroup
constexpr int KC2 = 64;   // stage 2: columns of W a chunk

__device__ inline int ncols_of(const PinvJob &j, int mat) {
  if (j.mode == 1) return 1;
  const int nsign = (mat == 0 || 2 * mat == j.P) ? 1 : 2;
  return j.nrhs * nsign;
}

__device__ inline size_t col_offset(const PinvJob &j, int mat, int c, int len, int ld) {
  if (j.mode == 1) return (size_t)mat * ld;
  const int nsign = (mat == 0 || 2 * mat == j.P) ? 1 : 2;
  const int rhs = c / nsign, s = c % nsign;
  const int bin = s ? j.P - mat : mat;
  return ((size_t)rhs * j.P + bin) * len;
}

__global__ __launch_bounds__(256) void pinv_stage1(PinvJob j) {
  const int mat = blockIdx.y;
  const MatDesc d = j.descs[mat];
  const int r = d.rank[0];
  const int i0 = blockIdx.x * S1I;
  if (i0 >= r) return;
  const int nc = ncols_of(j, mat);
  __shared__ double2 Us[S1I][KC1 + 1];
  __shared__ double2 Xs[MAXC][KC1 + 1];
  const int tid = threadIdx.x;
  const int ii = tid % S1I, cg = tid / S1I;   // column i0 + ii of U, right-hand sides cg + 16 t
  double2 acc[MAXC / 16];
#pragma unroll
  for (int t = 0; t < MAXC / 16; ++t) acc[t] = cz(0.0, 0.0);
  for (int m0 = 0; m0 < d.m; m0 += KC1) {
    // coalesced down the columns of U and of the right-hand sides
    for (int idx = tid; idx < KC1 * S1I; idx += 256) {
      const int mm = idx % KC1, c = idx / KC1;
      const int m = m0 + mm, i = i0 + c;
      Us[c][mm] = (m < d.m && i < r) ? d.u[(size_t)i * d.lda + m] : cz(0.0, 0.0);
    }
    for (int idx = tid; idx < KC1 * nc; idx += 256) {
      const int mm = idx % KC1, c = idx / KC1;
      const int m = m0 + mm;
      Xs[c][mm] = m < d.m ? j.x[col_offset(j, mat, c, d.m, j.ldx) + m] : cz(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll 4
    for (int mm = 0; mm < KC1; ++mm) {
      const double2 u = Us[ii][mm];
#pragma unroll
      for (int t = 0; t < MAXC / 16; ++t)
        if (cg + 16 * t < nc) cfmac(acc[t], u, Xs[cg + 16 * t][mm]);
    }
    __syncthreads();
  }
  const int i = i0 + ii;
  if (i < r) {
    double2 *y = j.ywork + (size_t)mat * j.maxcols * j.maxr;
#pragma unroll
    for (int t = 0; t < MAXC / 16; ++t) {
      const int c = cg + 16 * t;
      if (c < nc) y[(size_t)c * j.maxr + i] = acc[t];
    }
  }
}

__global__ __launch_bounds__(256) void pinv_stage2(PinvJob j) {
  const int mat = blockIdx.y;
  const MatDesc d = j.descs[mat];
  const int r = d.rank[0];
  const int nc = ncols_of(j, mat);
  const int n = d.n;
  const int jj0 = blockIdx.x * S2R;
  if (jj0 >= n) return;
  __shared__ double2 Ws[KC2][S2R + 1];
  __shared__ double2 Ys[MAXC][KC2 + 1];
  const int tid = threadIdx.x;
  const int jr = tid % S2R, cg = tid / S2R;   // output row jj0 + jr, right-hand sides cg + 16 t
  double2 acc[MAXC / 16];
#pragma unroll
  for (int t = 0; t < MAXC / 16; ++t) acc[t] = cz(0.0, 0.0);
  const double2 *y = j.ywork + (size_t)mat * j.maxcols * j.maxr;
  for (int i0 = 0; i0 < r; i0 += KC2) {
    for (int idx = tid; idx < KC2 * S2R; idx += 256) {
      const int rr = idx % S2R, ii = idx / S2R;
      const int i = i0 + ii, row = jj0 + rr;
      Ws[ii][rr] = (i < r && row < n) ? d.w[(size_t)i * d.ldg + row] : cz(0.0, 0.0);
    }
    for (int idx = tid; idx < KC2 * nc; idx += 256) {
      const int ii = idx % KC2, c = idx / KC2;
      const int i = i0 + ii;
      Ys[c][ii] = i < r ? y[(size_t)c * j.maxr + i] : cz(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll 4
    for (int ii = 0; ii < KC2; ++ii) {
      const double2 w = Ws[ii][jr];
#pragma unroll
      for (int t = 0; t < MAXC / 16; ++t)
        if (cg + 16 * t < nc) cfma(acc[t], w, Ys[cg + 16 * t][ii]);
    }
    __syncthreads();
  }
  const int row = jj0 + jr;
  if (row < n) {
#pragma unroll
    for (int t = 0; t < MAXC / 16; ++t) {
      const int c = cg + 16 * t;
      if (c < nc) j.out[col_offset(j, mat, c, n, j.ldo) + row] = acc[t];
    }
  }
}

constexpr int S2W = 8;   // waves per workgroup in the mode-1 stage 2

// mode 1, stage 1: y[mat][i] = sum_m conj(U[m][i]) x[mat][m], one wave per column i
__global__ __launch_bounds__(256) void pinv_gemvh_kernel(PinvJob j) {
  const int mat = blockIdx.y;
  const MatDesc d = j.descs[mat];
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= d.rank[0]) return;
  const int lane = threadIdx.x & 63;
  const double2 *u = d.u + (size_t)i * d.lda;
  const double2 *x = j.x + (size_t)mat * j.ldx;
  double2 a0 = cz(0.0, 0.0), a1 = cz(0.0, 0.0), a2 = cz(0.0, 0.0), a3 = cz(0.0, 0.0);
  int m = lane;
  for (; m + 192 < d.m; m += 256) {
    const double2 u0 = u[m], u1 = u[m + 64], u2 = u[m + 128], u3 = u[m + 192];
    const double2 x0 = x[m], x1 = x[m + 64], x2 = x[m + 128], x3 = x[m + 192];
    cfmac(a0, u0, x0);
    cfmac(a1, u1, x1);
    cfmac(a2, u2, x2);
    cfmac(a3, u3, x3);
  }
  for (; m < d.m; m += 64) cfmac(a0, u[m], x[m]);
  double2 acc = cadd(cadd(a0, a1), cadd(a2, a3));
  acc = wave_sum(acc);
  if (lane == 0) j.ywork[(size_t)mat * j.maxcols * j.maxr + i] = acc;
}

// mode 1, stage 2: out[mat][row] = sum_{i < rank} W[row][i] y[i]
__global__ __launch_bounds__(64 * S2W) void pinv_gemv_kernel(PinvJob j) {
  const int mat = blockIdx.y;
  const MatDesc d = j.descs[mat];
  const int r = d.rank[0];
  const int row = blockIdx.x * 64 + (threadIdx.x & 63);
  const int wv = threadIdx.x >> 6;
  __shared__ double2 part[S2W][64];
  const double2 *y = j.ywork + (size_t)mat * j.maxcols * j.maxr;
  double2 a0 = cz(0.0, 0.0), a1 = cz(0.0, 0.0);
  if (row < d.n) {
    const double2 *w = d.w + row;
    int i = wv;
    for (; i + S2W < r; i += 2 * S2W) {
      cfma(a0, w[(size_t)i * d.ldg], y[i]);
      cfma(a1, w[(size_t)(i + S2W) * d.ldg], y[i + S2W]);
    }
    for (; i < r; i += S2W) cfma(a0, w[(size_t)i * d.ldg], y[i]);
  }
  part[wv][threadIdx.x & 63] = cadd(a0, a1);
  __syncthreads();
  if (wv == 0 && row < d.n) {
    double2 t = part[0][threadIdx.x];
#pragma unroll
    for (int g = 1; g < S2W; ++g) t = cadd(t, part[g][threadIdx.x]);
    j.out[(size_t)mat * j.ldo + row] = t;
  }
}

// V[r][k0 .. k0 + N) of the panel at k0 (unit diagonal, zeros above it and
// past the last column): N loads issued together, masked ones reading the
// matrix's first element
template <int N>
__device__ inline void vpanel(const MatDesc &d, int r, bool live, int k0, double2 (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const int c = k0 + i;
    v[i] = ld_or0(d.a, (size_t)(c < d.n ? c : 0) * d.lda + (live ? r : 0), live && c < d.n && r > c);
  }
#pragma unroll
  for (int i = 0; i < N; ++i)
    if (live && r == k0 + i && k0 + i < d.n) v[i] = cz(1.0, 0.0);
}

// Q^H x for matrices kept as their Householder QR (reflectors below the
// diagonal, the compact-WY T of every NB-column panel): Q^H = H_n^H ... H_1^H
// applied panel after panel, x <- x - V T^H (V^H x).  Launch p (workgroup:
// QHR rows of one matrix) finishes panel p - 1 (the slices' partial sums of
// V^H x added, times T^H, subtracted from its rows) and forms panel p's
// partial sums over its rows; the launch after the last panel writes
// y = (Q^H x)[0, n) to the apply's work vector.  The slices' partials are
// double-buffered by panel parity: [2][mat][slice][NB].
template <int NB>
__global__ __launch_bounds__(QHR) void qh_panel_kernel(const MatDesc *__restrict__ descs, int p, int npan,
                                                       const double2 *__restrict__ xin, int ldx,
                                                       double2 *__restrict__ xw, double2 *__restrict__ part,
                                                       int nslmax, double2 *__restrict__ y, int ldy) {
  const MatDesc d = descs[blockIdx.y];
  const int slice = blockIdx.x, r0 = slice * QHR;
  if (r0 >= d.m) return;
  const int nsl = (d.m + QHR - 1) / QHR;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int r = r0 + tid;
  const bool live = r < d.m;
  double2 xr = live ? (p == 0 ? xin : xw)[(size_t)blockIdx.y * ldx + r] : cz(0.0, 0.0);
  __shared__ double2 ws[NB], tv[NB];
  __shared__ double2 red[QHR / 64][NB];
  __shared__ double2 sred[QHR];
  __shared__ double2 Ts[NB][NB + 1];
  // V[r][k0 + i .. + 16) of the panel at k0: 16 loads issued together (masked
  // ones read the matrix's first element), then the unit diagonal and zeros
  auto vload = [&](int k0, int i0, double2 (&v)[16]) {
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int c = k0 + i0 + i;
      v[i] = ld_or0(d.a, (size_t)(c < d.n ? c : 0) * d.lda + (live ? r : 0), live && c < d.n && r > c);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i)
      if (live && r == k0 + i0 + i && k0 + i0 + i < d.n) v[i] = cz(1.0, 0.0);
  };
  if constexpr (NB <= 32) {
    // both panels' reflectors loaded at once, before the partials' sum
    const int kp = (p - 1) * NB, k0 = p * NB;
    const bool fin = p > 0 && kp < d.n, par = p < npan && k0 < d.n;
    double2 vp[NB], vc[NB];
    if (fin) vpanel<NB>(d, r, live, kp, vp);
    if (par) vpanel<NB>(d, r, live, k0, vc);
    if (fin) {
      const double2 *pin = part + ((size_t)((p - 1) & 1) * gridDim.y + blockIdx.y) * nslmax * NB;
      constexpr int G = QHR / NB;
      {
        const int i = tid % NB, g0 = tid / NB;
        double2 t = cz(0.0, 0.0);
#pragma unroll 4
        for (int sl = g0; sl < nsl; sl += G) t = cadd(t, pin[(size_t)sl * NB + i]);
        sred[tid] = t;   // [g0][i]
      }
      const double2 *T = d.T + (size_t)(kp / NB) * NB * NB;   // column-major, upper
      for (int e = tid; e < NB * NB; e += QHR) Ts[e / NB][e % NB] = T[e];   // Ts[i][h] = T[h][i]
      __syncthreads();
      if (tid < NB) {
        double2 t = sred[tid];
#pragma unroll
        for (int g = 1; g < G; ++g) t = cadd(t, sred[g * NB + tid]);
        ws[tid] = t;
      }
      __syncthreads();
      if (tid < NB) {
        double2 t = cz(0.0, 0.0);
        for (int h = 0; h <= tid; ++h) cfmac(t, Ts[tid][h], ws[h]);   // (T^H w)_i
        tv[tid] = t;
      }
      __syncthreads();
      if (live && r >= kp) {
#pragma unroll
        for (int i = 0; i < NB; ++i) xr = csub(xr, cmul(vp[i], tv[i]));
      }
    }
    if (par) {
      double2 *pout = part + ((size_t)(p & 1) * gridDim.y + blockIdx.y) * nslmax * NB + (size_t)slice * NB;
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const double2 v = vc[i];
        vc[i] = cz(0.0, 0.0);
        cfmac(vc[i], v, xr);   // conj(V[r][i]) x[r]
      }
      lane_column_sums<NB>(vc, lane);
      if (lane < NB) red[wv][lane] = vc[0];
      __syncthreads();
      if (tid < NB) {
        double2 t = red[0][tid];
#pragma unroll
        for (int w = 1; w < QHR / 64; ++w) t = cadd(t, red[w][tid]);
        pout[tid] = t;
      }
    }
  } else {
    if (p > 0) {
      const int kp = (p - 1) * NB;
      if (kp < d.n) {
        const double2 *pin = part + ((size_t)((p - 1) & 1) * gridDim.y + blockIdx.y) * nslmax * NB;
        // the slices' partials summed by every thread (column tid % NB, every
        // G-th slice, loads in flight together), then across the G groups;
        // T staged through LDS alongside
        constexpr int G = QHR / NB;
        {
          const int i = tid % NB, g0 = tid / NB;
          double2 t = cz(0.0, 0.0);
  #pragma unroll 4
          for (int sl = g0; sl < nsl; sl += G) t = cadd(t, pin[(size_t)sl * NB + i]);
          sred[tid] = t;   // [g0][i]
        }
        const double2 *T = d.T + (size_t)(kp / NB) * NB * NB;   // column-major, upper
        for (int e = tid; e < NB * NB; e += QHR) Ts[e / NB][e % NB] = T[e];   // Ts[i][h] = T[h][i]
        __syncthreads();
        if (tid < NB) {
          double2 t = sred[tid];
  #pragma unroll
          for (int g = 1; g < G; ++g) t = cadd(t, sred[g * NB + tid]);
          ws[tid] = t;
        }
        __syncthreads();
        if (tid < NB) {
          double2 t = cz(0.0, 0.0);
          for (int h = 0; h <= tid; ++h) cfmac(t, Ts[tid][h], ws[h]);   // (T^H w)_i
          tv[tid] = t;
        }
        __syncthreads();
        if (live && r >= kp) {
          for (int i0 = 0; i0 < NB; i0 += 16) {
            double2 v[16];
            vload(kp, i0, v);
  #pragma unroll
            for (int i = 0; i < 16; ++i) xr = csub(xr, cmul(v[i], tv[i0 + i]));
          }
        }
      }
    }
    if (p < npan) {
      const int k0 = p * NB;
      double2 *pout = part + ((size_t)(p & 1) * gridDim.y + blockIdx.y) * nslmax * NB + (size_t)slice * NB;
      if (k0 < d.n) {
        constexpr int HB = NB < 32 ? NB : 32;   // columns summed together (registers)
  #pragma unroll
        for (int h0 = 0; h0 < NB; h0 += HB) {
          double2 v[HB];
  #pragma unroll
          for (int i0 = 0; i0 < HB; i0 += 16) {
            double2 vv[16];
            vload(k0, h0 + i0, vv);
  #pragma unroll
            for (int i = 0; i < 16; ++i) {
              v[i0 + i] = cz(0.0, 0.0);
              cfmac(v[i0 + i], vv[i], xr);   // conj(V[r][i]) x[r]
            }
          }
          lane_column_sums<HB>(v, lane);
          if (lane < HB) red[wv][h0 + lane] = v[0];
        }
        __syncthreads();
        if (tid < NB) {
          double2 t = red[0][tid];
  #pragma unroll
          for (int w = 1; w < QHR / 64; ++w) t = cadd(t, red[w][tid]);
          pout[tid] = t;
        }
      }
    }
  }
  if (live) {
    if (p < npan) xw[(size_t)blockIdx.y * ldx + r] = xr;
    else if (r < d.n) y[(size_t)blockIdx.y * ldy + r] = xr;
  }
}

template <int NB>
void qh_apply_t(const MatDesc *descs, int nmat, int mmax, int nmax, const double2 *x, int ldx, double2 *xw,
                double2 *part, int nslmax, double2 *y, int ldy, hipStream_t s) {
  const int npan = cdiv(nmax, NB);
  for (int p = 0; p <= npan; ++p)
    hipLaunchKernelGGL(qh_panel_kernel<NB>, dim3(cdiv(mmax, QHR), nmat), dim3(QHR), 0, s, descs, p, npan, x, ldx,
                       xw, part, nslmax, y, ldy);
  HIP_CHECK(hipGetLastError());
}

}  // namespace

void launch_pinv_apply(const PinvJob &j, hipStream_t s) {
  MFS_REQUIRE(j.maxcols <= MAXC, "too many right-hand sides in one apply (max 16 per call)");
  if (j.mode == 1) {
    hipLaunchKernelGGL(pinv_gemvh_kernel, dim3(cdiv(j.maxr, 4), j.nmat), dim3(256), 0, s, j);
    HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(pinv_gemv_kernel, dim3(cdiv(j.maxn, 64), j.nmat), dim3(64 * S2W), 0, s, j);
    HIP_CHECK(hipGetLastError());
    return;
  }
  hipLaunchKernelGGL(pinv_stage1, dim3(cdiv(j.maxr, S1I), j.nmat), dim3(256), 0, s, j);
  HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(pinv_stage2, dim3(cdiv(j.maxn, S2R), j.nmat), dim3(256), 0, s, j);
  HIP_CHECK(hipGetLastError());
}

}  // namespace mfs

namespace mfs {

size_t qh_apply_work(int nmat, int mmax, int ldx) {
  return ((size_t)nmat * ldx + 2 * (size_t)nmat * cdiv(mmax, QHR) * 64) * sizeof(double2);
}

void launch_qh_apply(const MatDesc *descs, int nmat, int mmax, int nmax, int nb, const double2 *x, int ldx,
                     double2 *work, double2 *y, int ldy, hipStream_t s) {
  double2 *xw = work, *part = work + (size_t)nmat * ldx;
  const int nslmax = cdiv(mmax, QHR);
  switch (nb) {
    case 16: qh_apply_t<16>(descs, nmat, mmax, nmax, x, ldx, xw, part, nslmax, y, ldy, s); break;
    case 32: qh_apply_t<32>(descs, nmat, mmax, nmax, x, ldx, xw, part, nslmax, y, ldy, s); break;
    case 64: qh_apply_t<64>(descs, nmat, mmax, nmax, x, ldx, xw, part, nslmax, y, ldy, s); break;
    default: MFS_THROW(MFS_EINVAL, "reflector apply: panel width must be 16, 32 or 64");
  }
}

void launch_pinv_apply_w(const PinvJob &j, hipStream_t s) {
  MFS_REQUIRE(j.mode == 1, "W-only apply is the one-matrix-per-rhs form");
  hipLaunchKernelGGL(pinv_gemv_kernel, dim3(cdiv(j.maxn, 64), j.nmat), dim3(64 * S2W), 0, s, j);
  HIP_CHECK(hipGetLastError());
}

}  // namespace mfs
