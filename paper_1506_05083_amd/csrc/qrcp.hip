// Blocked column-pivoted Householder QR of batched square triangles (the
// rank-revealing step of the truncated pseudoinverses, Sec. 4.2), the panel
// form of LAPACK's xGEQP3 (xLAQPS): within a panel of QP columns the
// trailing matrix is not updated; every step keeps the updates it owes in
// F (n x QP per matrix, F(c, i) = tau_i a_c^{(i)H} v_i, so that the
// updated column is a_c - V F(c, :)^H), updates only the pivot column and
// the pivot row, and downdates the column norms from the updated pivot
// row.  After the panel one matrix-core product applies all of it to the
// trailing block.  Per step the trailing matrix is read once (for
// F(:, j)); the unblocked form reads it twice and writes it once.
//
//   bqp_pivot_kernel   (one workgroup per matrix) the column of largest
//                      norm to position k (columns, F rows, norms, pivots
//                      swapped), its deferred updates applied, its
//                      reflector formed, aux_i = v_i^H v_k for i < j;
//   bqp_column_kernel  (one wave per trailing column) F(c, j), the pivot
//                      row's entry A(k, c) updated, the norm downdated (or
//                      recomputed from the updated column when cancellation
//                      makes the downdate unreliable, LAPACK's test);
//   bqp_trail_kernel   A(r, c) -= sum_i V(r, i) conj(F(c, i)) for the rows
//                      and columns past the panel (FP64 matrix cores).
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.hpp"

namespace mfs {
namespace {

constexpr int QP = 32;    // panel width (the T factors are built per 32 columns as well)
constexpr int PT = 512;   // threads of the pivot kernel

__global__ __launch_bounds__(PT) void bqp_pivot_kernel(const MatDesc *__restrict__ descs, int k0, int j,
                                                       double *__restrict__ vn1, double *__restrict__ vn2,
                                                       int *__restrict__ piv, double2 *__restrict__ F,
                                                       double2 *__restrict__ aux, int ld) {
  const MatDesc d = descs[blockIdx.x];
  const int k = k0 + j;
  if (k >= d.n) return;
  const size_t mo = (size_t)blockIdx.x * ld;
  double *n1 = vn1 + mo, *n2 = vn2 + mo;
  int *pv = piv + mo;
  double2 *Fm = F + mo * QP;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  __shared__ double rv[PT / 64];
  __shared__ int ri[PT / 64];
  __shared__ double2 red[PT / 64][QP];
  __shared__ double2 fk[QP];
  __shared__ int s_p;
  __shared__ double s_sum;
  // 1. pivot: largest remaining norm, ties to the lower index
  double best = -1.0;
  int bi = k;
  for (int c = k + tid; c < d.n; c += PT) {
    const double v = n1[c];
    if (v > best) { best = v; bi = c; }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(best, o, 64);
    const int oi = __shfl_xor(bi, o, 64);
    if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
  }
  if (lane == 0) { rv[wv] = best; ri[wv] = bi; }
  __syncthreads();
  if (tid == 0) {
    double b = rv[0];
    int i = ri[0];
    for (int w = 1; w < PT / 64; ++w)
      if (rv[w] > b || (rv[w] == b && ri[w] < i)) { b = rv[w]; i = ri[w]; }
    s_p = i;
  }
  __syncthreads();
  const int p = s_p;
  if (p != k) {
    double2 *ck = d.a + (size_t)k * d.lda, *cp = d.a + (size_t)p * d.lda;
    for (int r = tid; r < d.m; r += PT) {
      const double2 t = ck[r];
      ck[r] = cp[r];
      cp[r] = t;
    }
    if (tid < j) {
      const double2 t = Fm[(size_t)k * QP + tid];
      Fm[(size_t)k * QP + tid] = Fm[(size_t)p * QP + tid];
      Fm[(size_t)p * QP + tid] = t;
    }
    if (tid == 0) {
      double t = n1[k]; n1[k] = n1[p]; n1[p] = t;
      t = n2[k]; n2[k] = n2[p]; n2[p] = t;
      const int ti = pv[k]; pv[k] = pv[p]; pv[p] = ti;
    }
  }
  __syncthreads();
  if (tid < j) fk[tid] = Fm[(size_t)k * QP + tid];
  __syncthreads();
  // 2. the pivot column's deferred updates, rows k..m-1: a -= V F(k, :)^H
  double2 *col = d.a + (size_t)k * d.lda;
  if (j > 0) {
    for (int r = k + tid; r < d.m; r += PT) {
      double2 x = col[r];
      for (int i = 0; i < j; ++i) x = csub(x, cmul(d.a[(size_t)(k0 + i) * d.lda + r], cconj(fk[i])));
      col[r] = x;
    }
    __syncthreads();
  }
  // 3. its reflector (LAPACK's zlarfg convention)
  double s = 0.0;
  for (int r = k + 1 + tid; r < d.m; r += PT) s += cabs2(col[r]);
  s = wave_sum(s);
  if (lane == 0) rv[wv] = s;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int w = 0; w < PT / 64; ++w) t += rv[w];
    s_sum = t;
  }
  __syncthreads();
  const double ssum = s_sum;
  const double2 alpha = col[k];
  double2 tau = cz(0.0, 0.0);
  if (!(ssum == 0.0 && alpha.y == 0.0)) {
    const double beta = -copysign(sqrt(alpha.x * alpha.x + alpha.y * alpha.y + ssum), alpha.x);
    tau = cz((beta - alpha.x) / beta, -alpha.y / beta);
    const double2 den = cz(alpha.x - beta, alpha.y);
    const double dd = cabs2(den);
    const double2 scal = cz(den.x / dd, -den.y / dd);
    for (int r = k + 1 + tid; r < d.m; r += PT) col[r] = cmul(col[r], scal);
    __syncthreads();
    if (tid == 0) col[k] = cz(beta, 0.0);
  }
  if (tid == 0) d.tau[k] = tau;
  __syncthreads();
  // 4. aux_i = v_i^H v_k over rows k..m-1 (v_k(k) = 1; v_i(k) = a(k, k0 + i))
  if (j > 0) {
    double2 acc[QP];
#pragma unroll
    for (int i = 0; i < QP; ++i) acc[i] = cz(0.0, 0.0);
    for (int r = k + tid; r < d.m; r += PT) {
      const double2 vk = r == k ? cz(1.0, 0.0) : col[r];
#pragma unroll
      for (int i = 0; i < QP; ++i)
        if (i < j) cfmac(acc[i], d.a[(size_t)(k0 + i) * d.lda + r], vk);
    }
#pragma unroll
    for (int i = 0; i < QP; ++i) {
      if (i < j) {
        const double2 t = wave_sum(acc[i]);
        if (lane == 0) red[wv][i] = t;
      }
    }
    __syncthreads();
    if (tid < j) {
      double2 t = red[0][tid];
      for (int w = 1; w < PT / 64; ++w) t = cadd(t, red[w][tid]);
      aux[(size_t)blockIdx.x * QP + tid] = t;
    }
  }
}

// One wave per column c > k: F(c, j) = tau_k (a_c^H v_k - sum_{i<j} F(c, i)
// aux_i) from the panel-unupdated column, the pivot row's entry
// A(k, c) -= sum_{i<=j} V(k, i) conj(F(c, i)), then the norm of rows k+1..
// downdated (LAPACK's test on the cancellation: below sqrt(eps) of the last
// exact value the norm is recomputed from the updated column).
__global__ __launch_bounds__(256) void bqp_column_kernel(const MatDesc *__restrict__ descs, int k0, int j,
                                                         double *__restrict__ vn1, double *__restrict__ vn2,
                                                         double2 *__restrict__ F, const double2 *__restrict__ aux,
                                                         int ld) {
  const MatDesc d = descs[blockIdx.y];
  const int k = k0 + j;
  const int c = k + 1 + blockIdx.x * 4 + (threadIdx.x >> 6);
  if (k >= d.n || c >= d.n) return;
  const int lane = threadIdx.x & 63;
  const size_t mo = (size_t)blockIdx.y * ld;
  double2 *Fc = F + (mo + c) * QP;
  const double2 *av = aux + (size_t)blockIdx.y * QP;
  const double2 *vk = d.a + (size_t)k * d.lda;
  double2 *a = d.a + (size_t)c * d.lda;
  double2 dot = cz(0.0, 0.0);   // a_c^H v_k
  for (int r = k + lane; r < d.m; r += 64) {
    const double2 v = r == k ? cz(1.0, 0.0) : vk[r];
    cfmac(dot, a[r], v);
  }
  dot = wave_sum(dot);
  double2 corr = cz(0.0, 0.0);
  for (int i = 0; i < j; ++i) cfma(corr, Fc[i], av[i]);
  const double2 fj = cmul(d.tau[k], csub(dot, corr));
  // the pivot row: A(k, c) -= sum_{i<j} a(k, k0 + i) conj(F(c, i)) + conj(F(c, j))
  double2 akc = a[k];
  for (int i = 0; i < j; ++i) akc = csub(akc, cmul(d.a[(size_t)(k0 + i) * d.lda + k], cconj(Fc[i])));
  akc = csub(akc, cconj(fj));
  double nrm = vn1[mo + c];
  bool recompute = false;
  if (nrm != 0.0) {
    double t = sqrt(cabs2(akc)) / nrm;
    t = fmax(0.0, (1.0 + t) * (1.0 - t));
    const double r2 = vn2[mo + c];
    const double t2 = t * (nrm / r2) * (nrm / r2);
    if (t2 <= 1.4901161193847656e-08) recompute = true;   // sqrt(eps)
    else nrm *= sqrt(t);
  }
  if (recompute) {   // wave-uniform: norm of rows k+1.. of a_c - V F(c, 0..j)^H
    double ss = 0.0;
    for (int r = k + 1 + lane; r < d.m; r += 64) {
      double2 x = a[r];
      for (int i = 0; i < j; ++i) x = csub(x, cmul(d.a[(size_t)(k0 + i) * d.lda + r], cconj(Fc[i])));
      x = csub(x, cmul(vk[r], cconj(fj)));
      ss += cabs2(x);
    }
    ss = wave_sum(ss);
    nrm = sqrt(ss);
  }
  if (lane == 0) {
    Fc[j] = fj;
    a[k] = akc;
    vn1[mo + c] = nrm;
    if (recompute) vn2[mo + c] = nrm;
  }
}

// After the panel [k0, k1): A(r, c) -= sum_{i < k1 - k0} V(r, i) conj(F(c, i))
// for rows r >= k1 and columns c >= k1, V(r, i) = a(r, k0 + i) (r > k0 + i).
// Computed transposed on the matrix cores as in the QR's trailing update:
// D[c][r] = sum_i conj(F(c, i)) V(r, i); workgroup 64 rows x 64 columns,
// wave w the columns 16 w .. 16 w + 15.
__global__ __launch_bounds__(256) void bqp_trail_kernel(const MatDesc *__restrict__ descs, int k0, int k1,
                                                        const double2 *__restrict__ F, int ld) {
  const MatDesc d = descs[blockIdx.z];
  const int kend = min(k1, d.n);
  const int nb = kend - k0;
  if (nb <= 0) return;
  const int r0 = kend + blockIdx.x * 64;
  const int cw = kend + blockIdx.y * 64 + 16 * (threadIdx.x >> 6);
  if (r0 >= d.m || cw >= d.n) return;   // a whole wave (cw) or workgroup (r0): no barriers here
  const int lane = threadIdx.x & 63, l16 = lane & 15, k4 = lane >> 4;
  const double2 *Fm = F + (size_t)blockIdx.z * ld * QP;
  dx4 re[4], im[4];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) {
    re[rb] = dx4{0.0, 0.0, 0.0, 0.0};
    im[rb] = re[rb];
  }
  for (int i0 = 0; i0 < nb; i0 += 4) {
    const int i = i0 + k4;
    const int c = cw + l16;
    // A[c][i] = conj(F(c, i)); B[i][r] = V(r, i)
    const double2 f = ld_or0(Fm, (size_t)(c < d.n ? c : 0) * QP + (i < nb ? i : 0), c < d.n && i < nb);
    const double2 fa = cconj(f);
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      const int r = r0 + 16 * rb + l16;
      const double2 v = ld_or0(d.a, (size_t)(k0 + (i < nb ? i : 0)) * d.lda + (r < d.m ? r : 0), i < nb && r < d.m);
      re[rb] = mfma_f64(fa.x, v.x, re[rb]);
      re[rb] = mfma_f64(-fa.y, v.y, re[rb]);
      im[rb] = mfma_f64(fa.x, v.y, im[rb]);
      im[rb] = mfma_f64(fa.y, v.x, im[rb]);
    }
  }
  // lane (l16, k4) holds D[c = cw + k4 + 4 e][r = r0 + 16 rb + l16] in element e
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int c = cw + k4 + 4 * e;
    if (c >= d.n) continue;
    double2 *colp = d.a + (size_t)c * d.lda;
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      const int r = r0 + 16 * rb + l16;
      if (r < d.m) {
        const double2 x = colp[r];
        colp[r] = cz(x.x - re[rb][e], x.y - im[rb][e]);
      }
    }
  }
}

}  // namespace

// Column-pivoted QR of the batch (in place; tau; piv[w][i] the original
// column of position i, updated by the swaps; norms: [w][ld] the columns'
// norms on entry, destroyed).  Panels of 32 columns.
void qrcp_blocked(const MatDesc *descs, const std::vector<MatDesc> &h, double *norms, int *piv, int ld,
                  hipStream_t s) {
  const int W = (int)h.size();
  int nmax = 0, mmax = 0;
  for (const auto &d : h) {
    nmax = std::max(nmax, d.n);
    mmax = std::max(mmax, d.m);
  }
  if (W == 0 || nmax == 0) return;
  DevBuf vn2((size_t)W * ld * sizeof(double)), F((size_t)W * ld * QP * sizeof(double2)),
      aux((size_t)W * QP * sizeof(double2));
  HIP_CHECK(hipMemcpyAsync(vn2.p, norms, (size_t)W * ld * sizeof(double), hipMemcpyDeviceToDevice, s));
  for (int k0 = 0; k0 < nmax; k0 += QP) {
    const int jb = std::min(QP, nmax - k0);
    for (int j = 0; j < jb; ++j) {
      const int k = k0 + j;
      hipLaunchKernelGGL(bqp_pivot_kernel, dim3(W), dim3(PT), 0, s, descs, k0, j, norms, vn2.as<double>(), piv,
                         F.as<double2>(), aux.as<double2>(), ld);
      if (k + 1 < nmax)
        hipLaunchKernelGGL(bqp_column_kernel, dim3(cdiv(nmax - k - 1, 4), W), dim3(256), 0, s, descs, k0, j, norms,
                           vn2.as<double>(), F.as<double2>(), aux.as<double2>(), ld);
    }
    const int k1 = k0 + jb;
    if (k1 < nmax)
      hipLaunchKernelGGL(bqp_trail_kernel, dim3(cdiv(mmax - k1, 64), cdiv(nmax - k1, 64), W), dim3(256), 0, s,
                         descs, k0, k1, F.as<double2>(), ld);
    HIP_CHECK(hipGetLastError());
  }
}

}  // namespace mfs
