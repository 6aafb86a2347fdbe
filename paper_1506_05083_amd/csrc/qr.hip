// Batched blocked Householder QR of complex M x N blocks (the dense
// per-mode least-squares factorisation of Sec. 3, eq. (linsys), and of the
// periodizing matrix Q of Sec. 4.2).
//
// For each panel of NB = 32 columns:
//  * qr_panel_kernel (one workgroup per matrix): unblocked Householder QR of
//    the panel in place (LAPACK's zlarfg convention: H = I - tau v v^H,
//    v(1) = 1, H^H x = beta e_1 with beta real), then the compact-WY factor T
//    with H_1 ... H_nb = I - V T V^H from the Gram matrix V^H V;
//  * qr_block_apply_kernel (many workgroups per matrix, 16 columns each):
//    B <- (I - V T V^H)^H B = B - V T^H (V^H B) on the trailing columns, two
//    passes over 64-row chunks staged in LDS.
// The same block-apply kernel with T in place of T^H, run over the panels in
// reverse, forms U = Q [U_R; 0] for the explicit left singular vectors.
#include "internal.hpp"

namespace mfs {
namespace {

constexpr int NB = kQRNB;
constexpr int TC = 16;   // target columns per workgroup
constexpr int RC = 64;   // rows per LDS chunk

__device__ inline double2 vload(const double2 *a, int lda, int k0, int i, int r) {
  // element r of Householder vector i of the panel starting at column k0
  const int c = k0 + i;
  if (r < c) return cz(0.0, 0.0);
  if (r == c) return cz(1.0, 0.0);
  return a[(size_t)c * lda + r];
}

constexpr int PT = 512;    // panel kernel threads (8 waves)

// Block-wide sum of a complex value over PT threads (red: 16 slots).
__device__ inline double2 block_sum(double2 v, double2 *red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double2 t = cz(0.0, 0.0);
#pragma unroll
  for (int i = 0; i < PT / 64; ++i) t = cadd(t, red[i]);
  return t;
}

__global__ __launch_bounds__(PT) void qr_panel_kernel(const MatDesc *__restrict__ descs, int k0) {
  const MatDesc d = descs[blockIdx.x];
  if (k0 >= d.n) return;
  const int nbp = min(NB, d.n - k0);
  const int m = d.m, lda = d.lda;
  double2 *a = d.a;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  __shared__ double2 s_tau[NB];
  __shared__ double2 gram[NB][NB + 1];
  __shared__ double2 tmp[NB];
  __shared__ double2 red[PT / 64];
  __shared__ double2 wred[PT / 64][NB];

  for (int jj = 0; jj < nbp; ++jj) {
    const int j = k0 + jj;
    double2 *col = a + (size_t)j * lda;
    // Householder vector of column j (rows j..m-1), all threads
    double s = 0.0;
    for (int r = j + 1 + tid; r < m; r += PT) s += cabs2(col[r]);
    const double ssum = block_sum(cz(s, 0.0), red).x;
    const double2 alpha = col[j];
    double2 tau = cz(0.0, 0.0);
    if (!(ssum == 0.0 && alpha.y == 0.0)) {
      const double beta = -copysign(sqrt(alpha.x * alpha.x + alpha.y * alpha.y + ssum), alpha.x);
      tau = cz((beta - alpha.x) / beta, -alpha.y / beta);
      const double2 den = cz(alpha.x - beta, alpha.y);
      const double dd = cabs2(den);
      const double2 scal = cz(den.x / dd, -den.y / dd);
      for (int r = j + 1 + tid; r < m; r += PT) col[r] = cmul(col[r], scal);
      __syncthreads();   // alpha read by every thread before it is overwritten
      if (tid == 0) col[j] = cz(beta, 0.0);
    }
    if (tid == 0) {
      s_tau[jj] = tau;
      d.tau[j] = tau;
    }
    __syncthreads();
    // w_c = v^H A[:, c] for the remaining panel columns, one pass over the rows
    const int nc = k0 + nbp - (j + 1);
    if (nc > 0) {
      double2 w[NB];
#pragma unroll
      for (int c = 0; c < NB; ++c) w[c] = cz(0.0, 0.0);
      for (int r = j + tid; r < m; r += PT) {
        const double2 vr = (r == j) ? cz(1.0, 0.0) : col[r];
#pragma unroll
        for (int c = 0; c < NB; ++c)
          if (c < nc) cfmac(w[c], vr, a[(size_t)(j + 1 + c) * lda + r]);
      }
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        if (c < nc) {
          const double2 t = wave_sum(w[c]);
          if (lane == 0) wred[wv][c] = t;
        }
      }
      __syncthreads();
      if (tid < nc) {
        double2 t = cz(0.0, 0.0);
        for (int i = 0; i < PT / 64; ++i) t = cadd(t, wred[i][tid]);
        tmp[tid] = cmul(cconj(s_tau[jj]), t);
      }
      __syncthreads();
      for (int r = j + tid; r < m; r += PT) {
        const double2 vr = (r == j) ? cz(1.0, 0.0) : col[r];
#pragma unroll
        for (int c = 0; c < NB; ++c) {
          if (c < nc) {
            double2 *p = a + (size_t)(j + 1 + c) * lda + r;
            *p = csub(*p, cmul(vr, tmp[c]));
          }
        }
      }
      __syncthreads();
    }
  }

  // Gram matrix of the panel's Householder vectors, G[g][i] = v_g^H v_i, g < i
  const int npairs = nbp * (nbp - 1) / 2;
  for (int pidx = wv; pidx < npairs; pidx += PT / 64) {
    // unrank pidx -> (g, i) with g < i
    int i = 1, base = 0;
    while (base + i <= pidx) { base += i; ++i; }
    const int g = pidx - base;
    double2 acc = cz(0.0, 0.0);
    for (int r = k0 + i + lane; r < m; r += 64)
      cfmac(acc, vload(a, lda, k0, g, r), vload(a, lda, k0, i, r));
    acc = wave_sum(acc);
    if (lane == 0) gram[g][i] = acc;
  }
  __syncthreads();
  // T (forward, columnwise): T[i][i] = tau_i, T[0:i, i] = -tau_i T[0:i,0:i] G[0:i, i].
  // Row h of T is only ever written by thread h, so only tmp needs barriers.
  __shared__ double2 Tsh[NB][NB + 1];
  for (int i = 0; i < nbp; ++i) {
    const double2 ti = s_tau[i];
    if (tid < i) tmp[tid] = cmul(cz(-ti.x, -ti.y), gram[tid][i]);
    __syncthreads();
    if (tid < i) {
      double2 acc = cz(0.0, 0.0);
      for (int g = tid; g < i; ++g) cfma(acc, Tsh[tid][g], tmp[g]);
      Tsh[tid][i] = acc;
    }
    if (tid == i) Tsh[i][i] = ti;
    __syncthreads();
  }
  double2 *T = d.T + (size_t)(k0 / NB) * NB * NB;
  for (int idx = tid; idx < NB * NB; idx += PT) {
    const int r = idx % NB, c = idx / NB;
    T[idx] = (r <= c && c < nbp) ? Tsh[r][c] : cz(0.0, 0.0);
  }
}

// which = 0: B = the matrix itself, columns [k0 + nbp, n), trans = 1 (QR);
// which = 1: B = d.u, columns [0, rank), trans = 0 (form Q [U_R; 0]).
__global__ __launch_bounds__(256) void qr_block_apply_kernel(const MatDesc *__restrict__ descs,
                                                             int k0, int trans, int which) {
  const MatDesc d = descs[blockIdx.x];
  if (k0 >= d.n) return;
  const int nbp = min(NB, d.n - k0);
  const int m = d.m;
  double2 *B;
  int ldb, cbeg, cend;
  if (which == 0) {
    B = d.a; ldb = d.lda; cbeg = k0 + nbp; cend = d.n;
  } else {
    B = d.u; ldb = d.lda; cbeg = 0; cend = d.rank[0];
  }
  const int c0 = cbeg + blockIdx.y * TC;
  if (c0 >= cend) return;
  const int ncol = min(TC, cend - c0);

  __shared__ double2 Vs[RC][NB + 1];
  __shared__ double2 Bs[RC][TC + 1];
  __shared__ double2 Ws[NB][TC + 1];
  __shared__ double2 Ts[NB][NB + 1];
  const int tid = threadIdx.x;
  const double2 *a = d.a;
  const int lda = d.lda;

  // pass 1: Ws = V^H B
  const int pi = tid >> 3, pc = tid & 7;
  double2 acc0 = cz(0.0, 0.0), acc1 = cz(0.0, 0.0);
  for (int r0 = k0; r0 < m; r0 += RC) {
    for (int idx = tid; idx < RC * NB; idx += 256) {
      const int rr = idx % RC, i = idx / RC;
      const int r = r0 + rr;
      Vs[rr][i] = (r < m && i < nbp) ? vload(a, lda, k0, i, r) : cz(0.0, 0.0);
    }
    for (int idx = tid; idx < RC * TC; idx += 256) {
      const int rr = idx % RC, c = idx / RC;
      const int r = r0 + rr;
      Bs[rr][c] = (r < m && c < ncol) ? B[(size_t)(c0 + c) * ldb + r] : cz(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll 4
    for (int rr = 0; rr < RC; ++rr) {
      const double2 v = Vs[rr][pi];
      cfmac(acc0, v, Bs[rr][pc]);
      cfmac(acc1, v, Bs[rr][pc + 8]);
    }
    __syncthreads();
  }
  Ws[pi][pc] = acc0;
  Ws[pi][pc + 8] = acc1;
  const double2 *T = d.T + (size_t)(k0 / NB) * NB * NB;
  for (int idx = tid; idx < NB * NB; idx += 256) Ts[idx % NB][idx / NB] = T[idx];
  __syncthreads();
  // W2 = op(T) Ws, op(T) = T^H (trans) or T; T upper triangular
  double2 w0 = cz(0.0, 0.0), w1 = cz(0.0, 0.0);
  if (trans) {
    for (int h = 0; h <= pi; ++h) {
      cfmac(w0, Ts[h][pi], Ws[h][pc]);
      cfmac(w1, Ts[h][pi], Ws[h][pc + 8]);
    }
  } else {
    for (int h = pi; h < NB; ++h) {
      cfma(w0, Ts[pi][h], Ws[h][pc]);
      cfma(w1, Ts[pi][h], Ws[h][pc + 8]);
    }
  }
  __syncthreads();
  Ws[pi][pc] = w0;
  Ws[pi][pc + 8] = w1;
  __syncthreads();

  // pass 2: B -= V W2
  const int ur = tid & 63, ucg = tid >> 6;
  for (int r0 = k0; r0 < m; r0 += RC) {
    for (int idx = tid; idx < RC * NB; idx += 256) {
      const int rr = idx % RC, i = idx / RC;
      const int r = r0 + rr;
      Vs[rr][i] = (r < m && i < nbp) ? vload(a, lda, k0, i, r) : cz(0.0, 0.0);
    }
    __syncthreads();
    const int r = r0 + ur;
    if (r < m) {
      for (int c = ucg; c < ncol; c += 4) {
        double2 acc = cz(0.0, 0.0);
#pragma unroll 8
        for (int i = 0; i < NB; ++i) cfma(acc, Vs[ur][i], Ws[i][c]);
        double2 *p = B + (size_t)(c0 + c) * ldb + r;
        *p = csub(*p, acc);
      }
    }
    __syncthreads();
  }
}

}  // namespace

void qr_factor(const MatDesc *descs, const std::vector<MatDesc> &h, hipStream_t s) {
  int nmax = 0;
  for (const auto &d : h) nmax = std::max(nmax, d.n);
  const int nmat = (int)h.size();
  for (int k0 = 0; k0 < nmax; k0 += NB) {
    hipLaunchKernelGGL(qr_panel_kernel, dim3(nmat), dim3(PT), 0, s, descs, k0);
    HIP_CHECK(hipGetLastError());
    const int trail = nmax - k0 - NB;
    if (trail > 0) {
      hipLaunchKernelGGL(qr_block_apply_kernel, dim3(nmat, cdiv(trail, TC)), dim3(256), 0, s,
                         descs, k0, 1, 0);
      HIP_CHECK(hipGetLastError());
    }
  }
}

// Form U = Q [U_R; 0] in place in d.u (rows >= n of d.u must be zero).
void qr_form_u(const MatDesc *descs, const std::vector<MatDesc> &h, int maxrank, hipStream_t s) {
  int nmax = 0;
  for (const auto &d : h) nmax = std::max(nmax, d.n);
  const int nmat = (int)h.size();
  if (maxrank <= 0) return;
  for (int k0 = ((nmax - 1) / NB) * NB; k0 >= 0; k0 -= NB) {
    hipLaunchKernelGGL(qr_block_apply_kernel, dim3(nmat, cdiv(maxrank, TC)), dim3(256), 0, s,
                       descs, k0, 0, 1);
    HIP_CHECK(hipGetLastError());
  }
}

}  // namespace mfs
