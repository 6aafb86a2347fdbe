// Truncated SVD of the triangular QR factors (Sec. 4.2: A_n^+ applied as
// V S^+ (U^* x), singular values below rel_cutoff * s_max dropped).
//
// One-sided (Hestenes) Jacobi on G = R: pairs of columns (p, q) are rotated
// by the unitary J = [[c, s e^{i th}], [-s e^{-i th}, c]] that makes them
// orthogonal, where g_p^H g_q = |gamma| e^{i th}; with
// zeta = (|g_q|^2 - |g_p|^2) / (2 |gamma|), t = sign(zeta)/(|zeta| + sqrt(1+zeta^2)),
// c = 1/sqrt(1+t^2), s = c t.  The same rotations accumulate V.  At
// convergence G = U_R S with orthogonal columns, s_i = ||g_i||.
//
// Parallel ordering: the circle (round-robin) schedule pairs the n columns
// into n/2 disjoint pairs per round, n-1 rounds per sweep.  One wave64 per
// pair; one launch per round for the whole batch of matrices, so that many
// small blocks and a few large ones share every launch.  Sweeps repeat until
// no pair of any matrix needed a rotation (|gamma| <= tol ||g_p|| ||g_q||).
#include <algorithm>

#include "internal.hpp"

namespace mfs {

void qr_form_u(const MatDesc *descs, const std::vector<MatDesc> &h, int maxrank, hipStream_t s);

namespace {

__global__ void jac_init_kernel(const MatDesc *__restrict__ descs) {
  const MatDesc d = descs[blockIdx.y];
  const int n = d.n;
  const long total = (long)n * n;
  for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    const int r = (int)(idx % n), c = (int)(idx / n);
    d.g[(size_t)c * d.ldg + r] = (r <= c) ? d.a[(size_t)c * d.lda + r] : cz(0.0, 0.0);
    d.v[(size_t)c * d.ldg + r] = cz(r == c ? 1.0 : 0.0, 0.0);
  }
}

// Squared column norms of R into d.sv (kept up to date by the rotations) and
// the deflation threshold of each matrix: rel * max column norm, squared.
// The largest column norm bounds s_max from below, so pairs of columns whose
// norms are both below rel * s_max_estimate are certainly below the
// truncation cutoff and stay so: a rotation only moves norm between its two
// columns (|g_p|^2 + |g_q|^2 is invariant), and a rotation of a tiny column
// against a large one shrinks the tiny one.  Such pairs are skipped.
__global__ __launch_bounds__(256) void jac_norms_kernel(const MatDesc *__restrict__ descs,
                                                        double rel, double *__restrict__ thr) {
  const MatDesc d = descs[blockIdx.x];
  const int n = d.n;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __shared__ double wmax[4];
  double mx = 0.0;
  for (int c = wv; c < n; c += 4) {
    const double2 *a = d.a + (size_t)c * d.lda;
    double s = 0.0;
    for (int r = lane; r <= c; r += 64) s += cabs2(a[r]);
    s = wave_sum(s);
    if (lane == 0) d.sv[c] = s;
    mx = fmax(mx, s);
  }
  if (lane == 0) wmax[wv] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double m = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
    thr[blockIdx.x] = rel * rel * m;
  }
}

__global__ void jac_clear_flags(const MatDesc *__restrict__ descs, int nmat) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nmat) descs[i].flag[0] = 0;
}

__global__ __launch_bounds__(256) void jac_round_kernel(const MatDesc *__restrict__ descs,
                                                        int round, double tol,
                                                        const double *__restrict__ thr) {
  const MatDesc d = descs[blockIdx.y];
  const int n = d.n;
  const int np = n + (n & 1);
  const int lane = threadIdx.x & 63;
  const int pair = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (pair >= np / 2) return;
  const int mod = np - 1;
  const int rr = round % mod;
  int p, q;
  if (pair == 0) {
    p = rr;
    q = np - 1;
  } else {
    p = (rr + pair) % mod;
    q = (rr - pair + mod) % mod;
  }
  if (p >= n || q >= n) return;
  if (fmax(d.sv[p], d.sv[q]) < thr[blockIdx.y]) return;   // both negligible: skip
  double2 *gp = d.g + (size_t)p * d.ldg;
  double2 *gq = d.g + (size_t)q * d.ldg;
  double a = 0.0, b = 0.0;
  double2 c = cz(0.0, 0.0);
  for (int r = lane; r < n; r += 64) {
    const double2 x = gp[r], y = gq[r];
    a += cabs2(x);
    b += cabs2(y);
    cfmac(c, x, y);
  }
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  const double ac = sqrt(cabs2(c));
  if (!(ac > tol * sqrt(a) * sqrt(b))) return;
  if (lane == 0) d.flag[0] = 1;
  const double zeta = (b - a) / (2.0 * ac);
  const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  const double cs = 1.0 / sqrt(1.0 + t * t);
  const double sn = cs * t;
  const double2 e = cz(c.x / ac, c.y / ac);           // e^{i th}
  const double2 se = cz(sn * e.x, sn * e.y);            // s e^{i th}
  const double2 sec = cz(sn * e.x, -sn * e.y);          // s e^{-i th}
  if (lane == 0) {
    d.sv[p] = fmax(a - t * ac, 0.0);
    d.sv[q] = b + t * ac;
  }
  for (int r = lane; r < n; r += 64) {
    const double2 x = gp[r], y = gq[r];
    gp[r] = csub(cscale(x, cs), cmul(sec, y));
    gq[r] = cadd(cmul(se, x), cscale(y, cs));
  }
  double2 *vp = d.v + (size_t)p * d.ldg;
  double2 *vq = d.v + (size_t)q * d.ldg;
  for (int r = lane; r < n; r += 64) {
    const double2 x = vp[r], y = vq[r];
    vp[r] = csub(cscale(x, cs), cmul(sec, y));
    vq[r] = cadd(cmul(se, x), cscale(y, cs));
  }
}

// Column norms, descending order (rank by counting, ties by index), kept rank.
__global__ __launch_bounds__(256) void jac_sort_kernel(const MatDesc *__restrict__ descs,
                                                       double rel_cutoff) {
  extern __shared__ double sig[];
  const MatDesc d = descs[blockIdx.x];
  const int n = d.n;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int c = wv; c < n; c += 4) {
    const double2 *g = d.g + (size_t)c * d.ldg;
    double s = 0.0;
    for (int r = lane; r < n; r += 64) s += cabs2(g[r]);
    s = wave_sum(s);
    if (lane == 0) sig[c] = sqrt(s);
  }
  __syncthreads();
  __shared__ double smax;
  __shared__ int rank;
  if (threadIdx.x == 0) {
    double mx = 0.0;
    for (int i = 0; i < n; ++i) mx = fmax(mx, sig[i]);
    smax = mx;
    rank = 0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double si = sig[i];
    int pos = 0;
    for (int k = 0; k < n; ++k) {
      const double sk = sig[k];
      pos += (sk > si) || (sk == si && k < i);
    }
    d.perm[pos] = i;
    d.sv[pos] = si;
    if (si > rel_cutoff * smax && smax > 0.0) atomicAdd(&rank, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) d.rank[0] = rank;
}

// U[:, k] = g_{perm k} / s_k on rows < n (zero below), W[:, k] = v_{perm k} / s_k
// for k < rank; other columns zero.
__global__ void jac_form_kernel(const MatDesc *__restrict__ descs) {
  const MatDesc d = descs[blockIdx.y];
  const int k = blockIdx.x;
  if (k >= d.n) return;
  const int r = d.rank[0];
  double2 *u = d.u + (size_t)k * d.lda;
  double2 *w = d.w + (size_t)k * d.ldg;
  if (k >= r) {
    for (int i = threadIdx.x; i < d.m; i += blockDim.x) u[i] = cz(0.0, 0.0);
    for (int i = threadIdx.x; i < d.n; i += blockDim.x) w[i] = cz(0.0, 0.0);
    return;
  }
  const int c = d.perm[k];
  const double inv = 1.0 / d.sv[k];
  const double2 *g = d.g + (size_t)c * d.ldg;
  const double2 *v = d.v + (size_t)c * d.ldg;
  for (int i = threadIdx.x; i < d.m; i += blockDim.x) u[i] = (i < d.n) ? cscale(g[i], inv) : cz(0.0, 0.0);
  for (int i = threadIdx.x; i < d.n; i += blockDim.x) w[i] = cscale(v[i], inv);
}

}  // namespace

void svd_truncate(const MatDesc *descs, const std::vector<MatDesc> &h, double rel_cutoff,
                  hipStream_t s, std::vector<int> &ranks) {
  const int nmat = (int)h.size();
  int nmax = 0;
  for (const auto &d : h) nmax = std::max(nmax, d.n);
  const int npmax = nmax + (nmax & 1);
  hipLaunchKernelGGL(jac_init_kernel, dim3(std::min(1024, cdiv(nmax * nmax, 256)), nmat), dim3(256),
                     0, s, descs);
  HIP_CHECK(hipGetLastError());
  for (int i = 0; i < nmat; ++i) {
    MFS_REQUIRE(h[i].flag == h[0].flag + i && h[i].rank == h[0].rank + i,
                "svd_truncate: flags and ranks must be contiguous");
  }
  std::vector<int> flags(nmat);
  DevBuf thr((size_t)nmat * sizeof(double));
  // pairs of columns below 1e-3 of the cutoff are skipped (see jac_norms_kernel)
  hipLaunchKernelGGL(jac_norms_kernel, dim3(nmat), dim3(256), 0, s, descs, 1e-3 * rel_cutoff,
                     thr.as<double>());
  HIP_CHECK(hipGetLastError());
  // relative orthogonality reachable in floating point is ~ sqrt(n) eps (the
  // stopping rule of LAPACK's one-sided Jacobi)
  const double tol = 4.0 * sqrt((double)nmax) * 2.220446049250313e-16;
  const int max_sweeps = 40;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    hipLaunchKernelGGL(jac_clear_flags, dim3(cdiv(nmat, 256)), dim3(256), 0, s, descs, nmat);
    for (int rnd = 0; rnd < npmax - 1; ++rnd) {
      hipLaunchKernelGGL(jac_round_kernel, dim3(cdiv(npmax / 2, 4), nmat), dim3(256), 0, s, descs,
                         rnd, tol, thr.as<double>());
    }
    HIP_CHECK(hipGetLastError());
    bool any = false;
    HIP_CHECK(hipMemcpyAsync(flags.data(), h[0].flag, nmat * sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    for (int f : flags) any |= (f != 0);
    if (!any) break;
  }
  hipLaunchKernelGGL(jac_sort_kernel, dim3(nmat), dim3(256), (size_t)nmax * sizeof(double), s,
                     descs, rel_cutoff);
  HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(jac_form_kernel, dim3(nmax, nmat), dim3(256), 0, s, descs);
  HIP_CHECK(hipGetLastError());
  ranks.assign(nmat, 0);
  HIP_CHECK(hipMemcpyAsync(ranks.data(), h[0].rank, nmat * sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipStreamSynchronize(s));
  int maxrank = 0;
  for (int r : ranks) maxrank = std::max(maxrank, r);
  qr_form_u(descs, h, maxrank, s);
}

}  // namespace mfs
