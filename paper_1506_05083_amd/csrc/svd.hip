// One-sided Jacobi SVD used for the truncated pseudoinverses of Sec. 4.2
// (A_n^+ and Q^+ applied as V S^+ (U^* x), singular values below
// rel_cutoff * s_max dropped); driven by gpinv.hip.
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
#include <cstdio>
#include <cstdlib>

#include "internal.hpp"

namespace mfs {

namespace {

// mode 0: G = triu(a[0:n, 0:n]) (the R factor); mode 1: G = R^H (lower triangular)
__global__ void jac_init_kernel(const MatDesc *__restrict__ descs, int mode) {
  const MatDesc d = descs[blockIdx.y];
  const int n = d.n;
  const long total = (long)n * n;
  for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    const int r = (int)(idx % n), c = (int)(idx / n);
    double2 v;
    if (mode == 0) v = (r <= c) ? d.a[(size_t)c * d.lda + r] : cz(0.0, 0.0);
    else v = (c <= r) ? cconj(d.a[(size_t)r * d.lda + c]) : cz(0.0, 0.0);
    d.g[(size_t)c * d.ldg + r] = v;
    d.v[(size_t)c * d.ldg + r] = cz(r == c ? 1.0 : 0.0, 0.0);
  }
}

__global__ void jac_clear_flags(const MatDesc *__restrict__ descs, int nmat) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nmat) descs[i].flag[0] = 0;
}

__global__ __launch_bounds__(256) void jac_round_kernel(const MatDesc *__restrict__ descs,
                                                        int round, double tol) {
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
  if (lane == 0) atomicAdd(d.flag, 1);   // rotations this sweep
  const double zeta = (b - a) / (2.0 * ac);
  const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  const double cs = 1.0 / sqrt(1.0 + t * t);
  const double sn = cs * t;
  const double2 e = cz(c.x / ac, c.y / ac);           // e^{i th}
  const double2 se = cz(sn * e.x, sn * e.y);            // s e^{i th}
  const double2 sec = cz(sn * e.x, -sn * e.y);          // s e^{-i th}

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

}  // namespace

JacStats jac_run(const MatDesc *descs, const std::vector<MatDesc> &h, int init_mode, double rel_cutoff,
                 hipStream_t s) {
  JacStats st;
  const int nmat = (int)h.size();
  int nmax = 0;
  for (const auto &d : h) nmax = std::max(nmax, d.n);
  if (nmax == 0) return st;
  const int npmax = nmax + (nmax & 1);
  hipEvent_t e0, e1;
  HIP_CHECK(hipEventCreate(&e0));
  HIP_CHECK(hipEventCreate(&e1));
  hipLaunchKernelGGL(jac_init_kernel, dim3(std::min(1024, cdiv(nmax * nmax, 256)), nmat), dim3(256),
                     0, s, descs, init_mode);
  HIP_CHECK(hipGetLastError());
  for (int i = 0; i < nmat; ++i) {
    MFS_REQUIRE(h[i].flag == h[0].flag + i && h[i].rank == h[0].rank + i,
                "jacobi: flags and ranks must be contiguous");
  }
  std::vector<int> flags(nmat);
  // relative orthogonality reachable in floating point is ~ sqrt(n) eps (the
  // stopping rule of LAPACK's one-sided Jacobi)
  const double tol = 4.0 * sqrt((double)nmax) * 2.220446049250313e-16;
  const int max_sweeps = 40;
  const bool dbg = getenv("MFS_DEBUG") != nullptr;
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    hipLaunchKernelGGL(jac_clear_flags, dim3(cdiv(nmat, 256)), dim3(256), 0, s, descs, nmat);
    HIP_CHECK(hipEventRecord(e0, s));
    for (int rnd = 0; rnd < npmax - 1; ++rnd) {
      hipLaunchKernelGGL(jac_round_kernel, dim3(cdiv(npmax / 2, 4), nmat), dim3(256), 0, s, descs,
                         rnd, tol);
    }
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipEventRecord(e1, s));
    bool any = false;
    HIP_CHECK(hipMemcpyAsync(flags.data(), h[0].flag, nmat * sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    float ms = 0.f;
    HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
    st.ms += ms;
    st.launches += npmax - 1;
    // algorithmic bytes: every pair reads its two columns of G; a pair that
    // rotates also writes them and reads and writes its two columns of V
    for (int i = 0; i < nmat; ++i) {
      const double col = (double)h[i].n * sizeof(double2);
      st.bytes += 0.5 * h[i].n * (h[i].n - 1) * 2.0 * col + (double)flags[i] * 6.0 * col;
    }
    for (int f : flags) any |= (f != 0);
    if (dbg) {
      int nact = 0;
      long nrot = 0;
      for (int f : flags) { nact += (f != 0); nrot += f; }
      fprintf(stderr, "[jacobi] nmat %d n %d sweep %d active %d rotations %ld\n", nmat, nmax, sweep, nact,
              nrot);
    }
    if (!any) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

void jac_sort(const MatDesc *descs, const std::vector<MatDesc> &h, double rel_cutoff, hipStream_t s,
              std::vector<int> &ranks) {
  const int nmat = (int)h.size();
  int nmax = 0;
  for (const auto &d : h) nmax = std::max(nmax, d.n);
  hipLaunchKernelGGL(jac_sort_kernel, dim3(nmat), dim3(256), (size_t)std::max(nmax, 1) * sizeof(double), s,
                     descs, rel_cutoff);
  HIP_CHECK(hipGetLastError());
  ranks.assign(nmat, 0);
  HIP_CHECK(hipMemcpyAsync(ranks.data(), h[0].rank, nmat * sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipStreamSynchronize(s));
}

}  // namespace mfs
