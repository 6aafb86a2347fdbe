// One-sided Jacobi SVD used for the truncated pseudoinverses of Sec. 4.2
// (A_n^+ and Q^+ applied as V S^+ (U^* x), singular values below
// rel_cutoff * s_max dropped); driven by gpinv.hip.
//
// One-sided (Hestenes) Jacobi on G: a pair of columns (p, q) with
// a = |g_p|^2, b = |g_q|^2, gamma = g_p^H g_q = |gamma| e^{i th} is made
// orthogonal by [g_p, g_q] <- [g_p, g_q] [[c, s e^{i th}], [-s e^{-i th}, c]],
// zeta = (b - a) / (2 |gamma|), t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)),
// c = 1 / sqrt(1 + t^2), s = c t; the squared norms become a - t|gamma| and
// b + t|gamma|.  The same rotations accumulate V.  At convergence
// G = U S with orthogonal columns, s_i = |g_i|.
//
// Blocked form for the GPU: the columns are cut into blocks of 16 and the
// round-robin (circle) schedule pairs the blocks, n_b - 1 rounds per sweep.
// One workgroup per block pair (32 columns):
//   1. H = G_IJ^H G_IJ (32 x 32), every entry a dot product of two columns
//      accumulated from 64-row chunks staged in LDS;
//   2. one Jacobi sweep over the 32 columns carried out on H in LDS (the
//      two-sided update H <- R^H H R of each rotation R, with the exact
//      diagonal formulas above and the annihilated entry set to zero), the
//      product J of the rotations accumulated alongside;
//   3. if any pair rotated, G_IJ <- G_IJ J and V_IJ <- V_IJ J.
// Every pair of columns meets in some workgroup every sweep, pairs inside a
// block in every task of that block; sweeps repeat until no pair of a matrix
// needed a rotation (|gamma| <= tol sqrt(a b)), a matrix that converged
// is left out of later sweeps.  The Gram entries carry the error of a dot
// product, relative to sqrt(a b), which keeps the rotations of graded
// columns as accurate as the column-by-column method.
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

constexpr int JB = 16;        // columns per block
constexpr int JC = 2 * JB;    // columns per task
constexpr int JR = 64;        // rows per LDS chunk

__device__ inline void circle_pair(int np, int round, int pair, int &p, int &q) {
  const int mod = np - 1;
  const int rr = round % mod;
  if (pair == 0) {
    p = rr;
    q = np - 1;
  } else {
    p = (rr + pair) % mod;
    q = (rr - pair + mod) % mod;
  }
}

// One round of the blocked sweep: blockIdx.x = block pair, blockIdx.y = matrix.
// flag[mat] counts the tasks that rotated; act[mat] == 0 skips the matrix.
__global__ __launch_bounds__(256) void jac_block_kernel(const MatDesc *__restrict__ descs,
                                                        const int *__restrict__ act, int round,
                                                        double tol) {
  const int mat = blockIdx.y;
  if (!act[mat]) return;
  const MatDesc d = descs[mat];
  const int n = d.n;
  const int nb = (n + JB - 1) / JB;
  const int nbp = nb + (nb & 1);
  if ((int)blockIdx.x >= nbp / 2) return;
  int bi, bj;
  circle_pair(nbp, round, blockIdx.x, bi, bj);
  if (bi >= nb && bj >= nb) return;

  __shared__ double2 Gs[JR][JC + 1];   // chunk, row-major: lanes on rows or on columns read conflict-free
  __shared__ double2 Hs[JC][JC + 1];
  __shared__ double2 Js[JC][JC + 1];
  __shared__ int colx[JC];
  __shared__ double r_c[JB], r_tg[JB], r_a[JB], r_b[JB];
  __shared__ double2 r_se[JB];
  __shared__ int r_act[JB];
  __shared__ int s_nrot;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (tid < JC) {
    const int blk = tid < JB ? bi : bj;
    const int c = blk * JB + (tid & (JB - 1));
    colx[tid] = (blk < nb && c < n) ? c : -1;
  }
  if (tid == 0) s_nrot = 0;
  __syncthreads();

  // 1. Gram matrix: lane (ti, tj) -> entries H[ti + 8k][tj + 8k2], k, k2 < 4; wave -> rows wv, wv+4, ...
  const int ti = lane >> 3, tj = lane & 7;
  double2 acc[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = cz(0.0, 0.0);
  // chunk loads go through registers one chunk ahead of the LDS copy in use
  constexpr int PER = JC * JR / 256;   // elements per thread and chunk
  double2 pre[PER];
  auto fetch = [&](const double2 *M, int r0) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int a = wv + 4 * i, r = r0 + lane;
      const int c = colx[a];
      pre[i] = (c >= 0 && r < n) ? M[(size_t)c * d.ldg + r] : cz(0.0, 0.0);
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int i = 0; i < PER; ++i) Gs[lane][wv + 4 * i] = pre[i];
  };
  fetch(d.g, 0);
  for (int r0 = 0; r0 < n; r0 += JR) {
    stash();
    __syncthreads();
    if (r0 + JR < n) fetch(d.g, r0 + JR);
    for (int rr = wv; rr < JR; rr += 4) {
      double2 x[4], y[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        x[k] = Gs[rr][ti + 8 * k];
        y[k] = Gs[rr][tj + 8 * k];
      }
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) cfmac(acc[k][k2], x[k], y[k2]);
    }
    __syncthreads();
  }
  for (int w = 0; w < 4; ++w) {
    if (wv == w) {
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) {
          double2 &h = Hs[ti + 8 * k][tj + 8 * k2];
          h = (w == 0) ? acc[k][k2] : cadd(h, acc[k][k2]);
        }
    }
    __syncthreads();
  }
  for (int idx = tid; idx < JC * JC; idx += 256) {
    const int r = idx % JC, c = idx / JC;
    Js[r][c] = cz(r == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();

  // 2. one sweep over the 32 columns on H
  for (int rnd = 0; rnd < JC - 1; ++rnd) {
    if (tid < JB) {
      int p, q;
      circle_pair(JC, rnd, tid, p, q);
      const double a = Hs[p][p].x, b = Hs[q][q].x;
      const double2 gam = Hs[p][q];
      const double ag = sqrt(cabs2(gam));
      int on = ag > tol * sqrt(a) * sqrt(b);
      if (on) {
        const double zeta = (b - a) / (2.0 * ag);
        const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / sqrt(1.0 + t * t);
        const double sn = cs * t;
        r_c[tid] = cs;
        r_se[tid] = cz(sn * gam.x / ag, sn * gam.y / ag);
        r_tg[tid] = t * ag;
        r_a[tid] = a;
        r_b[tid] = b;
      }
      r_act[tid] = on;
    }
    __syncthreads();
    int any = 0;
#pragma unroll
    for (int i = 0; i < JB; ++i) any |= r_act[i];
    if (any) {   // uniform: every thread read the same flags
      if (tid == 0) {
        int cnt = 0;
        for (int i = 0; i < JB; ++i) cnt += r_act[i];
        s_nrot += cnt;
      }
      // columns p, q of H and J: X <- X R
      for (int item = tid; item < 2 * JB * JC; item += 256) {
        const int which = item / (JB * JC), rem = item % (JB * JC);
        const int pr = rem / JC, k = rem % JC;
        if (!r_act[pr]) continue;
        int p, q;
        circle_pair(JC, rnd, pr, p, q);
        double2(*M)[JC + 1] = which ? Js : Hs;
        const double2 x = M[k][p], y = M[k][q];
        const double cs = r_c[pr];
        const double2 se = r_se[pr], sec = cconj(r_se[pr]);
        M[k][p] = csub(cscale(x, cs), cmul(sec, y));
        M[k][q] = cadd(cmul(se, x), cscale(y, cs));
      }
      __syncthreads();
      // rows p, q of H: H <- R^H H; the 2x2 pivot block takes its exact values
      for (int item = tid; item < JB * JC; item += 256) {
        const int pr = item / JC, k = item % JC;
        if (!r_act[pr]) continue;
        int p, q;
        circle_pair(JC, rnd, pr, p, q);
        if (k == p) {
          Hs[p][p] = cz(r_a[pr] - r_tg[pr], 0.0);
          Hs[q][p] = cz(0.0, 0.0);
        } else if (k == q) {
          Hs[p][q] = cz(0.0, 0.0);
          Hs[q][q] = cz(r_b[pr] + r_tg[pr], 0.0);
        } else {
          const double2 x = Hs[p][k], y = Hs[q][k];
          const double cs = r_c[pr];
          const double2 se = r_se[pr], sec = cconj(r_se[pr]);
          Hs[p][k] = csub(cscale(x, cs), cmul(se, y));
          Hs[q][k] = cadd(cmul(sec, x), cscale(y, cs));
        }
      }
    }
    __syncthreads();   // flags of this round are read by all before the next round writes them
  }
  if (s_nrot == 0) return;
  if (tid == 0) atomicAdd(d.flag, 1);

  // 3. G_IJ <- G_IJ J and V_IJ <- V_IJ J; thread -> rows (rp, rp + 32), columns 4 cq .. 4 cq + 3
  const int rp = tid & 31, cq = tid >> 5;
  const int nch = (n + JR - 1) / JR;
  fetch(d.g, 0);
  for (int v = 0; v < 2 * nch; ++v) {
    double2 *M = v < nch ? d.g : d.v;
    const int r0 = (v % nch) * JR;
    __syncthreads();   // the previous chunk's readers are done with Gs
    stash();
    __syncthreads();
    if (v + 1 < 2 * nch) fetch(v + 1 < nch ? d.g : d.v, ((v + 1) % nch) * JR);
    double2 o0[4], o1[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) { o0[j] = cz(0.0, 0.0); o1[j] = cz(0.0, 0.0); }
#pragma unroll 4
    for (int a = 0; a < JC; ++a) {
      const double2 x0 = Gs[rp][a], x1 = Gs[rp + 32][a];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const double2 jj = Js[a][4 * cq + j];
        cfma(o0[j], x0, jj);
        cfma(o1[j], x1, jj);
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = colx[4 * cq + j];
      if (c < 0) continue;
      if (r0 + rp < n) M[(size_t)c * d.ldg + r0 + rp] = o0[j];
      if (r0 + rp + 32 < n) M[(size_t)c * d.ldg + r0 + rp + 32] = o1[j];
    }
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
  int nmax = 0, nbpmax = 0;
  for (const auto &d : h) {
    nmax = std::max(nmax, d.n);
    const int nb = cdiv(d.n, JB);
    nbpmax = std::max(nbpmax, nb + (nb & 1));
  }
  if (nmax == 0) return st;
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
  // per matrix and sweep: tasks and their mean width (columns), for the
  // algorithmic byte and flop counts
  const int rounds = std::max(1, nbpmax - 1);
  std::vector<double> tasks(nmat, 0.0), width(nmat, 0.0);
  for (int i = 0; i < nmat; ++i) {
    const int n = h[i].n, nb = cdiv(n, JB), nbp = nb + (nb & 1);
    double cols = 0.0;
    for (int r = 0; r < rounds; ++r)
      for (int pr = 0; pr < nbp / 2; ++pr) {
        const int mod = nbp - 1, rr = r % mod;
        const int p = pr == 0 ? rr : (rr + pr) % mod, q = pr == 0 ? nbp - 1 : (rr - pr + mod) % mod;
        int c = 0;
        if (p < nb) c += std::min(JB, n - p * JB);
        if (q < nb) c += std::min(JB, n - q * JB);
        if (c > 0) { tasks[i] += 1.0; cols += c; }
      }
    width[i] = tasks[i] > 0.0 ? cols / tasks[i] : 0.0;
  }
  std::vector<int> flags(nmat), active(nmat, 1);
  DevBuf act((size_t)nmat * sizeof(int));
  // relative orthogonality reachable in floating point is ~ sqrt(n) eps (the
  // stopping rule of LAPACK's one-sided Jacobi)
  const double tol = 4.0 * sqrt((double)nmax) * 2.220446049250313e-16;
  const int max_sweeps = 40;
  const bool dbg = getenv("MFS_DEBUG") != nullptr;
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    HIP_CHECK(hipMemcpyAsync(act.p, active.data(), nmat * sizeof(int), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(jac_clear_flags, dim3(cdiv(nmat, 256)), dim3(256), 0, s, descs, nmat);
    HIP_CHECK(hipEventRecord(e0, s));
    for (int rnd = 0; rnd < rounds; ++rnd) {
      hipLaunchKernelGGL(jac_block_kernel, dim3(std::max(1, nbpmax / 2), nmat), dim3(256), 0, s, descs,
                         act.as<int>(), rnd, tol);
    }
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipEventRecord(e1, s));
    HIP_CHECK(hipMemcpyAsync(flags.data(), h[0].flag, nmat * sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    float ms = 0.f;
    HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
    st.ms += ms;
    st.launches += rounds;
    // algorithmic work: every task reads its columns of G and forms the
    // Hermitian Gram matrix; a task that rotated writes them back and reads
    // and writes its columns of V, applying the c x c rotation product to both
    bool any = false;
    int nact = 0;
    long nrot = 0;
    for (int i = 0; i < nmat; ++i) {
      if (!active[i]) continue;
      const double n = h[i].n, c = width[i], col = n * sizeof(double2);
      st.bytes += tasks[i] * c * col + (double)flags[i] * 3.0 * c * col;
      st.flops += tasks[i] * 4.0 * c * (c + 1.0) * n + (double)flags[i] * 16.0 * c * c * n;
      if (flags[i] != 0) { any = true; ++nact; nrot += flags[i]; }
      else active[i] = 0;
    }
    if (dbg)
      fprintf(stderr, "[jacobi] nmat %d n %d sweep %d active %d rotating tasks %ld\n", nmat, nmax, sweep,
              nact, nrot);
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
