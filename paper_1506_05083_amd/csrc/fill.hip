// Modal fill of the one-body blocks (eqs. (ringkernelderiv) and (ptr)) and
// the incident-wave right-hand side (eqs. (neu), (fhatquad)).
//
// Fill.  For a target ring (rho, z) with normal (nrho, nz) and a source ring
// (rho', z'), the integrand of eq. (ringkernelderiv) at angle phi is
//   g(phi) = dG/dn_x = G (ik - 1/R) (d.n)/R,   G = e^{ikR}/(4 pi R),
//   R^2 = rho^2 + rho'^2 - 2 rho rho' cos phi + (z - z')^2,
//   d.n = (rho - rho' cos phi) nrho + (z - z') nz,
// so both R^2 and d.n are affine in cos phi.  g is even in phi, so the
// q-node trapezoid rule of eq. (ptr) for mode n folds onto l = 0..q/2:
//   A'_n = (1/q) [g_0 + (-1)^n g_{q/2} + 2 sum_{0<l<q/2} g_l cos(2 pi n l / q)],
// and A'_{-n} = A'_n: only n = 0..P/2 are computed.
//
// Layout: one workgroup per tile of 64 (m, j) pairs (m fastest, so stores
// of A[n][j][m] are coalesced), a wave per 16 pairs.  The q/2+1 nodes are
// processed in chunks of 32 whose cosine weights are staged in LDS from a
// per-operator table; each lane evaluates the sample of its pair at one
// node of every 4-node step (one rsqrt and one sincos) and the fold onto
// the P/2+1 modes runs on the FP64 matrix cores (fill_tile).
#include <algorithm>

#include "internal.hpp"

namespace mfs {
namespace {

constexpr int TP = 64;    // (m, j) pairs per workgroup
constexpr int LC = 32;    // trapezoid nodes per LDS chunk

// tab[l][0..nd-1] = c_l cos(2 pi n l / q) / q with c_0 = c_{q/2} = 1, else 2;
// tab[l][nd] = cos(2 pi l / q).  Argument reduction is exact (integer n l mod q).
__global__ void fill_table_kernel(int q, int nd, double *tab) {
  const int L = q / 2 + 1;
  const int ld = nd + 1;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < L * ld;
       idx += gridDim.x * blockDim.x) {
    int l = idx / ld, n = idx % ld;
    double v;
    if (n == nd) {
      v = cospi(2.0 * l / q);
    } else {
      long r = ((long)n * l) % q;
      double cl = (l == 0 || 2 * l == q) ? 1.0 : 2.0;
      v = cl * cospi(2.0 * (double)r / q) / q;
    }
    tab[idx] = v;
  }
}

// One sub-block of one body's mode blocks in the batched fill: the value
// kernel G (eq. (ringkernel)) or its normal derivative (eq.
// (ringkernelderiv)) at wavenumber k from the sources (srho, sz), times sign.
struct FillJob {
  int M, N, q, nd, ldA;
  int ncols;       // columns of one mode block (N, or 2N for transmission)
  int value;       // 1: G, 0: dG/dn_x
  double k, sign;
  const double *rho, *z, *nrho, *nz, *srho, *sz;
  const double *tab;
  double2 *A;      // entry (0, 0) of this sub-block in the mode-0 block
  long tile0;      // first tile of this job in the batch's tile list
};

// Tile `tile` (64 (m, j) pairs) of job J; all 256 threads take part.  The
// fold onto the modes is a real-by-complex product on the FP64 matrix
// cores: D[n][p] = sum_l W[n][l] g_l(p) with W[n][l] the weight
// c_l cos(2 pi n l / q) / q of the table and g_l(p) the kernel sample of pair
// p at node l, formed by each lane for its own pair (wave w: pairs
// 16 w .. 16 w + 15) and node (4 per step), so a sample feeds one product
// per 16-mode block and real or imaginary part.  The weights come from the
// table chunk staged in LDS; the output (lane group: 16 consecutive pairs of
// one mode) is stored in 256-byte pieces.
constexpr int FB = 7;   // 16-mode blocks: nd <= 104 (the table chunk's row)
__device__ void fill_tile(const FillJob &J, long tile, double *wt) {
  const int M = J.M, N = J.N, q = J.q, nd = J.nd, ldA = J.ldA;
  const double k = J.k;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int l16 = lane & 15, k4 = lane >> 4;
  const long pair = tile * TP + 16 * wv + l16;
  const bool valid = pair < (long)M * N;
  const int m = valid ? (int)(pair % M) : 0;
  const int j = valid ? (int)(pair / M) : 0;
  const double r = J.rho[m], rs = J.srho[j];
  const double dz = J.z[m] - J.sz[j];
  const double Ac = r * r + rs * rs + dz * dz;
  const double Bc = 2.0 * r * rs;
  const double Cc = r * J.nrho[m] + dz * J.nz[m];
  const double Dc = rs * J.nrho[m];
  const double inv4pi = 0.25 / kPi;
  const int L = q / 2 + 1;
  const int ld = nd + 1;
  const int nmb = (nd + 15) / 16;   // uniform over the workgroup

  dx4 re[FB], im[FB];
#pragma unroll
  for (int b = 0; b < FB; ++b) {
    re[b] = dx4{0.0, 0.0, 0.0, 0.0};
    im[b] = re[b];
  }

  for (int l0 = 0; l0 < L; l0 += LC) {
    const int lc = min(LC, L - l0);
    __syncthreads();
    for (int idx = tid; idx < lc * ld; idx += 256) wt[idx] = J.tab[(size_t)l0 * ld + idx];
    __syncthreads();
    for (int kk = 0; kk < lc; kk += 4) {
      const int ll = kk + k4;
      double2 g = cz(0.0, 0.0);
      if (ll < lc && valid) {
        const double c = wt[ll * ld + nd];
        const double R2 = fma(-Bc, c, Ac);
        const double dn = fma(-Dc, c, Cc);
        const double invR = rsqrt(R2);
        const double R = R2 * invR;
        double sn, cs;
        sincos(k * R, &sn, &cs);
        if (J.value) {
          // (cs + i sn) / (4 pi R)
          const double t = J.sign * invR * inv4pi;
          g = cz(t * cs, t * sn);
        } else {
          const double t = J.sign * dn * invR * invR * inv4pi;
          // (cs + i sn) (i k - invR) t
          g = cz(t * fma(-cs, invR, -sn * k), t * fma(cs, k, -sn * invR));
        }
      }
      // A[n][l] = W (lane l16 + 16 k4 holds mode 16 b + l16, node ll);
      // B[l][p] = g (lane l16 + 16 k4 holds node ll, pair l16)
#pragma unroll
      for (int b = 0; b < FB; ++b) {
        if (b < nmb) {
          const int n = 16 * b + l16;
          const double w = (ll < lc && n < nd) ? wt[ll * ld + n] : 0.0;
          re[b] = mfma_f64(w, g.x, re[b]);
          im[b] = mfma_f64(w, g.y, im[b]);
        }
      }
    }
  }
  if (valid) {
    // lane l16 + 16 k4 holds D[n = 16 b + k4 + 4 v][pair l16] in element v
#pragma unroll
    for (int b = 0; b < FB; ++b) {
      if (b >= nmb) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int n = 16 * b + k4 + 4 * v;
        if (n < nd) J.A[((size_t)n * J.ncols + j) * ldA + m] = cz(re[b][v], im[b][v]);
      }
    }
  }
}

// Persistent fill of every body of a batch: a fixed grid of workgroups takes
// tiles from a global counter until the batch's ntiles are done (jobs are in
// order of tile0, the costliest bodies first, so the tail is made of cheap
// tiles).  Every workgroup leaves once the counter passes ntiles.
__global__ __launch_bounds__(256) void fill_batch_kernel(const FillJob *__restrict__ jobs, int njobs,
                                                         long ntiles, unsigned long long *__restrict__ counter) {
  __shared__ double wt[LC * 105];
  __shared__ long s_tile;
  __shared__ int s_job;
  for (;;) {
    if (threadIdx.x == 0) {
      const long t = (long)atomicAdd(counter, 1ULL);
      int lo = 0, hi = njobs - 1;   // last job with tile0 <= t
      while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (jobs[mid].tile0 <= t) lo = mid;
        else hi = mid - 1;
      }
      s_tile = t;
      s_job = lo;
    }
    __syncthreads();
    const long t = s_tile;
    const int jb = s_job;
    __syncthreads();   // s_tile / s_job read by all before thread 0 overwrites them
    if (t >= ntiles) return;
    const FillJob J = jobs[jb];
    fill_tile(J, t - J.tile0, wt);
  }
}

// f = -du^i/dn = -i (k.n) e^{i k.x} (value = 0) or f = -u^i (value = 1, the
// transmission case) on the P x M surface nodes, folded into
// f_hat_b = (1/P) sum_l f_l e^{-2 pi i b l / P} and written at
// out[(w P + b) ldo + m].  One workgroup per 8 rings of one wave; twiddles
// from an exact table in LDS.
constexpr int RM = 8;
__global__ __launch_bounds__(256) void rhs_kernel(int M, int P, int ldo, int value, const double *__restrict__ rho,
                                                  const double *__restrict__ zc,
                                                  const double *__restrict__ nrho,
                                                  const double *__restrict__ nzc,
                                                  const double *__restrict__ kvec,
                                                  double2 *__restrict__ out) {
  extern __shared__ double2 sh[];
  double2 *tw = sh;          // [P]
  double2 *f = sh + P;       // [RM][P]
  const int w = blockIdx.y;
  const int m0 = blockIdx.x * RM;
  const double kx = kvec[3 * w], ky = kvec[3 * w + 1], kzv = kvec[3 * w + 2];
  for (int l = threadIdx.x; l < P; l += blockDim.x) {
    double s, c;
    sincospi(-2.0 * l / P, &s, &c);
    tw[l] = cz(c, s);
  }
  for (int idx = threadIdx.x; idx < RM * P; idx += blockDim.x) {
    const int ring = idx / P, l = idx % P;
    const int m = m0 + ring;
    double2 v = cz(0.0, 0.0);
    if (m < M) {
      double sp, cp;
      sincospi(2.0 * l / P, &sp, &cp);
      const double x = rho[m] * cp, y = rho[m] * sp;
      const double kn = kx * nrho[m] * cp + ky * nrho[m] * sp + kzv * nzc[m];
      double s, c;
      sincos(kx * x + ky * y + kzv * zc[m], &s, &c);
      // -i kn (c + i s) = kn s - i kn c ; or -(c + i s)
      v = value ? cz(-c, -s) : cz(kn * s, -kn * c);
    }
    f[idx] = v;
  }
  __syncthreads();
  const double invP = 1.0 / P;
  for (int idx = threadIdx.x; idx < RM * P; idx += blockDim.x) {
    const int ring = idx % RM, b = idx / RM;
    const int m = m0 + ring;
    if (m >= M) continue;
    double2 acc = cz(0.0, 0.0);
    int ph = 0;
    for (int l = 0; l < P; ++l) {
      cfma(acc, f[ring * P + l], tw[ph]);
      ph += b;
      if (ph >= P) ph -= P;
    }
    out[((size_t)w * P + b) * ldo + m] = cscale(acc, invP);
  }
}

}  // namespace

void launch_fill_all(const std::vector<BodyData *> &bodies, hipStream_t s) {
  const int nb = (int)bodies.size();
  if (nb == 0) return;
  std::vector<int> order(nb);
  for (int i = 0; i < nb; ++i) order[i] = i;
  // costliest first: work of a pair ~ (q/2+1)(P/2+1)
  auto cost = [&](int i) { return (double)(bodies[i]->q / 2 + 1) * (bodies[i]->nd + 1); };
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost(x) > cost(y); });
  std::vector<DevBuf> tabs(nb);
  std::vector<FillJob> jobs;
  long tiles = 0;
  for (int o = 0; o < nb; ++o) {
    BodyData &b = *bodies[order[o]];
    MFS_REQUIRE(b.nd <= 104, "P/2+1 exceeds the fill kernel's mode capacity (P <= 206)");
    const int L = b.q / 2 + 1;
    tabs[o].alloc((size_t)L * (b.nd + 1) * sizeof(double));
    hipLaunchKernelGGL(fill_table_kernel, dim3(cdiv(L * (b.nd + 1), 256)), dim3(256), 0, s, b.q, b.nd,
                       tabs[o].as<double>());
    FillJob J{};
    J.M = b.M; J.N = b.N; J.q = b.q; J.nd = b.nd; J.ldA = b.ldA; J.ncols = b.cols;
    J.rho = b.rho; J.z = b.z; J.nrho = b.nrho; J.nz = b.nz;
    J.tab = tabs[o].as<double>();
    double2 *A0 = b.blocks.as<double2>();
    auto add = [&](int value, double k, double sign, const double *srho, const double *sz, double2 *A) {
      J.value = value; J.k = k; J.sign = sign; J.srho = srho; J.sz = sz; J.A = A;
      J.tile0 = tiles;
      tiles += ((long)b.M * b.N + TP - 1) / TP;
      jobs.push_back(J);
    };
    if (!b.trans()) {
      add(0, b.k, 1.0, b.srho, b.sz, A0);
    } else {
      // eq. (trans): rows [values; normal derivatives], columns [exterior; interior]
      add(1, b.k, 1.0, b.srho, b.sz, A0);
      add(0, b.k, 1.0, b.srho, b.sz, A0 + b.M);
      add(1, b.km, -1.0, b.srho2, b.sz2, A0 + (size_t)b.N * b.ldA);
      add(0, b.km, -1.0, b.srho2, b.sz2, A0 + (size_t)b.N * b.ldA + b.M);
    }
  }
  HIP_CHECK(hipGetLastError());
  DevBuf jd(jobs.size() * sizeof(FillJob)), ctr(sizeof(unsigned long long));
  HIP_CHECK(hipMemcpyAsync(jd.p, jobs.data(), jobs.size() * sizeof(FillJob), hipMemcpyHostToDevice, s));
  HIP_CHECK(hipMemsetAsync(ctr.p, 0, sizeof(unsigned long long), s));
  int dev = 0, ncu = 256;
  HIP_CHECK(hipGetDevice(&dev));
  HIP_CHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const long grid = std::min<long>(tiles, (long)ncu * 4);
  hipLaunchKernelGGL(fill_batch_kernel, dim3((unsigned)grid), dim3(256), 0, s, jd.as<FillJob>(), (int)jobs.size(),
                     tiles, ctr.as<unsigned long long>());
  HIP_CHECK(hipGetLastError());
  // the tables and job list are freed on return; make sure the kernel is done with them
  HIP_CHECK(hipStreamSynchronize(s));
}

void launch_fill(BodyData &b, hipStream_t s) { launch_fill_all({&b}, s); }

void launch_rhs(const BodyData &b, int nw, const double *kvec_dev, double2 *out, hipStream_t s) {
  const size_t sh = (size_t)(b.P + RM * b.P) * sizeof(double2);
  if (!b.trans()) {
    hipLaunchKernelGGL(rhs_kernel, dim3(cdiv(b.M, RM), nw), dim3(256), sh, s, b.M, b.P, b.M, 0, b.rho, b.z,
                       b.nrho, b.nz, kvec_dev, out);
  } else {
    // [f_hat; f_hat'] per mode: f = -u^i in rows [0, M), f' = -du^i/dn in rows [M, 2M)
    hipLaunchKernelGGL(rhs_kernel, dim3(cdiv(b.M, RM), nw), dim3(256), sh, s, b.M, b.P, b.rows, 1, b.rho, b.z,
                       b.nrho, b.nz, kvec_dev, out);
    hipLaunchKernelGGL(rhs_kernel, dim3(cdiv(b.M, RM), nw), dim3(256), sh, s, b.M, b.P, b.rows, 0, b.rho, b.z,
                       b.nrho, b.nz, kvec_dev, out + b.M);
  }
  HIP_CHECK(hipGetLastError());
}

}  // namespace mfs
