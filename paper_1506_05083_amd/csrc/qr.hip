// Batched blocked Householder QR of tall complex matrices (the dense
// least-squares factorisations of Sec. 3, eq. (linsys), and of the
// periodizing matrix Q of Sec. 4.2), LAPACK's zlarfg convention:
// H = I - tau v v^H, v(1) = 1, H^H x = beta e_1 with beta real.
//
// Panels of NB = 32 columns.  The panel is factorised column by column with
// one launch per column that spans all rows of all matrices (CH-row chunks,
// one row per thread, the row's panel entries in registers):
//   * launch s finishes reflector s from the chunk partial sums written by
//     launch s-1: |x(2:)|^2 and x^H a_c for the panel columns c > s (so the
//     reflector and every w_c = v^H a_c follow from one pass over the rows),
//     with row j of the panel read from a side buffer that no workgroup of
//     launch s writes;
//   * it then applies H_s^H to its rows of the columns c > s and writes the
//     partial sums of step s + 1.
// The trailing matrix is updated with the compact-WY form
// C <- (I - V T V^H)^H C = C - V T^H (V^H C):
//   bqr_vhy_kernel   P = V^H [V | C], split over row slices (partials);
//   bqr_t_kernel     T from the V^H V part (forward, columnwise);
//   bqr_w2_kernel    W2 = op(T) (V^H C), the slices summed;
//   bqr_update       C -= V W2 on the matrix cores.
// The same three apply kernels with T in place of T^H, run over the panels
// in reverse, form U = Q [U_R; 0] for the explicit left singular vectors.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>

#include "internal.hpp"

namespace mfs {
namespace {

constexpr int CH = 256;     // rows per workgroup in the panel column step
constexpr int KRMIN = 256;  // fewest rows of a V^H Y split-K slice (sizes the partials' buffer)
constexpr int KS = 16;      // rows per LDS stage in V^H Y
// V^H Y tiles: YT columns of Y a workgroup, a wave IB x CB blocks of 16 x 16
// of the NB x YT tile, OCC waves a SIMD, DB: LDS stages double-buffered (one
// barrier a stage), KR rows a workgroup (one split-K slice: each slice writes
// an NB-row partial of P that W2 and T read back).  Measured on 8 matrices
// 4608 x 1275 with 256-row slices: 64-column panels 54 TFLOP/s (43 with one
// 16-row block of V^H and four column blocks a wave and the fragments loaded
// per product), 32: 43 (33), 16: 3.8 TB/s of Y.  The 64-wide panels take
// 512-row slices: on that shape V^H Y is 8% slower and W2 as much faster, on
// the 25088-row Q of the large cup the QR and U formation gain 2%.
template <int NB> struct VhyShape;
template <> struct VhyShape<64> { static constexpr int YT = 64, IB = 2, CB = 2, OCC = 2, DB = 0, KR = 512; };
template <> struct VhyShape<32> { static constexpr int YT = 64, IB = 1, CB = 2, OCC = 3, DB = 1, KR = 256; };
template <> struct VhyShape<16> { static constexpr int YT = 64, IB = 1, CB = 1, OCC = 4, DB = 1, KR = 256; };
constexpr int W2T = 16;     // columns per W2 tile (the slices' sum spread over more workgroups)
constexpr int W2WG = 8192;  // workgroups a W2 launch aims at; beyond it a workgroup takes several tiles

// element r of Householder vector i of the panel starting at column k0
__device__ inline double2 vel(const MatDesc &d, int k0, int i, int r) {
  const int c = k0 + i;
  const double2 x = ld_or0(d.a, (size_t)c * d.lda + r, c < d.n && r > c && r < d.m);
  return csel(c < d.n && r == c, cz(1.0, 0.0), x);
}

__device__ inline int ldu_of(const MatDesc &d) { return d.ldu ? d.ldu : d.lda; }

// Panel column step s (s = -1: partial sums of step 0 only).
// part: [mat][2][nchmax][NPART] (slot [0].x: |x(2:)|^2, slot 1 + c: x^H a_c)
// side: [mat][2][NB] row j of the panel columns
template <int NB>
__global__ __launch_bounds__(CH) void bqr_col_kernel(const MatDesc *__restrict__ descs, int k0, int s,
                                                     double2 *__restrict__ part, double2 *__restrict__ side,
                                                     int nchmax) {
  constexpr int NPART = NB + 1;
  constexpr int SUB = CH / NPART;   // threads per slot summing the chunk partials
  static_assert(SUB >= 1, "a column-step workgroup sums every partial slot");
  const MatDesc d = descs[blockIdx.y];
  if (k0 >= d.n) return;
  const int nbp = min(NB, d.n - k0);
  if (s >= nbp) return;
  const int mrows = d.m - k0;
  if ((int)blockIdx.x * CH >= mrows) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int r = k0 + blockIdx.x * CH + tid;
  const bool live = r < d.m;
  double2 *pb = part + (size_t)blockIdx.y * 2 * nchmax * NPART;
  double2 *sb = side + (size_t)blockIdx.y * 2 * NB;
  __shared__ double2 fin[NPART];
  __shared__ double2 fsum[NPART][SUB];
  __shared__ double2 sf[NB];
  __shared__ double2 red[CH / 64][NPART];
  __shared__ double2 s_scale, s_tau, s_alpha;
  __shared__ double s_beta;
  __shared__ int s_refl;

  double2 vals[NB];
  const int cfirst = s < 0 ? 0 : s;
#pragma unroll
  for (int c = 0; c < NB; ++c)
    vals[c] = ld_or0(d.a, (size_t)(k0 + c) * d.lda + r, live && c >= cfirst && c < nbp);

  if (s >= 0) {
    const int j = k0 + s;
    const double2 *pin = pb + (size_t)(s & 1) * nchmax * NPART;
    const double2 *srow = sb + (s & 1) * NB;
    const int nch = (mrows + CH - 1) / CH;
    // chunk partials summed by SUB threads per slot, then across them
    if (tid < NPART * SUB) {
      const int slot = tid / SUB, sub = tid % SUB;
      double2 t = cz(0.0, 0.0);
      for (int ch = sub; ch < nch; ch += SUB) t = cadd(t, pin[(size_t)ch * NPART + slot]);
      fsum[slot][sub] = t;
    }
    __syncthreads();
    if (tid < NPART) {
      double2 t = fsum[tid][0];
#pragma unroll
      for (int u = 1; u < SUB; ++u) t = cadd(t, fsum[tid][u]);
      fin[tid] = t;
    }
    __syncthreads();
    if (tid == 0) {
      const double ssum = fin[0].x;
      const double2 alpha = srow[s];
      s_alpha = alpha;
      if (ssum == 0.0 && alpha.y == 0.0) {
        s_refl = 0;
        s_tau = cz(0.0, 0.0);
        s_beta = alpha.x;
        s_scale = cz(0.0, 0.0);
      } else {
        const double beta = -copysign(sqrt(alpha.x * alpha.x + alpha.y * alpha.y + ssum), alpha.x);
        const double2 den = cz(alpha.x - beta, alpha.y);
        const double dd = cabs2(den);
        s_refl = 1;
        s_tau = cz((beta - alpha.x) / beta, -alpha.y / beta);
        s_beta = beta;
        s_scale = cz(den.x / dd, -den.y / dd);
      }
      if (blockIdx.x == 0) d.tau[j] = s_tau;
    }
    __syncthreads();
    const double2 scale = s_scale, tau = s_tau, alpha = s_alpha;
    const int refl = s_refl;
    if (tid > s && tid < nbp) {
      // w_c = v^H a_c = a_c(j) + conj(scale) (x^H a_c - conj(alpha) a_c(j))
      const double2 acj = srow[tid];
      double2 w = fin[1 + tid];
      w = csub(w, cmul(cconj(alpha), acj));
      w = cadd(acj, cmul(cconj(scale), w));
      sf[tid] = refl ? cmul(cconj(tau), w) : cz(0.0, 0.0);
    }
    __syncthreads();
    double2 xs = cz(0.0, 0.0);   // vals[s] without a run-time index into the array
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (c == s) xs = vals[c];
    if (live && r >= j) {
      double2 v;
      if (r == j) {
        v = cz(1.0, 0.0);
        d.a[(size_t)j * d.lda + j] = refl ? cz(s_beta, 0.0) : alpha;
      } else {
        v = refl ? cmul(xs, scale) : xs;
        d.a[(size_t)j * d.lda + r] = v;
      }
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        if (c > s && c < nbp) {
          vals[c] = csub(vals[c], cmul(v, sf[c]));
          d.a[(size_t)(k0 + c) * d.lda + r] = vals[c];
        }
      }
    }
  }

  // partial sums of step s + 1
  const int s1 = s + 1;
  if (s1 >= nbp) return;
  const int j1 = k0 + s1;
  double2 x = cz(0.0, 0.0);
#pragma unroll
  for (int c = 0; c < NB; ++c)
    if (c == s1) x = vals[c];
  if (!(live && r >= j1)) x = cz(0.0, 0.0);
  if (live && r == j1) {
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (c >= s1 && c < nbp) sb[(s1 & 1) * NB + c] = vals[c];
  }
  double2 *pout = pb + (size_t)(s1 & 1) * nchmax * NPART + (size_t)blockIdx.x * NPART;
  {
    double q = (live && r > j1) ? cabs2(x) : 0.0;
    q = wave_sum(q);
    if (lane == 0) red[wv][0] = cz(q, 0.0);
  }
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    if (c > s1 && c < nbp) {
      double2 p = cz(0.0, 0.0);
      cfmac(p, x, vals[c]);
      p = wave_sum(p);
      if (lane == 0) red[wv][1 + c] = p;
    }
  }
  __syncthreads();
  if (tid < NPART && (tid == 0 || (tid - 1 > s1 && tid - 1 < nbp))) {
    double2 t = red[0][tid];
#pragma unroll
    for (int w = 1; w < CH / 64; ++w) t = cadd(t, red[w][tid]);
    pout[tid] = t;
  }
}

// The whole panel at k0 of a matrix whose rows from k0 on fit one workgroup
// (m - k0 <= blockDim.x <= 512): one row per thread with the row's panel
// entries in registers, the NB column steps of bqr_col_kernel carried out
// in turn with block-wide sums (wave sums, then across the waves in LDS)
// instead of one launch each, so the panel is read and written once.  The
// arithmetic of a step is that of bqr_col_kernel: x^H a_c over the rows
// r >= j, |x(2:)|^2 over r > j, LAPACK's zlarfg reflector.
constexpr int PTMAX = 512;             // threads (rows) of the one-launch panel
constexpr int PWMAX = PTMAX / 64;
template <int NB>
__global__ __launch_bounds__(PTMAX) void bqr_panel_kernel(const MatDesc *__restrict__ descs, int k0) {
  constexpr int NPART = NB + 1;
  const MatDesc d = descs[blockIdx.x];
  if (k0 >= d.n) return;
  const int nbp = min(NB, d.n - k0);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nw = blockDim.x >> 6;
  const int r = k0 + tid;
  const bool live = r < d.m;
  __shared__ double2 red[PWMAX][NPART];
  __shared__ double2 fin[NPART];
  __shared__ double2 srow[NB];
  __shared__ double2 s_scale, s_tau, s_alpha;
  __shared__ double s_beta;
  __shared__ int s_refl;
  double2 vals[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) vals[c] = ld_or0(d.a, (size_t)(k0 + c) * d.lda + r, live && c < nbp);
  for (int s = 0; s < nbp; ++s) {
    const int j = k0 + s;
    double2 x = cz(0.0, 0.0);   // vals[s] without a run-time index into the array
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (c == s) x = vals[c];
    if (live && r == j) {
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c >= s && c < nbp) srow[c] = vals[c];
    }
    const double2 xr = (live && r >= j) ? x : cz(0.0, 0.0);
    {
      double q = (live && r > j) ? cabs2(x) : 0.0;
      q = wave_sum(q);
      if (lane == 0) red[wv][0] = cz(q, 0.0);
    }
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      if (c > s && c < nbp) {
        double2 p = cz(0.0, 0.0);
        cfmac(p, xr, vals[c]);
        p = wave_sum(p);
        if (lane == 0) red[wv][1 + c] = p;
      }
    }
    __syncthreads();
    if (tid < NPART && (tid == 0 || (tid - 1 > s && tid - 1 < nbp))) {
      double2 t = red[0][tid];
      for (int w = 1; w < nw; ++w) t = cadd(t, red[w][tid]);
      fin[tid] = t;
    }
    __syncthreads();
    if (tid == 0) {
      const double ssum = fin[0].x;
      const double2 alpha = srow[s];
      s_alpha = alpha;
      if (ssum == 0.0 && alpha.y == 0.0) {
        s_refl = 0;
        s_tau = cz(0.0, 0.0);
        s_beta = alpha.x;
        s_scale = cz(0.0, 0.0);
      } else {
        const double beta = -copysign(sqrt(alpha.x * alpha.x + alpha.y * alpha.y + ssum), alpha.x);
        const double2 den = cz(alpha.x - beta, alpha.y);
        const double dd = cabs2(den);
        s_refl = 1;
        s_tau = cz((beta - alpha.x) / beta, -alpha.y / beta);
        s_beta = beta;
        s_scale = cz(den.x / dd, -den.y / dd);
      }
      d.tau[j] = s_tau;
    }
    __syncthreads();
    const double2 scale = s_scale, tau = s_tau, alpha = s_alpha;
    const int refl = s_refl;
    if (live && r >= j) {
      const double2 v = (r == j) ? cz(1.0, 0.0) : (refl ? cmul(x, scale) : x);
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        if (c > s && c < nbp) {
          // w_c = v^H a_c = a_c(j) + conj(scale) (x^H a_c - conj(alpha) a_c(j))
          const double2 acj = srow[c];
          double2 w = csub(fin[1 + c], cmul(cconj(alpha), acj));
          w = cadd(acj, cmul(cconj(scale), w));
          const double2 f = refl ? cmul(cconj(tau), w) : cz(0.0, 0.0);
          vals[c] = csub(vals[c], cmul(v, f));
        }
      }
      const double2 nv = (r == j) ? (refl ? cz(s_beta, 0.0) : alpha) : v;
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c == s) vals[c] = nv;
    }
    __syncthreads();   // srow, fin and the scalars are rewritten by the next step
  }
  if (live) {
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (c < nbp) d.a[(size_t)(k0 + c) * d.lda + r] = vals[c];
  }
}

// Y columns: which = 0 -> trailing columns of the matrix after the panel,
// which = 1 -> columns [0, rank) of d.u, which = 2 -> columns [k0, rank) of
// d.u (forming Q from the identity: the reflectors of the panel at k0 and
// later leave columns below k0 of the identity as they are).
__device__ inline void y_source(const MatDesc &d, int k0, int nbp, int which, double2 *&B, int &ldb,
                                int &nb_cols) {
  if (which == 0) {
    nb_cols = d.n - k0 - nbp;
    // after the last panel there are no trailing columns and column k0 + nbp
    // is past the end of the matrix; masked loads (ld_or0) still read B[0],
    // so B then points at the matrix's first column instead
    B = d.a + (size_t)(nb_cols > 0 ? k0 + nbp : 0) * d.lda;
    ldb = d.lda;
  } else {
    B = d.u;
    ldb = ldu_of(d);
    nb_cols = d.rank[0];
    if (which == 2) {
      // with no columns left B stays at column 0, so that masked loads
      // (ld_or0, which read B[0]) stay inside the matrix
      const bool some = k0 < nb_cols;
      B += some ? (size_t)k0 * ldb : 0;
      nb_cols = some ? nb_cols - k0 : 0;
    }
  }
}

// Element (r, c) of Y = [V | B] (the nv = NB columns of the panel's
// Householder vectors first when withV, then the ny - nv columns of B),
// zero for rows r >= rend and columns c >= ny: one load, whose base is a
// column inside its matrix also when the element is masked (ld_or0 then
// reads the base's first element).
__device__ inline double2 yel(const MatDesc &d, int k0, int nv, const double2 *B, int ldb, int ny, int r, int c,
                              int rend) {
  const bool isv = c < nv;
  const int vc = k0 + c;   // matrix column of a V column
  const bool vin = isv && vc < d.n;
  const double2 *p = isv ? d.a + (size_t)(vin ? vc : 0) * d.lda : B + (size_t)(c < ny ? c - nv : 0) * ldb;
  const bool ok = r < rend && (isv ? (vin && r > vc) : c < ny);
  const double2 x = ld_or0(p, r, ok);
  return csel(vin && r == vc && r < rend, cz(1.0, 0.0), x);
}

// P[mat][kc][i][c] = sum over rows of slice kc of conj(V[r][i]) Y[r][c],
// Y = [V | B] (withV) or B, on the FP64 matrix cores.  The slice's rows are
// staged through LDS KS at a time (coalesced loads down the columns, the
// next stage's loads issued before the current stage's products); a 16 x 16
// tile of P is one v_mfma_f64_16x16x4f64 chain per real product (four per
// complex one), the NB x YT tile of the workgroup split over its four waves
// as VhyShape says.  cend (which = 0): the trailing columns end before
// matrix column cend.
template <int NB>
__global__ __launch_bounds__(256, VhyShape<NB>::OCC) void bqr_vhy_kernel(const MatDesc *__restrict__ descs, int k0,
                                                                        int which, int withV, int cend,
                                                                        double2 *__restrict__ P, int ldp,
                                                                        int nkcmax) {
  using S = VhyShape<NB>;
  constexpr int YT = S::YT, IB = S::IB, CB = S::CB, DB = S::DB, KR = S::KR;
  static_assert(KR >= KRMIN && KR % KS == 0, "a slice is whole LDS stages");
  constexpr int NWI = NB / 16 / IB;   // waves along the rows of P
  static_assert(NWI * (YT / 16 / CB) == 4, "four waves cover the tile");
  const MatDesc d = descs[blockIdx.z];
  if (k0 >= d.n) return;
  const int nbp = min(NB, d.n - k0);
  double2 *B;
  int ldb, nb_cols;
  y_source(d, k0, nbp, which, B, ldb, nb_cols);
  if (which == 0) nb_cols = min(nb_cols, cend - (k0 + nbp));
  const int nv = withV ? NB : 0;
  const int ny = nv + max(nb_cols, 0);
  const int c0 = blockIdx.x * YT;
  if (c0 >= ny) return;
  const int rbeg = k0 + blockIdx.y * KR;
  if (rbeg >= d.m) return;
  const int rend = min(d.m, rbeg + KR);
  __shared__ double2 Vs[DB + 1][KS][NB + 1];
  __shared__ double2 Ys[DB + 1][KS][YT + 1];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int l16 = lane & 15, k4 = lane >> 4;
  const int wi = wv % NWI, wc = wv / NWI;
  dx4 re[IB][CB], im[IB][CB];
#pragma unroll
  for (int u = 0; u < IB; ++u)
#pragma unroll
    for (int v = 0; v < CB; ++v) {
      re[u][v] = dx4{0.0, 0.0, 0.0, 0.0};
      im[u][v] = re[u][v];
    }
  double2 vv[KS * NB / 256], yy[KS * YT / 256];
  auto load_stage = [&](int r0) {
#pragma unroll
    for (int u = 0; u < KS * NB / 256; ++u) {
      const int idx = tid + 256 * u, rr = idx % KS, i = idx / KS;
      const int r = r0 + rr;
      vv[u] = csel(r < rend, vel(d, k0, i, r), cz(0.0, 0.0));
    }
#pragma unroll
    for (int u = 0; u < KS * YT / 256; ++u) {
      const int idx = tid + 256 * u, rr = idx % KS, cc = idx / KS;
      yy[u] = yel(d, k0, nv, B, ldb, ny, r0 + rr, c0 + cc, rend);
    }
  };
  auto store_stage = [&](int buf) {
#pragma unroll
    for (int u = 0; u < KS * NB / 256; ++u) {
      const int idx = tid + 256 * u;
      Vs[buf][idx % KS][idx / KS] = vv[u];
    }
#pragma unroll
    for (int u = 0; u < KS * YT / 256; ++u) {
      const int idx = tid + 256 * u;
      Ys[buf][idx % KS][idx / KS] = yy[u];
    }
  };
  auto products = [&](int buf) {
#pragma unroll
    for (int kk = 0; kk < KS; kk += 4) {
      // A[i][k] = conj(V[row k][col i]) (lane l16 + 16 k4 holds A[l16][k4]),
      // B[k][c] = Y[row k][col c]
      double2 a[IB], y[CB];
#pragma unroll
      for (int u = 0; u < IB; ++u) a[u] = Vs[buf][kk + k4][16 * (wi * IB + u) + l16];
#pragma unroll
      for (int v = 0; v < CB; ++v) y[v] = Ys[buf][kk + k4][16 * (wc * CB + v) + l16];
#pragma unroll
      for (int u = 0; u < IB; ++u)
#pragma unroll
        for (int v = 0; v < CB; ++v) {
          re[u][v] = mfma_f64(a[u].x, y[v].x, re[u][v]);
          re[u][v] = mfma_f64(a[u].y, y[v].y, re[u][v]);
          im[u][v] = mfma_f64(a[u].x, y[v].y, im[u][v]);
          im[u][v] = mfma_f64(-a[u].y, y[v].x, im[u][v]);
        }
    }
  };
  load_stage(rbeg);
  if (DB) {
    int buf = 0;
    store_stage(0);
    __syncthreads();
    for (int r0 = rbeg; r0 < rend; r0 += KS) {
      const bool more = r0 + KS < rend;
      if (more) load_stage(r0 + KS);
      products(buf);
      if (more) store_stage(buf ^ 1);   // the other buffer: read by no wave since the last barrier
      __syncthreads();
      buf ^= 1;
    }
  } else {
    for (int r0 = rbeg; r0 < rend; r0 += KS) {
      store_stage(0);
      __syncthreads();
      if (r0 + KS < rend) load_stage(r0 + KS);
      products(0);
      __syncthreads();
    }
  }
  // lane l16 + 16 k4 holds P[16 (wi IB + u) + k4 + 4 e][column block's l16] in element e
  double2 *out = P + ((size_t)blockIdx.z * nkcmax + blockIdx.y) * NB * ldp;
#pragma unroll
  for (int v = 0; v < CB; ++v) {
    const int c = c0 + 16 * (wc * CB + v) + l16;
    if (c < ny) {
#pragma unroll
      for (int u = 0; u < IB; ++u)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          out[(size_t)(16 * (wi * IB + u) + k4 + 4 * e) * ldp + c] = cz(re[u][v][e], im[u][v][e]);
    }
  }
}

// T of the panel (forward, columnwise): H_0 ... H_{NB-1} = I - V T V^H.
// Diagonal blocks of 16 by the column recurrence T[i][i] = tau_i,
// T[0:i, i] = -tau_i T[0:i, 0:i] (V^H V)[0:i, i], one wave a block, the
// blocks side by side (16 steps for any NB); then adjacent blocks of h = 16, 32
// joined as T12 = -T1 (V1^H V2) T2 (the product of two block reflectors).
// V^H V from the slices of P.  Written to the matrix's T of panel k0 / NB,
// or to Tx[mat] if Tx is set (an inner panel's T, needed only until its
// update is done).
template <int NB>
__global__ __launch_bounds__(256) void bqr_t_kernel(const MatDesc *__restrict__ descs, int k0,
                                                    const double2 *__restrict__ P, int ldp, int nkcmax,
                                                    double2 *__restrict__ Tx) {
  static_assert(NB % 16 == 0 && NB <= 64, "diagonal blocks of 16, one wave each");
  const MatDesc d = descs[blockIdx.x];
  if (k0 >= d.n) return;
  const int nbp = min(NB, d.n - k0);
  constexpr int KR = VhyShape<NB>::KR;
  const int nkc = (d.m - k0 + KR - 1) / KR;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  __shared__ double2 gram[NB][NB + 1];
  __shared__ double2 Tsh[NB][NB + 1];
  __shared__ double2 X[NB / 2][NB / 2 + 1];
  const double2 *base = P + (size_t)blockIdx.x * nkcmax * NB * ldp;
  {
    // strict upper part, summed over the slices (consecutive threads along a row of P)
    double2 t[NB * NB / 256];
#pragma unroll
    for (int u = 0; u < NB * NB / 256; ++u) t[u] = cz(0.0, 0.0);
#pragma unroll 4
    for (int kc = 0; kc < nkc; ++kc) {
#pragma unroll
      for (int u = 0; u < NB * NB / 256; ++u) {
        const int idx = tid + 256 * u, i = idx % NB, g = idx / NB;
        t[u] = cadd(t[u], ld_or0(base, ((size_t)kc * NB + g) * ldp + i, g < i && i < nbp));
      }
    }
#pragma unroll
    for (int u = 0; u < NB * NB / 256; ++u) {
      const int idx = tid + 256 * u;
      gram[idx / NB][idx % NB] = t[u];
    }
    for (int idx = tid; idx < NB * (NB + 1); idx += 256) Tsh[idx / (NB + 1)][idx % (NB + 1)] = cz(0.0, 0.0);
  }
  __syncthreads();
  // diagonal blocks, all at once: wave w < NB / 16 takes block w (lane l: row 16 w + l)
  __shared__ double2 tmp[NB];
  const bool blk = wv < NB / 16 && lane < 16;
  const int o = 16 * wv;
  for (int i = 0; i < 16; ++i) {
    const int ci = o + i;
    const double2 ti = blk && ci < nbp ? d.tau[k0 + ci] : cz(0.0, 0.0);
    if (blk && lane < i) tmp[o + lane] = cmul(cz(-ti.x, -ti.y), gram[o + lane][ci]);
    __syncthreads();
    if (blk && lane < i) {
      double2 acc = cz(0.0, 0.0);
      for (int g = lane; g < i; ++g) cfma(acc, Tsh[o + lane][o + g], tmp[o + g]);
      Tsh[o + lane][ci] = acc;
    }
    if (blk && lane == i) Tsh[ci][ci] = ti;
    __syncthreads();
  }
  for (int h = 16; h < NB; h *= 2) {
    // pairs (o, o + h), o = 2 h p: X = G12 T2, then T12 = -T1 X
    const int npair = NB / (2 * h), nout = npair * h * h;
    for (int idx = tid; idx < nout; idx += 256) {
      const int p = idx / (h * h), r = (idx / h) % h, c = idx % h, o = 2 * h * p;
      double2 acc = cz(0.0, 0.0);
      for (int g = 0; g <= c; ++g) cfma(acc, gram[o + r][o + h + g], Tsh[o + h + g][o + h + c]);
      X[p * h + r][c] = acc;
    }
    __syncthreads();
    for (int idx = tid; idx < nout; idx += 256) {
      const int p = idx / (h * h), r = (idx / h) % h, c = idx % h, o = 2 * h * p;
      double2 acc = cz(0.0, 0.0);
      for (int g = r; g < h; ++g) cfma(acc, Tsh[o + r][o + g], X[p * h + g][c]);
      Tsh[o + r][o + h + c] = cz(-acc.x, -acc.y);
    }
    __syncthreads();
  }
  double2 *T = Tx ? Tx + (size_t)blockIdx.x * NB * NB : d.T + (size_t)(k0 / NB) * NB * NB;
  for (int idx = tid; idx < NB * NB; idx += 256) {
    const int r = idx % NB, c = idx / NB;
    T[idx] = (r <= c && c < nbp) ? Tsh[r][c] : cz(0.0, 0.0);
  }
}

// W2[mat][i][c] = sum_h op(T)[i][h] W[h][c], W = V^H B summed over the slices;
// op(T) = T^H (trans, QR) or T; T from Tx[mat] if Tx is set (bqr_t_kernel).
// T is upper triangular: a workgroup stages its triangle once in LDS (packed
// by columns, entry (r, c) at c (c + 1) / 2 + r, half of the square's LDS, so
// three workgroups share a CU) and then takes W2T-column tiles gridDim.x
// apart, so that a batch of many small matrices stages each T once per
// several tiles instead of once per tile.  A thread holds one column of the
// tile and the NB / 16 rows g, g + 16, ... and accumulates them side by side.
// (256-obstacle batch, 64-column panels: 1.65 ms a launch with the square T
// staged per 16-column tile at one workgroup a CU and one output at a time.)
template <int NB>
__global__ __launch_bounds__(256, 3) void bqr_w2_kernel(const MatDesc *__restrict__ descs, int k0, int which,
                                                     int withV, int trans, int cend,
                                                     const double2 *__restrict__ P, int ldp, int nkcmax,
                                                     double2 *__restrict__ W2, int ldw,
                                                     const double2 *__restrict__ Tx) {
  static_assert(W2T == 16 && NB % 16 == 0, "a thread: one column of the tile, rows 16 apart");
  constexpr int R = NB / 16;
  const MatDesc d = descs[blockIdx.y];
  if (k0 >= d.n) return;
  const int nbp = min(NB, d.n - k0);
  double2 *B;
  int ldb, nb_cols;
  y_source(d, k0, nbp, which, B, ldb, nb_cols);
  if (which == 0) nb_cols = min(nb_cols, cend - (k0 + nbp));
  if ((int)blockIdx.x * W2T >= nb_cols) return;
  const int nv = withV ? NB : 0;
  constexpr int KR = VhyShape<NB>::KR;
  const int nkc = (d.m - k0 + KR - 1) / KR;
  __shared__ double2 Tp[NB * (NB + 1) / 2];
  __shared__ double2 Ws[NB][W2T + 1];
  const int tid = threadIdx.x, cc = tid % W2T, g = tid / W2T;
  const double2 *T = Tx ? Tx + (size_t)blockIdx.y * NB * NB : d.T + (size_t)(k0 / NB) * NB * NB;
  for (int idx = tid; idx < NB * NB; idx += 256) {
    const int r = idx % NB, c = idx / NB;
    if (r <= c) Tp[c * (c + 1) / 2 + r] = T[idx];
  }
  const double2 *base = P + (size_t)blockIdx.y * nkcmax * NB * ldp;
  double2 *out = W2 + (size_t)blockIdx.y * NB * ldw;
  for (int c0 = blockIdx.x * W2T; c0 < nb_cols; c0 += gridDim.x * W2T) {
    const int c = c0 + cc;
    const bool live = c < nb_cols;
    double2 t[R];
#pragma unroll
    for (int u = 0; u < R; ++u) t[u] = cz(0.0, 0.0);
#pragma unroll 6
    for (int kc = 0; kc < nkc; ++kc) {
#pragma unroll
      for (int u = 0; u < R; ++u)
        t[u] = cadd(t[u], ld_or0(base, ((size_t)kc * NB + g + 16 * u) * ldp + nv + c, live));
    }
    __syncthreads();   // Tp staged; the previous tile's products are done with Ws
#pragma unroll
    for (int u = 0; u < R; ++u) Ws[g + 16 * u][cc] = t[u];
    __syncthreads();
    double2 acc[R];
#pragma unroll
    for (int u = 0; u < R; ++u) acc[u] = cz(0.0, 0.0);
    if (trans) {
#pragma unroll 4
      for (int h = 0; h < NB; ++h) {
        const double2 w = Ws[h][cc];
#pragma unroll
        for (int u = 0; u < R; ++u) {
          const int i = g + 16 * u;
          if (h <= i) cfmac(acc[u], Tp[i * (i + 1) / 2 + h], w);
        }
      }
    } else {
#pragma unroll 4
      for (int h = 0; h < NB; ++h) {
        const double2 w = Ws[h][cc];
#pragma unroll
        for (int u = 0; u < R; ++u) {
          const int i = g + 16 * u;
          if (h >= i) cfma(acc[u], Tp[h * (h + 1) / 2 + i], w);
        }
      }
    }
    if (live) {
#pragma unroll
      for (int u = 0; u < R; ++u) out[(size_t)(g + 16 * u) * ldw + c] = acc[u];
    }
  }
}

// C -= V W2 on the FP64 matrix cores, in transposed orientation (D = W2^T
// V^T, so that a lane's outputs run down a column: 256-byte stores).  A wave
// updates 2 x 2 tiles of 16 x 16 (32 rows x 32 columns), each a real and an
// imaginary accumulator, and loads the next k-step's fragments of W2 and V
// while it multiplies the current ones; the four waves of a workgroup stack
// along the rows (128 x 32), three workgroups a CU.  (Measured on 8 matrices
// 4608 x 1275 with 64-column panels: 51 TFLOP/s, against 40 for 32 x 64
// wave tiles at two waves a SIMD and 26 for one 16-column block a wave.)
// cend (which = 0): the trailing columns end before matrix column cend.
struct UpdShape {
  static constexpr int RB = 2;              // 16-row blocks a wave
  static constexpr int CB = 2;              // 16-column blocks a wave
  static constexpr int UR = 4 * 16 * RB;    // rows of a workgroup tile (waves along the rows)
  static constexpr int UC = 16 * CB;        // columns of a workgroup tile
};

template <int NB>
__global__ __launch_bounds__(256, 3) void bqr_update_kernel(const MatDesc *__restrict__ descs, int k0, int which,
                                                            int cend, const double2 *__restrict__ W2, int ldw) {
  using S = UpdShape;
  constexpr int RB = S::RB, CB = S::CB;
  const MatDesc d = descs[blockIdx.z];
  if (k0 >= d.n) return;
  const int nbp = min(NB, d.n - k0);
  double2 *B;
  int ldb, nb_cols;
  y_source(d, k0, nbp, which, B, ldb, nb_cols);
  if (which == 0) nb_cols = min(nb_cols, cend - (k0 + nbp));
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int l16 = lane & 15, k4 = lane >> 4;
  // this wave's first row and column (no barriers: an idle wave may leave)
  const int rw = k0 + blockIdx.y * S::UR + wv * 16 * RB;
  const int cw = blockIdx.x * S::UC;
  if (rw >= d.m || cw >= nb_cols) return;
  const int ncb = min(CB, (nb_cols - cw + 15) / 16);   // column blocks holding columns (wave-uniform)
  const int nrb = min(RB, (d.m - rw + 15) / 16);       // row blocks holding rows
  const double2 *w2 = W2 + (size_t)blockIdx.z * NB * ldw;
  dx4 re[RB][CB], im[RB][CB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      re[rb][cb] = dx4{0.0, 0.0, 0.0, 0.0};
      im[rb][cb] = re[rb][cb];
    }
  // A[c][i] = W2[i][c] (lane l16 + 16 k4 holds A[l16][k4]); B[i][r] = V[r][i]
  auto load = [&](int ks, double2 (&a)[CB], double2 (&v)[RB]) {
    const int i = 4 * ks + k4;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      const int c = cw + 16 * cb + l16;
      a[cb] = ld_or0(w2, (size_t)i * ldw + c, c < nb_cols);
    }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) v[rb] = vel(d, k0, i, rw + 16 * rb + l16);   // zero for rows >= m
  };
  auto mma = [&](const double2 (&a)[CB], const double2 (&v)[RB]) {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        if (rb >= nrb || cb >= ncb) continue;   // wave-uniform: a block with no rows or no columns
        re[rb][cb] = mfma_f64(a[cb].x, v[rb].x, re[rb][cb]);
        re[rb][cb] = mfma_f64(-a[cb].y, v[rb].y, re[rb][cb]);
        im[rb][cb] = mfma_f64(a[cb].x, v[rb].y, im[rb][cb]);
        im[rb][cb] = mfma_f64(a[cb].y, v[rb].x, im[rb][cb]);
      }
  };
  static_assert(NB % 8 == 0, "k-steps in pairs");
  double2 a0[CB], v0[RB], a1[CB], v1[RB];
  load(0, a0, v0);
#pragma unroll
  for (int ks = 0; ks < NB / 4; ks += 2) {
    load(ks + 1, a1, v1);
    mma(a0, v0);
    if (ks + 2 < NB / 4) load(ks + 2, a0, v0);
    mma(a1, v1);
  }
  // lane l16 + 16 k4 holds D[k4 + 4 e][l16] in element e of tile (rb, cb):
  // column cw + 16 cb + k4 + 4 e, row rw + 16 rb + l16
#pragma unroll
  for (int cb = 0; cb < CB; ++cb)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int c = cw + 16 * cb + k4 + 4 * e;
      if (c >= nb_cols) continue;
      double2 *col = B + (size_t)c * ldb;
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        const int r = rw + 16 * rb + l16;
        if (r < d.m) {
          const double2 x = col[r];
          col[r] = cz(x.x - re[rb][cb][e], x.y - im[rb][cb][e]);
        }
      }
    }
}

struct ApplyWork {
  DevBuf P, W2;
  int ldp = 0, ldw = 0, nkcmax = 0;
  void size(int nmat, int mmax, int ncols, int nb) {
    ldp = nb + ncols;
    ldw = std::max(ncols, 1);
    nkcmax = cdiv(std::max(mmax, 1), KRMIN);
    P.alloc((size_t)nmat * nkcmax * nb * ldp * sizeof(double2));
    W2.alloc((size_t)nmat * nb * ldw * sizeof(double2));
  }
};

// C <- (I - V T V^H)^{op} C for the panel at k0 (which/withV/trans as above).
// cend: with which = 0, the trailing columns end before matrix column cend;
// Tx: T of the panel to and from Tx[mat] instead of the matrix's T.
constexpr int kNoEnd = 0x7fffffff;
template <int NB>
void apply_panel(const MatDesc *descs, int nmat, int mmax, int ncols_max, int k0, int which, int withV,
                 int trans, ApplyWork &w, bool build_t, hipStream_t s, int cend = kNoEnd,
                 double2 *Tx = nullptr) {
  const int ny = (withV ? NB : 0) + ncols_max;
  const int nkc = cdiv(std::max(mmax - k0, 1), VhyShape<NB>::KR);
  if (ny > 0)
    hipLaunchKernelGGL(bqr_vhy_kernel<NB>, dim3(cdiv(ny, VhyShape<NB>::YT), nkc, nmat), dim3(256), 0, s, descs, k0, which, withV,
                       cend, w.P.as<double2>(), w.ldp, w.nkcmax);
  if (build_t)
    hipLaunchKernelGGL(bqr_t_kernel<NB>, dim3(nmat), dim3(256), 0, s, descs, k0, w.P.as<double2>(), w.ldp,
                       w.nkcmax, Tx);
  if (ncols_max > 0) {
    const int w2x = std::min(cdiv(ncols_max, W2T), std::max(1, cdiv(W2WG, nmat)));
    hipLaunchKernelGGL(bqr_w2_kernel<NB>, dim3(w2x, nmat), dim3(256), 0, s, descs, k0, which,
                       withV, trans, cend, w.P.as<double2>(), w.ldp, w.nkcmax, w.W2.as<double2>(), w.ldw, Tx);
    hipLaunchKernelGGL(bqr_update_kernel<NB>,
                       dim3(cdiv(ncols_max, UpdShape::UC), cdiv(std::max(mmax - k0, 1), UpdShape::UR), nmat),
                       dim3(256), 0, s, descs, k0, which, cend, w.W2.as<double2>(), w.ldw);
  }
  HIP_CHECK(hipGetLastError());
}

// Householder vectors and tau of the columns [k0, k0 + NI) (NI = 16), the
// column steps of bqr_col_kernel or the one-launch bqr_panel_kernel
struct PanelWork {
  static constexpr int NI = 16;
  DevBuf part, side;
  int nchmax = 0;
  void size(int nmat, int mmax) {
    nchmax = cdiv(mmax, CH);
    part.alloc((size_t)nmat * 2 * nchmax * (NI + 1) * sizeof(double2));
    side.alloc((size_t)nmat * 2 * NI * sizeof(double2));
  }
  void factor(const MatDesc *descs, int nmat, int mmax, int nmax, int k0, hipStream_t s) {
    const int nbp = std::min(NI, nmax - k0);
    if (mmax - k0 <= PTMAX) {
      // every matrix's remaining rows fit one workgroup: the panel in one launch
      const int threads = round_up(std::max(mmax - k0, 1), 64);
      hipLaunchKernelGGL(bqr_panel_kernel<NI>, dim3(nmat), dim3(threads), 0, s, descs, k0);
    } else {
      const int nch = cdiv(std::max(mmax - k0, 1), CH);
      for (int st = -1; st < nbp; ++st)
        hipLaunchKernelGGL(bqr_col_kernel<NI>, dim3(nch, nmat), dim3(CH), 0, s, descs, k0, st,
                           part.as<double2>(), side.as<double2>(), nchmax);
    }
    HIP_CHECK(hipGetLastError());
  }
};

// Two-level blocking: panels of NB columns (the block reflector whose T the
// matrix keeps and whose trailing update is one pass over the matrix)
// factored as NB / 16 inner panels of 16 columns, each applied only to the
// rest of its NB-column panel (its T in a scratch buffer).  NB = 16 is the
// plain one-level form.  One panel at a time (panel(K0)), so that a caller
// may act between panels (the sketched pivoted QR moves columns).
template <int NB>
struct BlockedQR {
  static constexpr int NI = PanelWork::NI;
  static_assert(NB % NI == 0, "outer panels are whole inner panels");
  const MatDesc *descs = nullptr;
  int nmat = 0, nmax = 0, mmax = 0;
  PanelWork pw;
  ApplyWork w, wi;
  DevBuf tx;
  BlockedQR(const MatDesc *d, const std::vector<MatDesc> &h) : descs(d), nmat((int)h.size()) {
    for (const auto &m : h) {
      nmax = std::max(nmax, m.n);
      mmax = std::max(mmax, m.m);
    }
    if (nmax == 0 || nmat == 0) return;
    pw.size(nmat, mmax);
    w.size(nmat, mmax, nmax, NB);
    if (NB > NI) {
      wi.size(nmat, mmax, NB - NI, NI);
      tx.alloc((size_t)nmat * NI * NI * sizeof(double2));
    }
  }
  // the panel of columns [K0, K0 + NB) and its update of the columns after it
  void panel(int K0, hipStream_t s) {
    for (int k0 = K0; k0 < std::min(K0 + NB, nmax); k0 += NI) {
      pw.factor(descs, nmat, mmax, nmax, k0, s);
      const int rest = std::min(K0 + NB, nmax) - (k0 + NI);   // inner columns still to update
      if (NB > NI && rest > 0)
        apply_panel<NI>(descs, nmat, mmax, rest, k0, 0, 1, 1, wi, true, s, K0 + NB, tx.as<double2>());
    }
    apply_panel<NB>(descs, nmat, mmax, std::max(0, nmax - K0 - NB), K0, 0, 1, 1, w, true, s);
  }
};

template <int NB>
void qr_factor_t(const MatDesc *descs, const std::vector<MatDesc> &h, hipStream_t s) {
  BlockedQR<NB> q(descs, h);
  for (int K0 = 0; K0 < q.nmax; K0 += NB) q.panel(K0, s);
}

template <int NB>
void qr_form_u_t(const MatDesc *descs, const std::vector<MatDesc> &h, int maxrank, hipStream_t s,
                 bool from_identity) {
  int nmax = 0, mmax = 0;
  for (const auto &d : h) {
    nmax = std::max(nmax, d.n);
    mmax = std::max(mmax, d.m);
  }
  const int nmat = (int)h.size();
  if (maxrank <= 0 || nmax == 0) return;
  ApplyWork w;
  w.size(nmat, mmax, maxrank, NB);
  for (int k0 = ((nmax - 1) / NB) * NB; k0 >= 0; k0 -= NB) {
    if (from_identity)
      apply_panel<NB>(descs, nmat, mmax, std::max(0, maxrank - k0), k0, 2, 0, 0, w, false, s);
    else
      apply_panel<NB>(descs, nmat, mmax, maxrank, k0, 1, 0, 0, w, false, s);
  }
}

}  // namespace

// ------------------------------------------------------- panel width tuner
// The panel width trades the panel's column steps (one reduction over all
// rows per column, whatever the width) against the passes of the trailing
// update over the matrix (one per panel): which wins depends on the
// matrices' shape and the GPU.  The first batch of a size class (the number
// of rows and of columns, each rounded to a half octave) on a GPU model
// times the QR of up to 8 of its matrices with every width, followed by the
// formation of U from the identity that every caller does next (64-wide
// reflectors: a narrower QR leaves their T to be rebuilt), and keeps the
// fastest; later batches of that class reuse it.  MFS_QR_NB = 16, 32 or 64
// fixes the width; MFS_QR_TUNE_FILE names a file that keeps the choices
// across processes (one "key width" line per class).
namespace {

// U = the first n columns of the identity (the tuner's U formation)
__global__ void tune_identity_kernel(const MatDesc *__restrict__ descs) {
  const MatDesc d = descs[blockIdx.y];
  const int c = blockIdx.x;
  if (c >= d.n) return;
  for (int r = threadIdx.x; r < d.m; r += blockDim.x) d.u[(size_t)c * d.ldu + r] = cz(r == c ? 1.0 : 0.0, 0.0);
}

std::mutex g_tune_mu;
std::map<std::string, int> g_tune;
bool g_tune_loaded = false;

int half_octave(int x) { return x <= 1 ? 0 : (int)std::floor(2.0 * std::log2((double)x)); }

std::string tune_key(int mmax, int nmax) {
  int dev = 0;
  HIP_CHECK(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIP_CHECK(hipGetDeviceProperties(&prop, dev));
  std::string arch = prop.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch = arch.substr(0, colon);
  return arch + "/m" + std::to_string(half_octave(mmax)) + "/n" + std::to_string(half_octave(nmax));
}

void tune_load() {   // g_tune_mu held
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char *f = std::getenv("MFS_QR_TUNE_FILE");
  if (!f) return;
  std::FILE *fp = std::fopen(f, "r");
  if (!fp) return;
  char key[256];
  int nb = 0;
  while (std::fscanf(fp, "%255s %d", key, &nb) == 2)
    if (nb == 16 || nb == 32 || nb == 64) g_tune[key] = nb;
  std::fclose(fp);
}

void tune_store(const std::string &key, int nb) {   // g_tune_mu held
  g_tune[key] = nb;
  if (const char *f = std::getenv("MFS_QR_TUNE_FILE")) {
    if (std::FILE *fp = std::fopen(f, "a")) {
      std::fprintf(fp, "%s %d\n", key.c_str(), nb);
      std::fclose(fp);
    }
  }
}

}  // namespace

void qr_form_u(const MatDesc *descs, const std::vector<MatDesc> &h, int maxrank, hipStream_t s,
               bool from_identity, int nb);

int qr_tuned_nb(const std::vector<MatDesc> &h, hipStream_t s) {
  if (const char *e = std::getenv("MFS_QR_NB")) {
    const int nb = std::atoi(e);
    MFS_REQUIRE(nb == 16 || nb == 32 || nb == 64, "MFS_QR_NB must be 16, 32 or 64");
    return nb;
  }
  int nmax = 0, mmax = 0;
  for (const auto &d : h) {
    nmax = std::max(nmax, d.n);
    mmax = std::max(mmax, d.m);
  }
  if (h.empty() || nmax == 0) return kQRNB;
  const std::string key = tune_key(mmax, nmax);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load();
  auto it = g_tune.find(key);
  if (it != g_tune.end()) return it->second;
  // the batch's largest matrices, copied (the QR works in place): up to 8,
  // and no more than 2^25 elements in all once the first is taken
  std::vector<int> idx(h.size());
  for (size_t i = 0; i < h.size(); ++i) idx[i] = (int)i;
  std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) {
    return (double)h[x].m * h[x].n > (double)h[y].m * h[y].n;
  });
  {
    size_t keep = 0, elems = 0;
    while (keep < idx.size() && keep < 8) {
      const size_t e = (size_t)h[idx[keep]].lda * h[idx[keep]].n;
      if (keep > 0 && elems + e > ((size_t)1 << 25)) break;
      elems += e;
      ++keep;
    }
    idx.resize(keep);
  }
  // a sample matrix of more than 2^25 elements (one matrix only) is timed on
  // its leading block of about 2^25 elements, same aspect ratio
  std::vector<int> sm(idx.size()), sn(idx.size()), sld(idx.size());
  for (size_t k = 0; k < idx.size(); ++k) {
    const MatDesc &d = h[idx[k]];
    const double f = std::min(1.0, std::sqrt((double)((size_t)1 << 25) / ((double)d.m * d.n)));
    sn[k] = std::max(1, std::min(d.n, (int)(d.n * f)));
    sm[k] = std::max(sn[k], std::min(d.m, (int)(d.m * f)));
    sld[k] = f < 1.0 ? round_up(sm[k], 16) : d.lda;
  }
  const int snmax = *std::max_element(sn.begin(), sn.end());
  std::vector<MatDesc> hc;
  std::vector<size_t> off;
  size_t tot = 0;
  for (size_t k = 0; k < idx.size(); ++k) {
    off.push_back(tot);
    // a, tau, T for the widest panel (cdiv(n, 16) panels of 64 x 64 bound
    // every width), and U (lda x n) formed from the identity
    tot += ((size_t)2 * sld[k] * sn[k] + sn[k] + (size_t)cdiv(sn[k], 16) * 64 * 64 + 16) * sizeof(double2);
  }
  DevBuf buf(tot), dd;
  for (size_t k = 0; k < idx.size(); ++k) {
    MatDesc c{};
    double2 *p = reinterpret_cast<double2 *>(static_cast<char *>(buf.p) + off[k]);
    c.a = p; c.m = sm[k]; c.n = sn[k]; c.lda = sld[k];
    c.tau = p + (size_t)c.lda * c.n;
    c.T = c.tau + c.n;
    c.u = c.T + (size_t)cdiv(c.n, 16) * 64 * 64;
    c.ldu = c.lda;
    hc.push_back(c);
  }
  DevBuf ranks(hc.size() * sizeof(int));
  {
    std::vector<int> rk(hc.size());
    for (size_t k = 0; k < hc.size(); ++k) {
      rk[k] = hc[k].n;
      hc[k].rank = ranks.as<int>() + k;
    }
    HIP_CHECK(hipMemcpyAsync(ranks.p, rk.data(), rk.size() * sizeof(int), hipMemcpyHostToDevice, s));
    HIP_CHECK(hipStreamSynchronize(s));   // rk goes out of scope
  }
  dd.alloc(hc.size() * sizeof(MatDesc));
  HIP_CHECK(hipMemcpyAsync(dd.p, hc.data(), hc.size() * sizeof(MatDesc), hipMemcpyHostToDevice, s));
  hipEvent_t e0, e1;
  HIP_CHECK(hipEventCreate(&e0));
  HIP_CHECK(hipEventCreate(&e1));
  int best = kQRNB;
  float best_ms = 0.f;
  std::string report;
  for (int nb : {16, 32, 64}) {
    float ms = 0.f;
    // the first run loads the kernels; it is repeated unless it ran long
    // enough (50 ms) for the load to be lost in it
    for (int rep = 0; rep < 2 && (rep == 0 || ms < 50.f); ++rep) {
      for (size_t k = 0; k < idx.size(); ++k)
        HIP_CHECK(hipMemcpy2DAsync(hc[k].a, (size_t)hc[k].lda * sizeof(double2), h[idx[k]].a,
                                   (size_t)h[idx[k]].lda * sizeof(double2), (size_t)hc[k].m * sizeof(double2),
                                   hc[k].n, hipMemcpyDeviceToDevice, s));
      hipLaunchKernelGGL(tune_identity_kernel, dim3(snmax, (int)hc.size()), dim3(256), 0, s, dd.as<MatDesc>());
      HIP_CHECK(hipEventRecord(e0, s));
      qr_factor(dd.as<MatDesc>(), hc, s, nb);
      qr_form_u(dd.as<MatDesc>(), hc, snmax, s, true, nb);
      HIP_CHECK(hipEventRecord(e1, s));
      HIP_CHECK(hipEventSynchronize(e1));
      HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
    }
    report += " " + std::to_string(nb) + ": " + std::to_string(ms) + " ms";
    if (nb == 16 || ms < best_ms) { best = nb; best_ms = ms; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  progress("QR panel width for %s: %d (%s)", key.c_str(), best, report.c_str());
  tune_store(key, best);
  return best;
}

// One 32-column panel at a time (the panel width of the pivoted QR's T
// factors), for callers that act between panels.
struct QRPanels32::Impl {
  BlockedQR<32> q;
  Impl(const MatDesc *d, const std::vector<MatDesc> &h) : q(d, h) {}
};
QRPanels32::QRPanels32(const MatDesc *descs, const std::vector<MatDesc> &h) : impl(new Impl(descs, h)) {}
QRPanels32::~QRPanels32() { delete impl; }
void QRPanels32::panel(int K0, hipStream_t s) { impl->q.panel(K0, s); }

void qr_factor(const MatDesc *descs, const std::vector<MatDesc> &h, hipStream_t s, int nb) {
  switch (nb) {
    case 16: qr_factor_t<16>(descs, h, s); break;
    case 32: qr_factor_t<32>(descs, h, s); break;
    case 64: qr_factor_t<64>(descs, h, s); break;
    default: MFS_THROW(MFS_EINVAL, "QR panel width must be 16, 32 or 64");
  }
}

// Form U = Q [U_R; 0] in place in d.u (leading dimension d.ldu, or d.lda if
// zero); rows >= n of d.u must be zero.  T of every panel (of width nb, the
// width the QR ran with) must be present.  from_identity: d.u holds the
// first rank columns of the identity, so the panel at k0 updates its
// columns k0 and later only.
//
// Forming U is all trailing-update work (no panel to factor), so it always
// runs with 64-column block reflectors, whatever width the QR ran with:
// for a QR of panels of 16 or 32 columns, T of every 64 consecutive
// reflectors is formed first from their Householder vectors and tau
// (V^H V and the forward recurrence, as bqr_t_kernel does after a panel)
// into a buffer of its own, and U is formed with those.
void qr_form_u(const MatDesc *descs, const std::vector<MatDesc> &h, int maxrank, hipStream_t s,
               bool from_identity, int nb) {
  MFS_REQUIRE(nb == 16 || nb == 32 || nb == 64, "QR panel width must be 16, 32 or 64");
  int nmax = 0, mmax = 0;
  for (const auto &d : h) {
    nmax = std::max(nmax, d.n);
    mmax = std::max(mmax, d.m);
  }
  const int nmat = (int)h.size();
  if (maxrank <= 0 || nmax == 0 || nmat == 0) return;
  if (nb == 64 || nmax <= nb) {
    switch (nb) {
      case 16: qr_form_u_t<16>(descs, h, maxrank, s, from_identity); break;
      case 32: qr_form_u_t<32>(descs, h, maxrank, s, from_identity); break;
      default: qr_form_u_t<64>(descs, h, maxrank, s, from_identity); break;
    }
    return;
  }
  std::vector<MatDesc> h2(h);
  std::vector<size_t> off(nmat);
  size_t tot = 0;
  for (int i = 0; i < nmat; ++i) {
    off[i] = tot;
    tot += (size_t)cdiv(std::max(h[i].n, 1), 64) * 64 * 64;
  }
  DevBuf t64(tot * sizeof(double2)), d2(nmat * sizeof(MatDesc));
  for (int i = 0; i < nmat; ++i) h2[i].T = t64.as<double2>() + off[i];
  HIP_CHECK(hipMemcpyAsync(d2.p, h2.data(), nmat * sizeof(MatDesc), hipMemcpyHostToDevice, s));
  {
    ApplyWork w;
    w.size(nmat, mmax, 0, 64);
    for (int k0 = 0; k0 < nmax; k0 += 64)   // V^H V of the group only (no trailing columns), then T
      apply_panel<64>(d2.as<MatDesc>(), nmat, mmax, 0, k0, 0, 1, 1, w, true, s, k0 + 64);
  }
  qr_form_u_t<64>(d2.as<MatDesc>(), h2, maxrank, s, from_identity);
}

}  // namespace mfs
