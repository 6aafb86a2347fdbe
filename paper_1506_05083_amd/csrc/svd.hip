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
// Blocked form for the GPU: the columns are cut into blocks of JB (16, or 32
// once a batch's widest matrix has kJacWideMinCols columns) and the
// round-robin (circle) schedule pairs the blocks, n_b - 1 rounds per sweep.
// A task is a block pair (JC = 2 JB columns); a round is three launches over
// all tasks of all matrices:
//   1. jac_gram_mfma_kernel (JB = 16) / jac_gram_mfma32_kernel (JB = 32):
//      partial H = G_IJ^H G_IJ (JC x JC) over 128-row tiles on the FP64
//      matrix cores, every entry a dot product of two columns;
//   2. jac_inner_kernel (one workgroup per task): H summed over the tiles,
//      one Jacobi sweep over the JC columns carried out on H in LDS (the
//      two-sided update H <- R^H H R of each rotation R, with the exact
//      diagonal formulas above and the annihilated entry set to zero), the
//      product J of the rotations accumulated alongside;
//   3. jac_apply_mfma_kernel / jac_apply_mfma32_kernel: if any pair of the
//      task rotated, G_IJ <- G_IJ J and V_IJ <- V_IJ J over row tiles.
// The row tiles spread every round over the whole chip whatever the number
// of tasks, and the apply streams G and V once per round.
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

constexpr int kJacWideMinCols = 2048;  // 32-column blocks from this width on

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

constexpr int GT = 128;   // rows per workgroup of the partial Gram matrices
constexpr int AT = 64;    // rows per workgroup of the rotation apply

// Blocks (bi, bj) of block pair `pair` of matrix d in this round (blocks of
// JB columns); false if the pair is out of range or both blocks are padding.
template <int JB>
__device__ inline bool task_blocks(const MatDesc &d, int round, int pair, int &bi, int &bj, int &nb) {
  nb = (d.n + JB - 1) / JB;
  const int nbp = nb + (nb & 1);
  // a matrix runs its own nbp - 1 rounds, whatever else is in the batch, so
  // that its factors do not depend on its batch-mates
  if (pair >= nbp / 2 || round >= nbp - 1) return false;
  circle_pair(nbp, round, pair, bi, bj);
  return bi < nb || bj < nb;
}
// column of local index a of the task (-1: past n or in the padding block)
template <int JB>
__device__ inline int task_col(int a, int bi, int bj, int nb, int n) {
  const int blk = a < JB ? bi : bj;
  const int c = blk * JB + (a & (JB - 1));
  return (blk < nb && c < n) ? c : -1;
}

// Converged pairs.  A block pair found converged (no rotation) needs no new
// check until one of its blocks turns: bmod[mat][blk] is the round (counted
// over sweeps) in which block blk last turned, pchk[mat][a][b] (a < b) the
// round in which the pair was last found converged, -1 for never.  The Gram
// matrix and inner sweep of such a pair would reproduce the same verdict from
// the same columns, so skipping them changes no result.
struct JacClean {
  int *bmod, *pchk;
  int *nchk;   // [mat] pairs checked (not skipped) in the current sweep
  int nbp;
};
__device__ inline bool jac_clean(const JacClean &cs, int mat, int bi, int bj) {
  const int a = min(bi, bj), b = max(bi, bj);
  const int c = cs.pchk[((size_t)mat * cs.nbp + a) * cs.nbp + b];
  return c >= 0 && c > cs.bmod[mat * cs.nbp + bi] && c > cs.bmod[mat * cs.nbp + bj];
}
__global__ void jac_clean_init(JacClean cs, int nmat) {
  const long n = (long)nmat * cs.nbp * (cs.nbp + 1);
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    cs.bmod[i] = -1;   // bmod and pchk are one allocation
}
__global__ void jac_clear_checks(JacClean cs, int nmat) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nmat) cs.nchk[i] = 0;
}

// 2. one workgroup per task: H = sum of the partials, one Jacobi sweep over
//    its JC columns on H, J = product of the rotations -> jbuf, rot = any rotation
template <int JB>
__global__ __launch_bounds__(JB * JB) void jac_inner_kernel(const MatDesc *__restrict__ descs,
                                                        const int *__restrict__ act, int round, double tol_eps,
                                                        const double2 *__restrict__ hpart,
                                                        double2 *__restrict__ jbuf, int *__restrict__ rot,
                                                        int npair_max, int ntile_max, JacClean cs, int gr) {
  constexpr int JC = 2 * JB, IT = JB * JB;   // one 2 x 2 block of H per thread
  const int mat = blockIdx.y;
  if (!act[mat]) return;
  const MatDesc d = descs[mat];
  const int pair = blockIdx.x;
  int tbi, tbj;
  {
    int nb;
    if (!task_blocks<JB>(d, round, pair, tbi, tbj, nb)) return;
  }
  if (jac_clean(cs, mat, tbi, tbj)) {   // uniform; nothing of this pair changes this round
    if (threadIdx.x == 0) rot[(size_t)mat * npair_max + pair] = 0;
    return;
  }
  __shared__ double2 Hs[JC][JC + 1];
  __shared__ double2 Js[JC][JC + 1];
  __shared__ double r_c[JB], r_tg[JB], r_a[JB], r_b[JB];
  __shared__ double2 r_se[JB];
  __shared__ int r_act[JB];
  __shared__ int s_nrot;
  const int tid = threadIdx.x;
  const int ntile = (d.n + GT - 1) / GT;
  // relative orthogonality reachable in floating point, ~ sqrt(n) eps of this
  // matrix (the stopping rule of LAPACK's one-sided Jacobi)
  const double tol = tol_eps * sqrt((double)d.n), tol2 = tol * tol;
  const double2 *hp = hpart + ((size_t)mat * npair_max + pair) * ntile_max * JC * JC;
  {
    double2 h[JC * JC / IT];
#pragma unroll
    for (int u = 0; u < JC * JC / IT; ++u) h[u] = cz(0.0, 0.0);
    for (int t = 0; t < ntile; ++t) {
#pragma unroll
      for (int u = 0; u < JC * JC / IT; ++u) h[u] = cadd(h[u], hp[(size_t)t * JC * JC + tid + IT * u]);
    }
#pragma unroll
    for (int u = 0; u < JC * JC / IT; ++u) {
      const int idx = tid + IT * u;
      Hs[idx / JC][idx % JC] = h[u];
      Js[idx / JC][idx % JC] = cz(idx / JC == idx % JC ? 1.0 : 0.0, 0.0);
    }
  }
  if (tid == 0) s_nrot = 0;
  __syncthreads();
  // one sweep over the JC columns on H.  Rotation of pair (p, q) from
  // a = H_pp, b = H_qq, gamma = H_pq, d = b - a:
  //   q' = 2 sign(d) / (|d| + sqrt(d^2 + 4 |gamma|^2)),  t = q' |gamma|,
  //   c = 1 / sqrt(1 + t^2),  s e^{i th} = c q' gamma,  t |gamma| = q' |gamma|^2
  // (the formulas of the header with zeta = d / (2 |gamma|), |gamma| never formed).
  // H <- R^H H R acts on every 2 x 2 block (rows of pair i, columns of pair j)
  // on its own: JB x JB blocks over the threads, J <- J R alongside.
  for (int rnd = 0; rnd < JC - 1; ++rnd) {
    if (tid < JB) {
      int p, q;
      circle_pair(JC, rnd, tid, p, q);
      const double a = Hs[p][p].x, b = Hs[q][q].x;
      const double2 gam = Hs[p][q];
      const double g2 = cabs2(gam);
      const int on = g2 > tol2 * a * b;
      if (on) {
        const double dd = b - a;
        const double qq = copysign(2.0, dd) / (fabs(dd) + sqrt(fma(dd, dd, 4.0 * g2)));
        const double cs = rsqrt(fma(qq * qq, g2, 1.0));
        r_c[tid] = cs;
        r_se[tid] = cz(cs * qq * gam.x, cs * qq * gam.y);
        r_tg[tid] = qq * g2;
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
      {
        // H block (pair i rows, pair j columns)
        const int bi = tid / JB, bj = tid % JB;
        int p, q, u, v;
        circle_pair(JC, rnd, bi, p, q);
        circle_pair(JC, rnd, bj, u, v);
        const int ai = r_act[bi], aj = r_act[bj];
        if (ai || aj) {
          double2 h_pu = Hs[p][u], h_pv = Hs[p][v], h_qu = Hs[q][u], h_qv = Hs[q][v];
          if (bi == bj) {
            // pivot block: exact values
            h_pu = cz(r_a[bi] - r_tg[bi], 0.0);
            h_qv = cz(r_b[bi] + r_tg[bi], 0.0);
            h_pv = cz(0.0, 0.0);
            h_qu = cz(0.0, 0.0);
          } else {
            if (aj) {   // columns: [x_u, x_v] <- [c x_u - conj(se) x_v, se x_u + c x_v]
              const double cs = r_c[bj];
              const double2 se = r_se[bj], sec = cconj(r_se[bj]);
              const double2 pu = csub(cscale(h_pu, cs), cmul(sec, h_pv));
              const double2 pv = cadd(cmul(se, h_pu), cscale(h_pv, cs));
              const double2 qu = csub(cscale(h_qu, cs), cmul(sec, h_qv));
              const double2 qv = cadd(cmul(se, h_qu), cscale(h_qv, cs));
              h_pu = pu; h_pv = pv; h_qu = qu; h_qv = qv;
            }
            if (ai) {   // rows: [y_p; y_q] <- [c y_p - se y_q; conj(se) y_p + c y_q]
              const double cs = r_c[bi];
              const double2 se = r_se[bi], sec = cconj(r_se[bi]);
              const double2 pu = csub(cscale(h_pu, cs), cmul(se, h_qu));
              const double2 qu = cadd(cmul(sec, h_pu), cscale(h_qu, cs));
              const double2 pv = csub(cscale(h_pv, cs), cmul(se, h_qv));
              const double2 qv = cadd(cmul(sec, h_pv), cscale(h_qv, cs));
              h_pu = pu; h_pv = pv; h_qu = qu; h_qv = qv;
            }
          }
          Hs[p][u] = h_pu; Hs[p][v] = h_pv; Hs[q][u] = h_qu; Hs[q][v] = h_qv;
        }
        // J columns of pair bj, rows 2 bi and 2 bi + 1
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int k = 2 * bi + e;
          if (aj) {
            const double cs = r_c[bj];
            const double2 se = r_se[bj], sec = cconj(r_se[bj]);
            const double2 x = Js[k][u], y = Js[k][v];
            Js[k][u] = csub(cscale(x, cs), cmul(sec, y));
            Js[k][v] = cadd(cmul(se, x), cscale(y, cs));
          }
        }
      }
    }
    __syncthreads();   // H, J and the flags of this round settled before the next
  }
  double2 *jo = jbuf + ((size_t)mat * npair_max + pair) * JC * JC;
  for (int idx = tid; idx < JC * JC; idx += IT) jo[idx] = Js[idx / JC][idx % JC];
  if (tid == 0) {
    rot[(size_t)mat * npair_max + pair] = s_nrot > 0;
    atomicAdd(cs.nchk + mat, 1);
    if (s_nrot > 0) {
      atomicAdd(d.flag, 1);
      cs.bmod[mat * cs.nbp + tbi] = gr;
      cs.bmod[mat * cs.nbp + tbj] = gr;
    } else {
      cs.pchk[((size_t)mat * cs.nbp + min(tbi, tbj)) * cs.nbp + max(tbi, tbj)] = gr;
    }
  }
}

// FP64 matrix-core forms of steps 1 and 3 for 16-column blocks (mfma_f64:
// lane layout in common.hpp); a complex product is four real ones on the
// split real and imaginary parts.

// 1'. partial Gram matrix of one GT-row tile, one wave per workgroup.  The
//     rows are the summation index: step s takes rows 4 s + k of the tile, and
//     the fragment a lane loads (row 4 s + k of task column c) is at once its
//     A operand (conj(G)^T) and its B operand (G), for the column blocks
//     (0, 0), (0, 1) and (1, 1); block (1, 0) is the conjugate transpose of
//     (0, 1).
__global__ __launch_bounds__(64) void jac_gram_mfma_kernel(const MatDesc *__restrict__ descs,
                                                           const int *__restrict__ act, int round,
                                                           double2 *__restrict__ hpart, int npair_max,
                                                           int ntile_max, JacClean cs) {
  constexpr int JB = 16, JC = 32, KB = 8;
  const int mat = blockIdx.z;
  if (!act[mat]) return;
  const MatDesc d = descs[mat];
  const int n = d.n;
  const int rbeg = blockIdx.x * GT;
  if (rbeg >= n) return;
  int bi, bj, nb;
  if (!task_blocks<JB>(d, round, blockIdx.y, bi, bj, nb)) return;
  if (jac_clean(cs, mat, bi, bj)) return;   // converged and unchanged since
  const int l = threadIdx.x, c = l & 15, k = l >> 4;
  const int c0 = task_col<JB>(c, bi, bj, nb, n), c1 = task_col<JB>(JB + c, bi, bj, nb, n);
  const double2 *g0 = d.g + (size_t)max(c0, 0) * d.ldg, *g1 = d.g + (size_t)max(c1, 0) * d.ldg;
  const int rend = min(n, rbeg + GT);
  dx4 r00 = {0, 0, 0, 0}, i00 = r00, r01 = r00, i01 = r00, r11 = r00, i11 = r00;
  for (int rb = rbeg; rb < rend; rb += 4 * KB) {   // uniform trip count
    double2 x0[KB], x1[KB];
#pragma unroll
    for (int s = 0; s < KB; ++s) {
      const int r = rb + 4 * s + k;
      x0[s] = ld_or0(g0, r, r < rend && c0 >= 0);
      x1[s] = ld_or0(g1, r, r < rend && c1 >= 0);
    }
#pragma unroll
    for (int s = 0; s < KB; ++s) {
      // conj(x_I)^T x_J: real part xr^T xr + xi^T xi, imaginary xr^T xi - xi^T xr
      r00 = mfma_f64(x0[s].x, x0[s].x, r00);
      r00 = mfma_f64(x0[s].y, x0[s].y, r00);
      i00 = mfma_f64(x0[s].x, x0[s].y, i00);
      i00 = mfma_f64(-x0[s].y, x0[s].x, i00);
      r01 = mfma_f64(x0[s].x, x1[s].x, r01);
      r01 = mfma_f64(x0[s].y, x1[s].y, r01);
      i01 = mfma_f64(x0[s].x, x1[s].y, i01);
      i01 = mfma_f64(-x0[s].y, x1[s].x, i01);
      r11 = mfma_f64(x1[s].x, x1[s].x, r11);
      r11 = mfma_f64(x1[s].y, x1[s].y, r11);
      i11 = mfma_f64(x1[s].x, x1[s].y, i11);
      i11 = mfma_f64(-x1[s].y, x1[s].x, i11);
    }
  }
  double2 *out = hpart + (((size_t)mat * npair_max + blockIdx.y) * ntile_max + blockIdx.x) * JC * JC;
  const int j = l & 15, g = l >> 4;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = g + 4 * v;
    out[i * JC + j] = cz(r00[v], i00[v]);
    out[(JB + i) * JC + JB + j] = cz(r11[v], i11[v]);
    out[i * JC + JB + j] = cz(r01[v], i01[v]);
    out[(JB + j) * JC + i] = cz(r01[v], -i01[v]);
  }
}

// 3'. G_IJ <- G_IJ J and V_IJ <- V_IJ J: one wave per 64-row tile (tiles
//     [0, nt) of G, [nt, 2 nt) of V), four 16-row blocks and all 32 task
//     columns, so that each fragment of J serves four row blocks; step s sums
//     over task columns 4 s .. 4 s + 3.  The wave reads its rows of every
//     column before it writes any, and tiles share no rows, so the update is
//     in place.
__global__ __launch_bounds__(64) void jac_apply_mfma_kernel(const MatDesc *__restrict__ descs,
                                                            const int *__restrict__ act, int round,
                                                            const double2 *__restrict__ jbuf,
                                                            const int *__restrict__ rot, int npair_max) {
  constexpr int JB = 16, JC = 32, KS = JC / 4, RB = AT / 16;
  const int mat = blockIdx.z;
  if (!act[mat]) return;
  const MatDesc d = descs[mat];
  const int n = d.n;
  const int pair = blockIdx.y;
  const int nt = (n + AT - 1) / AT;
  if ((int)blockIdx.x >= 2 * nt) return;
  int bi, bj, nb;
  if (!task_blocks<JB>(d, round, pair, bi, bj, nb)) return;
  if (!rot[(size_t)mat * npair_max + pair]) return;
  const int l = threadIdx.x;
  const int r0 = ((int)blockIdx.x % nt) * AT;
  double2 *M = (int)blockIdx.x < nt ? d.g : d.v;
  const double2 *ji = jbuf + ((size_t)mat * npair_max + pair) * JC * JC;
  const int i = l & 15, k = l >> 4;
  double2 b0[KS], b1[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    b0[s] = ji[(4 * s + k) * JC + i];
    b1[s] = ji[(4 * s + k) * JC + JB + i];
  }
  dx4 re0[RB], im0[RB], re1[RB], im1[RB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    re0[rb] = dx4{0, 0, 0, 0};
    im0[rb] = re0[rb];
    re1[rb] = re0[rb];
    im1[rb] = re0[rb];
  }
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const int col = task_col<JB>(4 * s + k, bi, bj, nb, n);
    const double2 *mc = M + (size_t)max(col, 0) * d.ldg;
    double2 a[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const int r = r0 + 16 * rb + i;
      a[rb] = ld_or0(mc, r, r < n && col >= 0);
    }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      re0[rb] = mfma_f64(a[rb].x, b0[s].x, re0[rb]);
      re0[rb] = mfma_f64(-a[rb].y, b0[s].y, re0[rb]);
      im0[rb] = mfma_f64(a[rb].x, b0[s].y, im0[rb]);
      im0[rb] = mfma_f64(a[rb].y, b0[s].x, im0[rb]);
      re1[rb] = mfma_f64(a[rb].x, b1[s].x, re1[rb]);
      re1[rb] = mfma_f64(-a[rb].y, b1[s].y, re1[rb]);
      im1[rb] = mfma_f64(a[rb].x, b1[s].y, im1[rb]);
      im1[rb] = mfma_f64(a[rb].y, b1[s].x, im1[rb]);
    }
  }
  const int j = l & 15, g = l >> 4;
  const int cA = task_col<JB>(j, bi, bj, nb, n), cB = task_col<JB>(JB + j, bi, bj, nb, n);
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = r0 + 16 * rb + g + 4 * v;
      if (row < n) {
        if (cA >= 0) M[(size_t)cA * d.ldg + row] = cz(re0[rb][v], im0[rb][v]);
        if (cB >= 0) M[(size_t)cB * d.ldg + row] = cz(re1[rb][v], im1[rb][v]);
      }
    }
}

// 1''. partial Gram matrix for 32-column blocks (64 task columns, four
//      16-column fragments per step), two waves per GT-row tile: the ten
//      block pairs (I <= J) of the Hermitian 64 x 64 matrix, five per wave
//      (wave 0: (0,0) (0,1) (0,2) (0,3) (1,1); wave 1: (1,2) (1,3) (2,2)
//      (2,3) (3,3)); the blocks below the diagonal are written as conjugate
//      transposes.
__device__ inline void gram32_pair(int w, int p, int &I, int &J) {
  // pairs (I <= J) in row order, the first five to wave 0
  const int q = 5 * w + p;
  const int rows[10] = {0, 0, 0, 0, 1, 1, 1, 2, 2, 3}, cols[10] = {0, 1, 2, 3, 1, 2, 3, 2, 3, 3};
  I = rows[q];
  J = cols[q];
}

__global__ __launch_bounds__(128) void jac_gram_mfma32_kernel(const MatDesc *__restrict__ descs,
                                                              const int *__restrict__ act, int round,
                                                              double2 *__restrict__ hpart, int npair_max,
                                                              int ntile_max, JacClean cs) {
  constexpr int JB = 32, JC = 64, NF = 4, NP = 5;
  const int mat = blockIdx.z;
  if (!act[mat]) return;
  const MatDesc d = descs[mat];
  const int n = d.n;
  const int rbeg = blockIdx.x * GT;
  if (rbeg >= n) return;
  int bi, bj, nb;
  if (!task_blocks<JB>(d, round, blockIdx.y, bi, bj, nb)) return;
  if (jac_clean(cs, mat, bi, bj)) return;   // converged and unchanged since
  const int l = threadIdx.x & 63, c = l & 15, k = l >> 4;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int cf[NF];
  const double2 *gf[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    cf[f] = task_col<JB>(16 * f + c, bi, bj, nb, n);
    gf[f] = d.g + (size_t)max(cf[f], 0) * d.ldg;
  }
  const int rend = min(n, rbeg + GT);
  dx4 re[NP], im[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    re[p] = dx4{0, 0, 0, 0};
    im[p] = re[p];
  }
  for (int rb = rbeg; rb < rend; rb += 4) {   // uniform trip count
    const int r = rb + k;
    double2 x[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) x[f] = ld_or0(gf[f], r, r < rend && cf[f] >= 0 && (w == 1 ? f > 0 : true));
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      int I, J;
      gram32_pair(w, p, I, J);
      // I, J are wave-uniform: the selects below stay in registers
      double2 xi = x[0], xj = x[0];
#pragma unroll
      for (int f = 1; f < NF; ++f) {
        xi = csel(I == f, x[f], xi);
        xj = csel(J == f, x[f], xj);
      }
      re[p] = mfma_f64(xi.x, xj.x, re[p]);
      re[p] = mfma_f64(xi.y, xj.y, re[p]);
      im[p] = mfma_f64(xi.x, xj.y, im[p]);
      im[p] = mfma_f64(-xi.y, xj.x, im[p]);
    }
  }
  double2 *out = hpart + (((size_t)mat * npair_max + blockIdx.y) * ntile_max + blockIdx.x) * JC * JC;
  const int j = l & 15, g = l >> 4;
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    int I, J;
    gram32_pair(w, p, I, J);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = g + 4 * v;
      out[(16 * I + i) * JC + 16 * J + j] = cz(re[p][v], im[p][v]);
      if (I != J) out[(16 * J + j) * JC + 16 * I + i] = cz(re[p][v], -im[p][v]);
    }
  }
}

// 3''. G_IJ <- G_IJ J and V_IJ <- V_IJ J for 32-column blocks: one wave per
//      16-row tile (tiles [0, nt) of G, [nt, 2 nt) of V) against all 64 task
//      columns, step s summing over task columns
//      4 s .. 4 s + 3 with the fragments of J read as they are needed.  The
//      wave reads its rows of every column before it writes any, and tiles
//      share no rows, so the update is in place.
__global__ __launch_bounds__(64) void jac_apply_mfma32_kernel(const MatDesc *__restrict__ descs,
                                                              const int *__restrict__ act, int round,
                                                              const double2 *__restrict__ jbuf,
                                                              const int *__restrict__ rot, int npair_max) {
  constexpr int JB = 32, JC = 64, KS = JC / 4, NF = 4, RB = 1, TR = 16 * RB;
  const int mat = blockIdx.z;
  if (!act[mat]) return;
  const MatDesc d = descs[mat];
  const int n = d.n;
  const int pair = blockIdx.y;
  const int nt = (n + TR - 1) / TR;
  if ((int)blockIdx.x >= 2 * nt) return;
  int bi, bj, nb;
  if (!task_blocks<JB>(d, round, pair, bi, bj, nb)) return;
  if (!rot[(size_t)mat * npair_max + pair]) return;
  const int l = threadIdx.x;
  const int r0 = ((int)blockIdx.x % nt) * TR;
  double2 *M = (int)blockIdx.x < nt ? d.g : d.v;
  const double2 *ji = jbuf + ((size_t)mat * npair_max + pair) * JC * JC;
  const int i = l & 15, k = l >> 4;
  dx4 re[RB][NF], im[RB][NF];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int J = 0; J < NF; ++J) {
      re[rb][J] = dx4{0, 0, 0, 0};
      im[rb][J] = re[rb][J];
    }
#pragma unroll 2
  for (int s = 0; s < KS; ++s) {
    const int col = task_col<JB>(4 * s + k, bi, bj, nb, n);
    const double2 *mc = M + (size_t)max(col, 0) * d.ldg;
    double2 a[RB], b[NF];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const int r = r0 + 16 * rb + i;
      a[rb] = ld_or0(mc, r, r < n && col >= 0);
    }
#pragma unroll
    for (int J = 0; J < NF; ++J) b[J] = ji[(4 * s + k) * JC + 16 * J + i];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int J = 0; J < NF; ++J) {
        re[rb][J] = mfma_f64(a[rb].x, b[J].x, re[rb][J]);
        re[rb][J] = mfma_f64(-a[rb].y, b[J].y, re[rb][J]);
        im[rb][J] = mfma_f64(a[rb].x, b[J].y, im[rb][J]);
        im[rb][J] = mfma_f64(a[rb].y, b[J].x, im[rb][J]);
      }
  }
  const int j = l & 15, g = l >> 4;
#pragma unroll
  for (int J = 0; J < NF; ++J) {
    const int cJ = task_col<JB>(16 * J + j, bi, bj, nb, n);
    if (cJ < 0) continue;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = r0 + 16 * rb + g + 4 * v;
        if (row < n) M[(size_t)cJ * d.ldg + row] = cz(re[rb][J][v], im[rb][J][v]);
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

namespace {

template <int JB>
JacStats jac_run_t(const MatDesc *descs, const std::vector<MatDesc> &h, int init_mode, hipStream_t s) {
  constexpr int JC = 2 * JB;
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
    for (int r = 0; r < nbp - 1; ++r)
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
  std::vector<int> flags(nmat), checked(nmat), active(nmat, 1);
  DevBuf act((size_t)nmat * sizeof(int));
  const int npair_max = std::max(1, nbpmax / 2);
  const int ntile_max = cdiv(nmax, GT), atile_max = cdiv(nmax, AT);
  DevBuf hpart((size_t)nmat * npair_max * ntile_max * JC * JC * sizeof(double2));
  DevBuf jbuf((size_t)nmat * npair_max * JC * JC * sizeof(double2));
  DevBuf rotf((size_t)nmat * npair_max * sizeof(int));
  const size_t ncl = (size_t)nmat * nbpmax * (nbpmax + 1);
  DevBuf cleanbuf((ncl + nmat) * sizeof(int));
  JacClean cs{cleanbuf.as<int>(), cleanbuf.as<int>() + (size_t)nmat * nbpmax, cleanbuf.as<int>() + ncl, nbpmax};
  hipLaunchKernelGGL(jac_clean_init, dim3(std::min(1024, cdiv(nmat * nbpmax * (nbpmax + 1), 256))), dim3(256), 0,
                     s, cs, nmat);
  HIP_CHECK(hipGetLastError());
  // rotation threshold 4 sqrt(n) eps, n of each matrix (set in the kernel)
  const double tol = 4.0 * 2.220446049250313e-16;
  // sweep cap; MFS_JACOBI_MAX_SWEEPS lowers it (a test of the not-converged
  // status forces a cap of one sweep)
  int max_sweeps = 40;
  if (const char *e = getenv("MFS_JACOBI_MAX_SWEEPS")) max_sweeps = std::max(1, std::min(40, atoi(e)));
  const bool dbg = getenv("MFS_DEBUG") != nullptr;
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    HIP_CHECK(hipMemcpyAsync(act.p, active.data(), nmat * sizeof(int), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(jac_clear_flags, dim3(cdiv(nmat, 256)), dim3(256), 0, s, descs, nmat);
    hipLaunchKernelGGL(jac_clear_checks, dim3(cdiv(nmat, 256)), dim3(256), 0, s, cs, nmat);
    HIP_CHECK(hipEventRecord(e0, s));
    for (int rnd = 0; rnd < rounds; ++rnd) {
      if (JB == 16)
        hipLaunchKernelGGL(jac_gram_mfma_kernel, dim3(ntile_max, npair_max, nmat), dim3(64), 0, s, descs,
                           act.as<int>(), rnd, hpart.as<double2>(), npair_max, ntile_max, cs);
      else
        hipLaunchKernelGGL(jac_gram_mfma32_kernel, dim3(ntile_max, npair_max, nmat), dim3(128), 0, s, descs,
                           act.as<int>(), rnd, hpart.as<double2>(), npair_max, ntile_max, cs);
      hipLaunchKernelGGL(jac_inner_kernel<JB>, dim3(npair_max, nmat), dim3(JB * JB), 0, s, descs, act.as<int>(), rnd,
                         tol, hpart.as<double2>(), jbuf.as<double2>(), rotf.as<int>(), npair_max, ntile_max, cs,
                         sweep * rounds + rnd);
      if (JB == 16)
        hipLaunchKernelGGL(jac_apply_mfma_kernel, dim3(2 * atile_max, npair_max, nmat), dim3(64), 0, s, descs,
                           act.as<int>(), rnd, jbuf.as<double2>(), rotf.as<int>(), npair_max);
      else
        hipLaunchKernelGGL(jac_apply_mfma32_kernel, dim3(2 * cdiv(nmax, 16), npair_max, nmat), dim3(64), 0, s,
                           descs, act.as<int>(), rnd, jbuf.as<double2>(), rotf.as<int>(), npair_max);
    }
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipEventRecord(e1, s));
    HIP_CHECK(hipMemcpyAsync(flags.data(), h[0].flag, nmat * sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipMemcpyAsync(checked.data(), cs.nchk, nmat * sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    float ms = 0.f;
    HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
    st.ms += ms;
    st.launches += 3 * rounds;
    // algorithmic work: every checked task (a pair not known converged) reads
    // its columns of G and forms the Hermitian Gram matrix; a task that
    // rotated writes them back and reads and writes its columns of V, applying
    // the c x c rotation product to both
    bool any = false;
    int nact = 0;
    long nrot = 0, nchecked = 0;
    for (int i = 0; i < nmat; ++i) {
      if (!active[i]) continue;
      nchecked += checked[i];
      const double n = h[i].n, c = width[i], col = n * sizeof(double2);
      st.bytes += (double)checked[i] * c * col + (double)flags[i] * 3.0 * c * col;
      st.flops += (double)checked[i] * 4.0 * c * (c + 1.0) * n + (double)flags[i] * 16.0 * c * c * n;
      if (flags[i] != 0) { any = true; ++nact; nrot += flags[i]; }
      else active[i] = 0;
    }
    if (dbg)
      fprintf(stderr, "[jacobi] nmat %d n %d sweep %d active %d rotating tasks %ld checked %ld\n", nmat, nmax,
              sweep, nact, nrot, nchecked);
    progress("Jacobi sweep %d (%d matrices, up to %d columns): %d still rotating, %.0f ms", sweep + 1, nmat, nmax,
             nact, ms);
    if (!any) break;
  }
  // matrices that still rotated in the last sweep allowed did not converge
  if (sweep == max_sweeps)
    for (int i = 0; i < nmat; ++i) st.unconverged += active[i] ? 1 : 0;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

}  // namespace

JacStats jac_run(const MatDesc *descs, const std::vector<MatDesc> &h, int init_mode, double rel_cutoff,
                 hipStream_t s) {
  (void)rel_cutoff;
  int nmax = 0;
  for (const auto &d : h) nmax = std::max(nmax, d.n);
  // 32-column blocks halve the passes over G and V per sweep (one per block
  // round) at the price of an inner problem of twice as many rounds per
  // task; that pays only once the passes over G and V dominate (measured:
  // slower at 600 and 800 columns, faster at several thousand)
  int wide = kJacWideMinCols;
  if (const char *e = getenv("MFS_JACOBI_WIDE_MIN_COLS")) wide = atoi(e);
  if (nmax >= wide) return jac_run_t<32>(descs, h, init_mode, s);
  return jac_run_t<16>(descs, h, init_mode, s);
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
