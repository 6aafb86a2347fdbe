// Direct phased near-neighbour Helmholtz sums (eqs. (A) and (Phinear)): the
// A_else action on the surface nodes, the C block on the wall nodes, and
// field evaluation at arbitrary points.
//
//   out[r][t] = sum_img w[g][img][r] sum_s K(x_t - a e_x - b e_y, y_s) sigma[r][s]
//
// with K = G (value) or the derivative of G along the target's direction.
// Targets are grouped (a group shares one image list, one kind and per-rhs
// weights) and every 64-target tile belongs to one group.  A workgroup takes
// one tile (lane = target) and one slice of the sources; its four waves
// split the slice, staged through LDS in chunks with the strengths of all
// right-hand sides, so the geometry part of each pair (one rsqrt, one
// sincos) is shared by every right-hand side.  Slices are summed by a second
// kernel.  FP64 VALU bound; the only HBM traffic is the strengths and the
// output.
#include <cstdlib>
#include <algorithm>

#include "internal.hpp"

namespace mfs {
namespace {

constexpr int SC = 128;     // sources per LDS chunk (32 per wave)
constexpr int MAXR = 16;    // right-hand sides per launch
constexpr int DU = 16;      // stored values in flight per wave in the dense sum

// Targets of a group whose values a paired stored field keeps (whole tiles):
// the first mt for the surface shift (when mt fills whole tiles), all for the
// first group of a cross pair, none for the group its partner serves, the
// first half for a self-paired group; -1 if the group cannot be paired.
__host__ __device__ inline int dense_kept(const NsumGroup &g) {
  switch (g.pkind) {
    case 1: return g.mt % 64 == 0 ? g.mt : -1;
    case 2: return (g.nt + 63) / 64 * 64;
    case 3: return 0;
    case 4: return (g.nt / 2 + 63) / 64 * 64;
    default: return -1;
  }
}
// targets (from the first) whose sums and mirror sums a paired workgroup forms
__host__ __device__ inline int pair_primaries(const NsumGroup &g) {
  return g.pkind == 1 ? g.mt : g.pkind == 2 ? g.nt : g.pkind == 4 ? g.nt / 2 : 0;
}
// the target paired with group-local target q of a paired group, as an index
// into the whole plan
__device__ inline int pair_target(const NsumGroup *groups, const NsumGroup &g, int q) {
  if (g.pkind == 1) return g.t0 + q + g.mt;
  if (g.pkind == 4) return g.t0 + g.nt - 1 - q;
  const int a = q / g.m1, b = q % g.m1;   // pkind 2: node (a, b) -> (m1-1-a, b) of the partner
  return groups[g.pg].t0 + (g.m1 - 1 - a) * g.m1 + b;
}

// G(x - y) = e^{ikR} / (4 pi R) for (dx, dy, dz) = x - y, or its derivative
// along the target direction (tx, ty, tz) when deriv is set
__device__ inline double2 near_kernel(double ddx, double ddy, double ddz, double tx, double ty, double tz,
                                      double k, int deriv) {
  const double inv4pi = 0.25 / kPi;
  const double R2 = fma(ddx, ddx, fma(ddy, ddy, ddz * ddz));
  const double invR = rsqrt(R2);
  const double R = R2 * invR;
  double sn, cs;
  sincos(k * R, &sn, &cs);
  if (deriv) {
    const double dn = fma(tx, ddx, fma(ty, ddy, tz * ddz));
    const double tt = dn * invR * invR * inv4pi;
    return cz(tt * fma(-cs, invR, -sn * k), tt * fma(cs, k, -sn * invR));
  }
  const double tt = invR * inv4pi;
  return cz(cs * tt, sn * tt);
}

// With MIR (every group mirror-paired, NsumGroup::pkind) a workgroup takes
// the primary targets of its tile (the first mt of the surface, all of the
// first wall of a cross pair, the first half of a self-paired wall, none of a
// wall its partner serves) and forms the sums of each and of its mirror from
// the same kernel values, against the strengths of the sources s and s + ms
// (mod S) and the weights of the mirror images (the partner group's, times
// psign): half the kernel evaluations.  A lane past the primaries writes
// nothing (its sum arrives as a mirror) unless it is a padding target, which
// gets zero; tiles wholly past them only write their padding zeros.
template <int NR, bool MIR>
__global__ __launch_bounds__(256) void nsum_kernel(const double *__restrict__ tgt, int ntp,
                                                   const NsumGroup *__restrict__ groups,
                                                   const int *__restrict__ tile_group, int nrhs,
                                                   double k, double ex, double ey,
                                                   const double *__restrict__ src, int S,
                                                   const double2 *__restrict__ sigma,
                                                   const double2 *__restrict__ wts, int nsplit,
                                                   double2 *__restrict__ out) {
  extern __shared__ double shm[];
  double *sx = shm, *sy = shm + SC, *szs = shm + 2 * SC;
  double2 *ssig = reinterpret_cast<double2 *>(shm + 3 * SC);   // [NR][SC], then [NR][SC] mirror
  double2 *ssig2 = ssig + NR * SC;
  const int tile = blockIdx.x;
  const int split = blockIdx.y;
  const int gi = tile_group[tile];
  const NsumGroup g = groups[gi];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int t = tile * 64 + lane;
  const int tl = tile * 64 - g.t0;   // first target of the tile within its group
  const int nprim = MIR ? pair_primaries(g) : 0;
  if (MIR && tl >= nprim) {
    for (int idx = threadIdx.x; idx < NR * 64; idx += 256) {
      const int r = idx / 64, l = idx % 64;
      if (r < nrhs && tl + l >= g.nt) out[((size_t)split * nrhs + r) * ntp + tile * 64 + l] = cz(0.0, 0.0);
    }
    return;
  }
  const double xt = tgt[t], yt = tgt[ntp + t], zt = tgt[2 * ntp + t];
  const double dxt = tgt[3 * ntp + t], dyt = tgt[4 * ntp + t], dzt = tgt[5 * ntp + t];
  const int per = (S + nsplit - 1) / nsplit;
  const int s_begin = split * per;
  const int s_end = min(S, s_begin + per);

  double2 tot[NR], tot2[MIR ? NR : 1];
#pragma unroll
  for (int r = 0; r < NR; ++r) tot[r] = cz(0.0, 0.0);
  if (MIR)
#pragma unroll
    for (int r = 0; r < NR; ++r) tot2[r] = cz(0.0, 0.0);

  for (int im = 0; im < g.nimg; ++im) {
    const double xs = xt - groups[gi].ia[im] * ex, ys = yt - groups[gi].ib[im] * ey;
    double2 acc[NR], acc2[MIR ? NR : 1];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = cz(0.0, 0.0);
    if (MIR)
#pragma unroll
      for (int r = 0; r < NR; ++r) acc2[r] = cz(0.0, 0.0);
    for (int c0 = s_begin; c0 < s_end; c0 += SC) {
      const int nc = min(SC, s_end - c0);
      __syncthreads();
      for (int idx = threadIdx.x; idx < SC; idx += 256) {
        const int s = c0 + idx;
        const bool ok = idx < nc;
        sx[idx] = ok ? src[s] : 0.0;
        sy[idx] = ok ? src[S + s] : 0.0;
        szs[idx] = ok ? src[2 * S + s] : 1e3;   // far dummy source, zero strength
      }
      for (int idx = threadIdx.x; idx < NR * SC; idx += 256) {
        const int r = idx / SC, ss = idx % SC;
        const bool ok = r < nrhs && ss < nc;
        ssig[idx] = ok ? sigma[(size_t)r * S + c0 + ss] : cz(0.0, 0.0);
        if (MIR) {
          const int sm = c0 + ss + g.ms >= S ? c0 + ss + g.ms - S : c0 + ss + g.ms;
          ssig2[idx] = ok ? sigma[(size_t)r * S + sm] : cz(0.0, 0.0);
        }
      }
      __syncthreads();
      const int sbeg = wv * (SC / 4);
      for (int ss = sbeg; ss < sbeg + SC / 4; ++ss) {
        const double2 K = near_kernel(xs - sx[ss], ys - sy[ss], zt - szs[ss], dxt, dyt, dzt, k, g.deriv);
#pragma unroll
        for (int r = 0; r < NR; ++r) cfma(acc[r], K, ssig[r * SC + ss]);
        if (MIR)
#pragma unroll
          for (int r = 0; r < NR; ++r) cfma(acc2[r], K, ssig2[r * SC + ss]);
      }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r)
      if (r < nrhs) cfma(tot[r], wts[((size_t)gi * 9 + im) * nrhs + r], acc[r]);
    if (MIR) {
      const int jm = groups[gi].mir[im];
#pragma unroll
      for (int r = 0; r < NR; ++r)
        if (r < nrhs) cfma(tot2[r], cscale(wts[((size_t)g.pg * 9 + jm) * nrhs + r], (double)g.psign), acc2[r]);
    }
  }
  // reduce the four waves (the target sums, then for MIR the mirror sums)
  double2 *red = reinterpret_cast<double2 *>(shm);    // [4][NR][64]
  for (int half = 0; half < (MIR ? 2 : 1); ++half) {
    __syncthreads();
#pragma unroll
    for (int r = 0; r < NR; ++r) red[(wv * NR + r) * 64 + lane] = (MIR && half) ? tot2[r] : tot[r];
    __syncthreads();
    for (int idx = threadIdx.x; idx < NR * 64; idx += 256) {
      const int r = idx / 64, l = idx % 64;
      if (r >= nrhs) continue;
      double2 v = red[(0 * NR + r) * 64 + l];
      for (int w2 = 1; w2 < 4; ++w2) v = cadd(v, red[(w2 * NR + r) * 64 + l]);
      double2 *row = out + ((size_t)split * nrhs + r) * ntp;
      const int q = tl + l;   // group-local target
      if (!MIR) row[tile * 64 + l] = v;
      else if (half) {
        if (q < nprim) row[pair_target(groups, g, q)] = v;
      } else if (q < nprim) {
        row[tile * 64 + l] = v;
      } else if (q >= g.nt) {
        row[tile * 64 + l] = cz(0.0, 0.0);
      }
    }
  }
}

// Dense near field: the values K(x_t - a e_x - b e_y, y_s) of every group,
// image and source are written once, per 64-target tile, image-major then
// source-major with the tile's targets contiguous:
//   dense[koff[g] + ((tile_g * nimg_g + img) * S + s) * 64 + lane],
// so that every wave of the sum streams one contiguous range; a mirror-paired
// group (NsumGroup::mt) stores its first mt targets only.
// The sums then stream them instead of evaluating them (they depend on the
// geometry, the lattice and k only, not on the incident wave or the iterate).
__global__ __launch_bounds__(256) void nsum_fill_kernel(const double *__restrict__ tgt, int ntp,
                                                        const NsumGroup *__restrict__ groups,
                                                        const int *__restrict__ tile_group,
                                                        const size_t *__restrict__ koff, double k, double ex,
                                                        double ey, const double *__restrict__ src, int S,
                                                        int nsplit, int paired, double2 *__restrict__ dense) {
  __shared__ double sx[SC], sy[SC], szs[SC];
  const int tile = blockIdx.x, split = blockIdx.y;
  const int gi = tile_group[tile];
  const NsumGroup &g = groups[gi];
  if (paired && tile * 64 - g.t0 >= dense_kept(g)) return;   // values served by the mirror: not stored
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int t = tile * 64 + lane;
  const double xt = tgt[t], yt = tgt[ntp + t], zt = tgt[2 * ntp + t];
  const double dxt = tgt[3 * ntp + t], dyt = tgt[4 * ntp + t], dzt = tgt[5 * ntp + t];
  const int per = (S + nsplit - 1) / nsplit;
  const int s_begin = split * per, s_end = min(S, s_begin + per);
  const int nimg = g.nimg, deriv = g.deriv;
  double2 *base = dense + koff[gi] + (size_t)((t - g.t0) >> 6) * nimg * S * 64 + lane;
  for (int c0 = s_begin; c0 < s_end; c0 += SC) {
    const int nc = min(SC, s_end - c0);
    __syncthreads();
    for (int idx = threadIdx.x; idx < SC; idx += 256) {
      const int sidx = c0 + idx;
      const bool ok = idx < nc;
      sx[idx] = ok ? src[sidx] : 0.0;
      sy[idx] = ok ? src[S + sidx] : 0.0;
      szs[idx] = ok ? src[2 * S + sidx] : 0.0;
    }
    __syncthreads();
    for (int im = 0; im < nimg; ++im) {
      const double xs = xt - groups[gi].ia[im] * ex, ys = yt - groups[gi].ib[im] * ey;
      for (int ss = wv; ss < nc; ss += 4) {
        const double2 K = near_kernel(xs - sx[ss], ys - sy[ss], zt - szs[ss], dxt, dyt, dzt, k, deriv);
        base[((size_t)im * S + c0 + ss) * 64] = K;
      }
    }
  }
}

// sigT[s][r] = sigma[r][s] for r < nrhs, zero up to NR: the strengths of one
// source side by side, so that a wave reads them with one uniform address.
__global__ void sig_transpose_kernel(int nrhs, int NRp, int S, const double2 *__restrict__ sigma,
                                     double2 *__restrict__ sigT) {
  const long n = (long)S * NRp;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const int r = (int)(i % NRp);
    const long sidx = i / NRp;
    sigT[i] = r < nrhs ? sigma[(size_t)r * S + sidx] : cz(0.0, 0.0);
  }
}

// Stored near field: every wave of a workgroup streams its own contiguous
// quarter of the split's sources for the workgroup's 64 targets (one lane
// per target, 16 B per lane and source, coalesced), eight non-temporal loads
// in flight, and takes the NR strengths of each source from sigT through a
// wave-uniform address (scalar loads: no LDS staging, no barrier in the
// loop).  The four waves' partial sums meet in LDS at the end.
template <int NR>
__global__ __launch_bounds__(256) void nsum_dense_kernel(int ntp, const NsumGroup *__restrict__ groups,
                                                         const int *__restrict__ tile_group,
                                                         const size_t *__restrict__ koff,
                                                         const double2 *__restrict__ dense, int nrhs, int S,
                                                         const double2 *__restrict__ sigT,
                                                         const double2 *__restrict__ wts, int nsplit,
                                                         double2 *__restrict__ out) {
  extern __shared__ double shm[];
  const int tile = blockIdx.x, split = blockIdx.y;
  const int gi = tile_group[tile];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int t = tile * 64 + lane;
  const int t0 = groups[gi].t0, nimg = groups[gi].nimg;
  const int per = (S + nsplit - 1) / nsplit;
  const int s_begin = split * per, s_end = min(S, s_begin + per);
  const int qw = (s_end - s_begin + 3) / 4;
  const int w_begin = min(s_end, s_begin + wv * qw), w_end = min(s_end, w_begin + qw);
  const double2 *base = dense + koff[gi] + (size_t)((t - t0) >> 6) * nimg * S * 64 + lane;
  double2 tot[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) tot[r] = cz(0.0, 0.0);
  for (int im = 0; im < nimg; ++im) {
    double2 acc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = cz(0.0, 0.0);
    const double2 *kim = base + (size_t)im * S * 64;
    for (int c0 = w_begin; c0 < w_end; c0 += DU) {
      double2 kv[DU];
#pragma unroll
      for (int e = 0; e < DU; ++e) {
        // streamed once per launch: non-temporal loads keep them out of the caches
        const bool ok = c0 + e < w_end;
        const double2 *pk = kim + (size_t)(ok ? c0 + e : c0) * 64;
        double2 v;
        v.x = __builtin_nontemporal_load(&pk->x);
        v.y = __builtin_nontemporal_load(&pk->y);
        const long long m = ok ? -1LL : 0LL;
        kv[e] = cz(__longlong_as_double(__double_as_longlong(v.x) & m),
                   __longlong_as_double(__double_as_longlong(v.y) & m));
      }
#pragma unroll
      for (int e = 0; e < DU; ++e) {
        // a source past the wave's range (kv = 0) reads the last valid row
        const double2 *sv = sigT + (size_t)min(c0 + e, w_end - 1) * NR;
#pragma unroll
        for (int r = 0; r < NR; ++r) cfma(acc[r], kv[e], sv[r]);
      }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r)
      if (r < nrhs) cfma(tot[r], wts[((size_t)gi * 9 + im) * nrhs + r], acc[r]);
  }
  double2 *red = reinterpret_cast<double2 *>(shm);    // [4][NR][64]
#pragma unroll
  for (int r = 0; r < NR; ++r) red[(wv * NR + r) * 64 + lane] = tot[r];
  __syncthreads();
  for (int idx = threadIdx.x; idx < NR * 64; idx += 256) {
    const int r = idx / 64, l = idx % 64;
    if (r >= nrhs) continue;
    double2 v = red[(0 * NR + r) * 64 + l];
    for (int w2 = 1; w2 < 4; ++w2) v = cadd(v, red[(w2 * NR + r) * 64 + l]);
    out[((size_t)split * nrhs + r) * ntp + tile * 64 + l] = v;
  }
}

// The mirror form on the FP64 matrix cores, for NR = 8 or 16 right-hand
// sides: per image, out[t][c] += sum_s K[t][s] B[s][c] as 16 x 16 x 4
// products with the 64 targets of the tile as four row blocks (A = the
// stored values, 16 targets by 4 sources, read as before) and 2 NR columns
// in blocks of 16: B[s][c] = w_c sigma_c(s) for the NR sums (weights of the
// image) and w'_(c-NR) sigma_(c-NR)(s + ms) for the NR mirror sums (weights
// of the mirror image), each lane forming its own element of B per step.
// The weights sit in B, so the accumulators are the totals.  The pairing is
// that of the group (NsumGroup::pkind): the surface shift t -> t + mt, a wall
// node and its mirror on the opposite wall (the partner group's weights, and
// a sign for the normal derivatives the half-turn reverses), or a node and
// its mirror on the same wall.  The grid runs over the stored tiles only
// (tiles[], those with the most images first, so that a launch ends on short
// workgroups).
// One stored field of a launch of the mirror form: its plan's device arrays,
// weights, source slices and output (see nsum_dense_mirror_mfma_kernel).
struct DenseView {
  int ntp, ntiles, nsplit;
  const NsumGroup *groups;
  const int *tile_group;
  const size_t *koff;
  const int *tiles;
  const double2 *dense, *wts;
  double2 *out;
};

template <int NR>
__global__ __launch_bounds__(256, NR == 8 ? 4 : 2) void nsum_dense_mirror_mfma_kernel(DenseView va, DenseView vb,
                                                                     int nrhs, int S,
                                                                     const double2 *__restrict__ sigT) {
  static_assert(NR == 8 || NR == 16, "two NR columns in blocks of 16");
  constexpr int RB = 4, CB = 2 * NR / 16, KU = 2;   // KU steps of 4 sources per batch of loads
  extern __shared__ double shm[];
  // the first va.ntiles workgroups of x serve the first field, the rest the
  // second (the surface and the wall sums of one iteration in one launch)
  const bool second = (int)blockIdx.x >= va.ntiles;
  const DenseView &V = second ? vb : va;
  if ((int)blockIdx.y >= V.nsplit) return;
  const int ntp = V.ntp, nsplit = V.nsplit;
  const NsumGroup *__restrict__ groups = V.groups;
  const size_t *__restrict__ koff = V.koff;
  const double2 *__restrict__ dense = V.dense;
  const double2 *__restrict__ wts = V.wts;
  double2 *__restrict__ out = V.out;
  const int tile = V.tiles[second ? blockIdx.x - va.ntiles : blockIdx.x], split = blockIdx.y;   // stored tiles only
  const int *__restrict__ tile_group = V.tile_group;
  const int gi = tile_group[tile];
  const int l = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const NsumGroup &G = groups[gi];
  const int t0 = G.t0, nimg = G.nimg, ms = G.ms;
  const int tl = tile * 64 - t0;
  if (tl >= dense_kept(G)) return;   // values served by the mirror (or by the partner group)
  const int nprim = pair_primaries(G);
  const double psign = G.psign;
  const int per = (S + nsplit - 1) / nsplit;
  const int s_begin = split * per, s_end = min(S, s_begin + per);
  const int qw = (s_end - s_begin + 3) / 4;
  const int w_begin = min(s_end, s_begin + wv * qw), w_end = min(s_end, w_begin + qw);
  const double2 *base = dense + koff[gi] + (size_t)(tl >> 6) * nimg * S * 64;
  const int i = l & 15, k = l >> 4;          // A: target 16 rb + i, source 4 step + k
  const int j = l & 15;                      // B: column 16 cb + j, source 4 step + k
  dx4 tr[RB][CB], ti[RB][CB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      tr[rb][cb] = dx4{0, 0, 0, 0};
      ti[rb][cb] = tr[rb][cb];
    }
  for (int im = 0; im < nimg; ++im) {
    double2 wj[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      const int c = 16 * cb + j, jr = c < NR ? c : c - NR;
      // the mirror columns take the partner group's weight of the mirror image
      const double2 wv2 = jr < nrhs ? (c < NR ? wts[((size_t)gi * 9 + im) * nrhs + jr]
                                              : wts[((size_t)G.pg * 9 + G.mir[im]) * nrhs + jr])
                                    : cz(0.0, 0.0);
      wj[cb] = c < NR ? wv2 : cscale(wv2, psign);
    }
    const double2 *kim = base + (size_t)im * S * 64;
    for (int c0 = w_begin; c0 < w_end; c0 += 4 * KU) {   // wave-uniform trip count
      double2 a[KU][RB], bb[KU][CB];
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        const int sidx = c0 + 4 * u + k;
        const bool ok = sidx < w_end;
        const int sc = ok ? sidx : w_begin;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          const double2 *pk = kim + (size_t)sc * 64 + 16 * rb + i;
          double2 v;
          v.x = __builtin_nontemporal_load(&pk->x);
          v.y = __builtin_nontemporal_load(&pk->y);
          const long long m = ok ? -1LL : 0LL;
          a[u][rb] = cz(__longlong_as_double(__double_as_longlong(v.x) & m),
                        __longlong_as_double(__double_as_longlong(v.y) & m));
        }
        const int smir = sc + ms >= S ? sc + ms - S : sc + ms;
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
          const int c = 16 * cb + j, jr = c < NR ? c : c - NR;
          bb[u][cb] = cmul(wj[cb], sigT[(size_t)(c < NR ? sc : smir) * NR + jr]);   // zero past nrhs via wj
        }
      }
#pragma unroll
      for (int u = 0; u < KU; ++u)
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
          for (int cb = 0; cb < CB; ++cb) {
            tr[rb][cb] = mfma_f64(a[u][rb].x, bb[u][cb].x, tr[rb][cb]);
            tr[rb][cb] = mfma_f64(-a[u][rb].y, bb[u][cb].y, tr[rb][cb]);
            ti[rb][cb] = mfma_f64(a[u][rb].x, bb[u][cb].y, ti[rb][cb]);
            ti[rb][cb] = mfma_f64(a[u][rb].y, bb[u][cb].x, ti[rb][cb]);
          }
    }
  }
  // element v of lane j + 16 g: target 16 rb + g + 4 v, column 16 cb + j; the
  // four waves' sums meet in LDS [4][NR][64 targets], the NR sums first, then
  // the NR mirror sums
  double2 *red = reinterpret_cast<double2 *>(shm);
  const int g = l >> 4;
  for (int half = 0; half < 2; ++half) {
    if (half) __syncthreads();
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      const int c = 16 * cb + j;
      if ((c >= NR) == (half == 1)) {
        const int jr = c < NR ? c : c - NR;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            red[(wv * NR + jr) * 64 + 16 * rb + g + 4 * v] = cz(tr[rb][cb][v], ti[rb][cb][v]);
      }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < NR * 64; idx += 256) {
      const int r = idx / 64, tt = idx % 64;
      if (r >= nrhs) continue;
      double2 v = red[(0 * NR + r) * 64 + tt];
      for (int w2 = 1; w2 < 4; ++w2) v = cadd(v, red[(w2 * NR + r) * 64 + tt]);
      const int q = tl + tt;   // group-local target
      double2 *row = out + ((size_t)split * nrhs + r) * ntp;
      if (!half) {
        // a target past the primaries of a self pair or a shift is a mirror, written by its partner
        if (q < nprim || G.pkind == 2) row[tile * 64 + tt] = v;
      } else if (q < nprim) {
        row[pair_target(groups, G, q)] = v;
      }
    }
  }
}

__global__ void nsum_reduce(int nsplit, int nrhs, int ntp, const double2 *__restrict__ part,
                            double2 *__restrict__ out) {
  const long n = (long)nrhs * ntp;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    double2 v = part[i];
    for (int s = 1; s < nsplit; ++s) v = cadd(v, part[(size_t)s * n + i]);
    out[i] = v;
  }
}

// Wall rows of C from the 12 padded target groups (R L Rx Lx F B Fy By T Tz D Dz):
// [R+L, Rx+Lx, F+B, Fy+By, T, Tz, D, Dz], each M1^2 rows.
__global__ void combine_walls_kernel(int nw, int M1sq, const double2 *__restrict__ in,
                                     double2 *__restrict__ out) {
  const int pad = (M1sq + 63) / 64 * 64;
  const int ntp = 12 * pad;
  const long n = (long)nw * 8 * M1sq;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const int w = (int)(i / (8 * M1sq));
    const int row = (int)(i % (8 * M1sq));
    const int blk = row / M1sq, t = row % M1sq;
    const double2 *src = in + (size_t)w * ntp;
    double2 v;
    if (blk < 4) v = cadd(src[(2 * blk) * pad + t], src[(2 * blk + 1) * pad + t]);
    else v = src[(blk + 4) * pad + t];
    out[i] = v;
  }
}

// every group mirror-paired (the on-the-fly sum then runs its MIR form) /
// every group mirror-paired on whole tiles (the stored field keeps half the
// tiles and its sum runs the MIR form); a plan mixing paired and unpaired
// groups is refused
bool plan_mirrored(const NsumPlan &plan, bool dense) {
  bool any = false, all = true;
  for (const auto &g : plan.groups) {
    const bool p = dense ? dense_kept(g) >= 0 : (g.pkind == 1 ? g.mt > 0 : g.pkind >= 2);
    any = any || p;
    all = all && p;
  }
  MFS_REQUIRE(any == all, "neighbour sum: mirror pairing must hold for every group or none");
  return all;
}

DenseView dense_view(const NsumPlan &plan, const double2 *w, int nsplit, double2 *dst) {
  DenseView v{};
  v.ntp = plan.ntarget_pad;
  v.ntiles = plan.ndense_tiles;
  v.nsplit = nsplit;
  v.groups = plan.grp.as<NsumGroup>();
  v.tile_group = plan.tile_group.as<int>();
  v.koff = plan.koff.as<size_t>();
  v.tiles = plan.dense_tiles.as<int>();
  v.dense = plan.dense.as<double2>();
  v.wts = w;
  v.out = dst;
  return v;
}

template <int NR>
void launch_nsum_dense_t(const NsumPlan &plan, int nrhs, int S, const double2 *sigma, const double2 *w,
                         int nsplit, double2 *dst, hipStream_t s) {
  double2 *sigT = plan.sigT.as<double2>();
  const long n = (long)S * NR;
  hipLaunchKernelGGL(sig_transpose_kernel, dim3((unsigned)std::min<long>(1024, (n + 255) / 256)), dim3(256), 0, s,
                     nrhs, NR, S, sigma, sigT);
  const size_t sh = (size_t)4 * NR * 64 * sizeof(double2);
  if (plan_mirrored(plan, true)) {
    MFS_REQUIRE(NR == 8 || NR == 16, "neighbour sum: the mirror form runs with 8 or 16 right-hand sides");
    MFS_REQUIRE(plan.ndense_tiles > 0, "neighbour sum: stored tiles of the paired field missing");
    const DenseView va = dense_view(plan, w, nsplit, dst), vb{};
    hipLaunchKernelGGL((nsum_dense_mirror_mfma_kernel<NR == 16 ? 16 : 8>), dim3(plan.ndense_tiles, nsplit),
                       dim3(256), (size_t)4 * NR * 64 * sizeof(double2), s, va, vb, nrhs, S, sigT);
  }
  else
    hipLaunchKernelGGL(nsum_dense_kernel<NR>, dim3(plan.ntarget_pad / 64, nsplit), dim3(256), sh, s,
                       plan.ntarget_pad, plan.grp.as<NsumGroup>(), plan.tile_group.as<int>(),
                       plan.koff.as<size_t>(), plan.dense.as<double2>(), nrhs, S, sigT, w, nsplit, dst);
  HIP_CHECK(hipGetLastError());
}

template <int NR>
void launch_nsum_t(const NsumPlan &plan, int nrhs, double k, double ex, double ey,
                   const double *src, int S, const double2 *sigma, const double2 *w,
                   int nsplit, double2 *dst, hipStream_t s) {
  const bool mir = plan_mirrored(plan, false);
  const size_t sh = std::max((size_t)(3 * SC) * sizeof(double) + (size_t)(mir ? 2 : 1) * NR * SC * sizeof(double2),
                             (size_t)4 * NR * 64 * sizeof(double2));
  if (mir)
    hipLaunchKernelGGL((nsum_kernel<NR, true>), dim3(plan.ntarget_pad / 64, nsplit), dim3(256), sh, s,
                       plan.tgt.as<double>(), plan.ntarget_pad, plan.grp.as<NsumGroup>(),
                       plan.tile_group.as<int>(), nrhs, k, ex, ey, src, S, sigma, w, nsplit, dst);
  else
    hipLaunchKernelGGL((nsum_kernel<NR, false>), dim3(plan.ntarget_pad / 64, nsplit), dim3(256), sh, s,
                       plan.tgt.as<double>(), plan.ntarget_pad, plan.grp.as<NsumGroup>(),
                       plan.tile_group.as<int>(), nrhs, k, ex, ey, src, S, sigma, w, nsplit, dst);
  HIP_CHECK(hipGetLastError());
}

}  // namespace

// Source slices per tile: about five rounds of resident workgroups (256 CUs x
// 3 workgroups of 256 threads for the stored-field sum), rounded down so that
// the last round is (nearly) full: 240 surface tiles -> 16 slices, 3840
// workgroups.
int nsum_splits(const NsumPlan &plan, int S) {
  // tiles with work in the stored-field sum (a mirror pair's second half has none)
  int tiles = 0;
  for (const auto &g : plan.groups)
    tiles += g.pkind == 1 && g.mt > 0 ? cdiv(g.mt, 64)
             : dense_kept(g) >= 0     ? dense_kept(g) / 64
                                      : round_up(std::max(g.nt, 1), 64) / 64;
  tiles = std::max(tiles, 1);
  // eight rounds of workgroups at three 256-thread workgroups per CU on 256 CUs;
  // MFS_NSUM_WORKGROUPS (read once) sets another target
  static const int target = []() -> int {
    const char *e = std::getenv("MFS_NSUM_WORKGROUPS");
    const int t = e ? std::atoi(e) : 0;
    return t > 0 ? t : 6144;
  }();
  int ns = std::max(1, target / tiles);
  ns = std::min(ns, std::max(1, S / 256));
  return ns;
}

void launch_nsum(const NsumPlan &plan, int nrhs, double k, double ex, double ey, const double *src,
                 int S, const double2 *sigma, const double2 *w, double2 *out, double2 *partial,
                 hipStream_t s) {
  MFS_REQUIRE(nrhs >= 1 && nrhs <= MAXR, "neighbour sum: 1 <= nrhs <= 16");
  const int nsplit = nsum_splits(plan, S);
  double2 *dst = (nsplit == 1) ? out : partial;
  if (plan.dense.p && plan.dense_src == src && plan.dense_S == S && plan.dense_k == k) {
    if (plan_mirrored(plan, true)) {
      // the matrix-core mirror form: 8 columns for up to 8 right-hand sides, else 16
      if (nrhs <= 8) launch_nsum_dense_t<8>(plan, nrhs, S, sigma, w, nsplit, dst, s);
      else launch_nsum_dense_t<16>(plan, nrhs, S, sigma, w, nsplit, dst, s);
    } else if (nrhs <= 1) launch_nsum_dense_t<1>(plan, nrhs, S, sigma, w, nsplit, dst, s);
    else if (nrhs <= 2) launch_nsum_dense_t<2>(plan, nrhs, S, sigma, w, nsplit, dst, s);
    else if (nrhs <= 4) launch_nsum_dense_t<4>(plan, nrhs, S, sigma, w, nsplit, dst, s);
    else if (nrhs <= 8) launch_nsum_dense_t<8>(plan, nrhs, S, sigma, w, nsplit, dst, s);
    else launch_nsum_dense_t<16>(plan, nrhs, S, sigma, w, nsplit, dst, s);
  } else if (nrhs <= 1) launch_nsum_t<1>(plan, nrhs, k, ex, ey, src, S, sigma, w, nsplit, dst, s);
  else if (nrhs <= 2) launch_nsum_t<2>(plan, nrhs, k, ex, ey, src, S, sigma, w, nsplit, dst, s);
  else if (nrhs <= 4) launch_nsum_t<4>(plan, nrhs, k, ex, ey, src, S, sigma, w, nsplit, dst, s);
  else if (nrhs <= 8) launch_nsum_t<8>(plan, nrhs, k, ex, ey, src, S, sigma, w, nsplit, dst, s);
  else launch_nsum_t<16>(plan, nrhs, k, ex, ey, src, S, sigma, w, nsplit, dst, s);
  if (nsplit > 1) {
    const long n = (long)nrhs * plan.ntarget_pad;
    hipLaunchKernelGGL(nsum_reduce, dim3((unsigned)std::min<long>(2048, (n + 255) / 256)), dim3(256),
                       0, s, nsplit, nrhs, plan.ntarget_pad, partial, out);
    HIP_CHECK(hipGetLastError());
  }
}

bool nsum_pair_fusable(const NsumPlan &a, const NsumPlan &b, double k, const double *src, int S, int nrhs) {
  auto stored = [&](const NsumPlan &p) {
    return p.dense.p && p.dense_src == src && p.dense_S == S && p.dense_k == k && plan_mirrored(p, true) &&
           p.ndense_tiles > 0;
  };
  return nrhs >= 1 && nrhs <= MAXR && stored(a) && stored(b);
}

void launch_nsum_pair(const NsumPlan &pa, const double2 *wa, double2 *outa, double2 *parta, const NsumPlan &pb,
                      const double2 *wb, double2 *outb, double2 *partb, int nrhs, int S, const double2 *sigma,
                      hipStream_t s) {
  const int na = nsum_splits(pa, S), nb = nsum_splits(pb, S);
  double2 *da = na == 1 ? outa : parta, *db = nb == 1 ? outb : partb;
  const int NR = nrhs <= 8 ? 8 : 16;
  double2 *sigT = pa.sigT.as<double2>();
  const long n = (long)S * NR;
  hipLaunchKernelGGL(sig_transpose_kernel, dim3((unsigned)std::min<long>(1024, (n + 255) / 256)), dim3(256), 0, s,
                     nrhs, NR, S, sigma, sigT);
  const DenseView va = dense_view(pa, wa, na, da), vb = dense_view(pb, wb, nb, db);
  const dim3 grid(pa.ndense_tiles + pb.ndense_tiles, std::max(na, nb));
  const size_t sh = (size_t)4 * NR * 64 * sizeof(double2);
  if (NR == 8)
    hipLaunchKernelGGL(nsum_dense_mirror_mfma_kernel<8>, grid, dim3(256), sh, s, va, vb, nrhs, S, sigT);
  else
    hipLaunchKernelGGL(nsum_dense_mirror_mfma_kernel<16>, grid, dim3(256), sh, s, va, vb, nrhs, S, sigT);
  HIP_CHECK(hipGetLastError());
  if (na > 1) {
    const long m = (long)nrhs * pa.ntarget_pad;
    hipLaunchKernelGGL(nsum_reduce, dim3((unsigned)std::min<long>(2048, (m + 255) / 256)), dim3(256), 0, s, na,
                       nrhs, pa.ntarget_pad, parta, outa);
  }
  if (nb > 1) {
    const long m = (long)nrhs * pb.ntarget_pad;
    hipLaunchKernelGGL(nsum_reduce, dim3((unsigned)std::min<long>(2048, (m + 255) / 256)), dim3(256), 0, s, nb,
                       nrhs, pb.ntarget_pad, partb, outb);
  }
  HIP_CHECK(hipGetLastError());
}

bool nsum_build_dense(NsumPlan &plan, double k, double ex, double ey, const double *src, int S,
                      size_t max_bytes, hipStream_t s) {
  const bool paired = plan_mirrored(plan, true);
  size_t off = 0;
  std::vector<size_t> koff(plan.groups.size());
  for (size_t gi = 0; gi < plan.groups.size(); ++gi) {
    const NsumGroup &g = plan.groups[gi];
    koff[gi] = off;
    off += (size_t)g.nimg * S * (paired ? dense_kept(g) : round_up(std::max(g.nt, 1), 64));
  }
  const size_t bytes = off * sizeof(double2);
  // the values the method needs, without the tile padding: every real target
  // whose values are stored (half of a self-paired wall group)
  size_t alg = 0;
  for (const NsumGroup &g : plan.groups) {
    const size_t real = !paired ? (size_t)g.nt
                        : g.pkind == 1 ? (size_t)g.mt
                        : g.pkind == 2 ? (size_t)g.nt
                        : g.pkind == 4 ? (size_t)(g.nt + 1) / 2 : 0;
    alg += (size_t)g.nimg * S * real * sizeof(double2);
  }
  if (bytes > max_bytes) return false;
  if (bytes + ((size_t)2 << 30) > device_free_bytes()) return false;   // keep 2 GiB of headroom
  plan.dense.alloc(bytes);
  plan.sigT.alloc((size_t)S * MAXR * sizeof(double2));
  plan.koff.alloc(koff.size() * sizeof(size_t));
  HIP_CHECK(hipMemcpyAsync(plan.koff.p, koff.data(), koff.size() * sizeof(size_t), hipMemcpyHostToDevice, s));
  std::vector<int> tiles;
  if (paired) {
    // the sum's workgroups run over the stored tiles only, those with the
    // most images (the longest workgroups) first
    std::vector<std::pair<int, int>> kt;   // (images, tile)
    for (const NsumGroup &g : plan.groups)
      for (int t = 0; t < dense_kept(g) / 64; ++t) kt.emplace_back(g.nimg, g.t0 / 64 + t);
    std::stable_sort(kt.begin(), kt.end(), [](const std::pair<int, int> &a, const std::pair<int, int> &b) {
      return a.first > b.first;
    });
    for (const auto &e : kt) tiles.push_back(e.second);
    MFS_REQUIRE(!tiles.empty(), "neighbour sum: a paired field with no stored tile");
    plan.dense_tiles.alloc(tiles.size() * sizeof(int));
    HIP_CHECK(hipMemcpyAsync(plan.dense_tiles.p, tiles.data(), tiles.size() * sizeof(int), hipMemcpyHostToDevice, s));
  }
  plan.ndense_tiles = (int)tiles.size();
  HIP_CHECK(hipStreamSynchronize(s));   // the host vectors above are copied before they go
  const int nsplit = nsum_splits(plan, S);
  hipLaunchKernelGGL(nsum_fill_kernel, dim3(plan.ntarget_pad / 64, nsplit), dim3(256), 0, s, plan.tgt.as<double>(),
                     plan.ntarget_pad, plan.grp.as<NsumGroup>(), plan.tile_group.as<int>(), plan.koff.as<size_t>(),
                     k, ex, ey, src, S, nsplit, paired ? 1 : 0, plan.dense.as<double2>());
  HIP_CHECK(hipGetLastError());
  plan.dense_src = src;
  plan.dense_S = S;
  plan.dense_k = k;
  plan.dense_bytes = bytes;
  plan.dense_alg_bytes = alg;
  return true;
}

void launch_combine_walls(int nw, int M1sq, const double2 *in, double2 *out, hipStream_t s) {
  const long n = (long)nw * 8 * M1sq;
  hipLaunchKernelGGL(combine_walls_kernel, dim3((unsigned)std::min<long>(1024, (n + 255) / 256)),
                     dim3(256), 0, s, nw, M1sq, in, out);
  HIP_CHECK(hipGetLastError());
}

}  // namespace mfs
