// Internal data structures and kernel launchers of libmfs (not part of the
// C ABI).  All device matrices are column-major complex double (double2).
#pragma once

#include <memory>
#include <vector>

#include "common.hpp"

namespace mfs {

// ------------------------------------------------------------ device buffer
// Device memory of the calling thread's current device.  Blocks of 1 MiB
// and more come from a per-device cache (pool.cpp): release keeps them for
// the next request of about their size, after the device has finished the
// work queued before the release (the rule hipFree keeps).
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  int dev = 0;
  size_t cached = 0;   // size of the cached block behind p (0: plain hipMalloc)
  DevBuf() = default;
  explicit DevBuf(size_t n) { alloc(n); }
  ~DevBuf() { release(); }
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  DevBuf(DevBuf &&o) noexcept : p(o.p), bytes(o.bytes), dev(o.dev), cached(o.cached) {
    o.p = nullptr; o.bytes = 0; o.cached = 0;
  }
  DevBuf &operator=(DevBuf &&o) noexcept {
    if (this != &o) {
      release();
      p = o.p; bytes = o.bytes; dev = o.dev; cached = o.cached;
      o.p = nullptr; o.bytes = 0; o.cached = 0;
    }
    return *this;
  }
  void alloc(size_t n);
  void release();
  template <class T> T *as() const { return static_cast<T *>(p); }
};
// Idle bytes held by the cache of device dev; free them all (pool_trim).
size_t pool_idle_bytes(int dev);
void pool_trim(int dev);
// bytes of live DevBufs on device dev, their peak since pool_reset_peak, idle cached bytes
void pool_stats(int dev, size_t *in_use, size_t *peak, size_t *idle);
void pool_reset_peak(int dev);
// Free device memory of the current device counting the cache's idle blocks.
size_t device_free_bytes();

// ------------------------------------------------------ batched matrices
// A matrix taking part in a batched QR / Jacobi SVD / pseudoinverse apply.
struct MatDesc {
  double2 *a;     // m x n, lda (QR in place: R above, Householder vectors below)
  int m, n, lda;
  double2 *tau;   // [n] Householder scalars
  double2 *T;     // [npanels][nb*nb] compact-WY triangular factors
  double2 *g;     // n x n, ldg: Jacobi work matrix (R, rotated to U S)
  int ldg;
  double2 *v;     // n x n, ldg: Jacobi right vectors
  double2 *u;     // m x n, lda: left singular vectors (kept columns)
  double2 *w;     // n x n, ldg: V S^+ (kept columns)
  double *sv;     // [n] singular values, descending
  int *perm;      // [n] work
  int *rank;      // [1] kept rank
  int *flag;      // [1] Jacobi sweep activity flag
  int ldu;        // leading dimension of u (0: lda)
};

constexpr int kQRNB = 32;   // Householder panel width where it is not tuned (pivoted triangles, LQ)

// One body of an operator: geometry and its P/2+1 distinct mode blocks.
// Sound-hard (km = 0): blocks A'_n, rows = M, cols = N.  Transmission
// (km > 0, eq. (trans)): blocks [[A_n, -A^-_n], [A'_n, -A'^-_n]] of
// rows = 2M (values, then normal derivatives) by cols = 2N (exterior
// coefficients with the sources inside, then interior coefficients at km
// with the sources srho2, sz2 outside).
struct NearLowRank;

struct BodyData {
  int M, N, P, q, nd, ldA;
  int rows, cols;
  double k, km = 0.0;
  DevBuf geom;        // rho z nrho nz [M] each, srho sz [N] each, then srho2 sz2 [N] each
  double *rho, *z, *nrho, *nz, *srho, *sz;
  double *srho2 = nullptr, *sz2 = nullptr;
  std::vector<double> h_rho, h_z, h_nrho, h_nz, h_srho, h_sz, h_srho2, h_sz2;
  bool trans() const { return km > 0.0; }
  DevBuf blocks;      // [nd][cols][ldA]
  DevBuf fac;         // tau, T, g, v, u, w, sv, perm, rank, flag for all nd blocks
  DevBuf descs;       // MatDesc[nd] on device
  std::vector<MatDesc> h_descs;
  std::vector<int> rank;
  std::vector<double> h_sv;   // [nd][cols] singular values after mfs_factor_modes (descending, zero-filled)
  DevBuf src_P;       // point sources at q = P angles, SoA x y z [P*N] each
  // low-rank factors of the surface image blocks of A_else for one lattice
  // (built on first use by a periodic solve whose stored near field does
  // not fit; kept for later solves on the same lattice)
  std::shared_ptr<NearLowRank> lowrank;
};

// ---------------------------------------------------------- launchers
void launch_fill(BodyData &b, hipStream_t s);
// every body's blocks in one persistent launch (work queue of 64-pair tiles)
void launch_fill_all(const std::vector<BodyData *> &bodies, hipStream_t s);
void launch_rhs(const BodyData &b, int nw, const double *kvec_dev, double2 *out, hipStream_t s);
// out[r][b][x] = scale * sum_l in[r][l][x] e^{sgn 2 pi i b l / P}, r < nr, x < X
void launch_dft(int nr, int P, int X, const double2 *in, double2 *out, int sgn, double scale,
                hipStream_t s);
// out[r][b][x] = (1/P) sum_l in[r][x][l] e^{-2 pi i b l / P}: angle samples laid
// out [nr][X][P] to modes [nr][P][X]
void launch_angle_to_modes(int nr, int P, int X, const double2 *in, double2 *out, hipStream_t s);
// sigma[r][l][j] = (1/qs) sum_n c[r][bin(n)][j] e^{+i n 2 pi l / qs}, j < N;
// c has ldc entries per bin (N, or 2N for the exterior half of a
// transmission body's coefficients)
void launch_point_strengths(int nr, int P, int qs, int N, const double2 *c, double2 *sigma,
                            hipStream_t s, int ldc = 0);

struct JacStats {
  double ms = 0.0;       // time of the sweep launches (HIP events)
  int launches = 0;
  double bytes = 0.0;    // algorithmic HBM bytes of the sweeps
  double flops = 0.0;    // algorithmic FP64 flops of the sweeps
  int unconverged = 0;   // matrices still rotating when the sweep cap was reached
};
JacStats jac_run(const MatDesc *descs, const std::vector<MatDesc> &h, int init_mode, double rel_cutoff,
                 hipStream_t s);

// batched QR of nmat matrices described by descs (device) / h (host copy),
// panels of nb = 16, 32 or 64 columns (each matrix's T holds cdiv(n, nb)
// nb x nb factors)
void qr_factor(const MatDesc *descs, const std::vector<MatDesc> &h, hipStream_t s, int nb = kQRNB);
// Column-pivoted QR steps and forms (gpinv.hip, qrcp.hip, qrcp_sketch.hip):
// the triangles of descs in place (R above the diagonal, reflectors below,
// tau), piv[w][i] the original column at position i (identity on entry).
void launch_qrcp_step(const MatDesc *descs, int W, int nmax, int k, double *norms, int *piv, int ld,
                      hipStream_t s);
void qrcp_sketched(const MatDesc *descs, const std::vector<MatDesc> &h, int *piv, int ld, hipStream_t s);
// The same QR (panels of 32) one panel at a time: panel(K0) factors columns
// [K0, K0 + 32) of every matrix and updates the columns after them.
struct QRPanels32 {
  struct Impl;
  Impl *impl;
  QRPanels32(const MatDesc *descs, const std::vector<MatDesc> &h);
  ~QRPanels32();
  QRPanels32(const QRPanels32 &) = delete;
  QRPanels32 &operator=(const QRPanels32 &) = delete;
  void panel(int K0, hipStream_t s);
};
// the panel width for a batch like h: measured once per size class and GPU
// model (see qr.hip), or MFS_QR_NB
int qr_tuned_nb(const std::vector<MatDesc> &h, hipStream_t s);

// y = A^+ x with the kept factors: job layout
//   mode 0 (one-body blocks): mat d = distinct mode, columns = bins d and P-d
//           of nrhs right-hand sides, x: [nrhs][P][M], out: [nrhs][P][N]
//   mode 1 (one matrix per rhs): mat r, one column, x: [nrhs][ldx], out [nrhs][ldo]
struct PinvJob {
  int mode, nmat, P, nrhs, ldx, ldo, maxcols, maxr, maxm, maxn;
  const MatDesc *descs;
  const double2 *x;
  double2 *out;
  double2 *ywork;   // [nmat][maxcols][maxr]
};
void launch_pinv_apply(const PinvJob &j, hipStream_t s);
// mode 1, second stage only: out = W y with y already in j.ywork
void launch_pinv_apply_w(const PinvJob &j, hipStream_t s);
// y[mat][0, n) = (Q^H x)[0, n) for matrices kept as their Householder QR
// (descs: reflectors below the diagonal, T of every nb-column panel), x
// [mat][ldx]; work: qh_apply_work bytes
size_t qh_apply_work(int nmat, int mmax, int ldx);
void launch_qh_apply(const MatDesc *descs, int nmat, int mmax, int nmax, int nb, const double2 *x, int ldx,
                     double2 *work, double2 *y, int ldy, hipStream_t s);

// ------------------------------------------------------- neighbour sums
// Targets are grouped; every group shares an image list and per-rhs weights.
struct NsumGroup {
  int t0, nt;         // target range [t0, t0+nt) (nt padded to 64 in the launch)
  int deriv;          // 0: value, 1: derivative along the target direction
  int nimg;
  int ia[9], ib[9];   // image shifts (a, b)
  // Mirror pairing (0: none).  When the half-turn about the body's axis maps
  // target t to t + mt (t < mt, nt = 2 mt) and source s to s + ms (mod S),
  // image (a, b) onto image mir[.] = (-a, -b), the values of the first mt
  // targets serve the other half through K_(-a,-b)[t + mt][s] =
  // K_(a,b)[t][s + ms]: the on-the-fly sum evaluates half the kernel values,
  // and when mt is a multiple of 64 the stored near field keeps the first mt
  // targets only.
  int mt, ms;
  int mir[9];
  // General pairing of the stored field (pkind 0: none; 1: the shift above;
  // 2: this group's target (a, b) pairs target (m1-1-a, b) of group pg, whose
  // values are not stored; 3: group served by its partner pg (nothing
  // stored); 4: target i pairs target nt-1-i of the same group).  psign is
  // the factor of the mirror values (-1 for a normal derivative whose
  // direction the half-turn reverses); mir[] indexes the partner's images.
  int pkind, pg, psign, m1;
};
struct NsumPlan {
  int ntarget_pad;    // targets padded per group to multiples of 64
  std::vector<NsumGroup> groups;
  DevBuf tgt;         // SoA x y z dx dy dz [ntarget_pad] each
  DevBuf grp;         // NsumGroup[] on device
  DevBuf tile_group;  // int [ntarget_pad/64]
  // optional dense near field (nsum_build_dense): kernel values of every
  // group, image, source and target, for the sources `dense_src` (S of them)
  DevBuf dense, koff;
  DevBuf dense_tiles; // int [ndense_tiles]: the tiles whose values are stored (paired form), most images first
  int ndense_tiles = 0;
  DevBuf sigT;        // [S][MAXR] strengths of one launch, source-major (scratch of the dense sum)
  const double *dense_src = nullptr;
  int dense_S = 0;
  double dense_k = 0.0;
  size_t dense_bytes = 0;
  size_t dense_alg_bytes = 0;   // dense_bytes less the padding of partly filled tiles
};
// out[r][t] = sum_img w[g][img][r] sum_s K(x_t - a ex - b ey, y_s) sigma[r][s]
// w: device [ngroups][9][nrhs] complex; src: SoA x y z [S]; sigma [nrhs][S]
void launch_nsum(const NsumPlan &plan, int nrhs, double k, double ex, double ey,
                 const double *src, int S, const double2 *sigma, const double2 *w,
                 double2 *out, double2 *partial, hipStream_t s);
int nsum_splits(const NsumPlan &plan, int S);
// Both plans' stored, mirror-paired fields in one launch (the surface and
// the wall sums of an iteration read the same strengths): true if both are
// stored for these sources and paired.  partial buffers: nsum_splits(plan,
// S) * nrhs * ntarget_pad each, separate for the two plans.
bool nsum_pair_fusable(const NsumPlan &a, const NsumPlan &b, double k, const double *src, int S, int nrhs);
void launch_nsum_pair(const NsumPlan &pa, const double2 *wa, double2 *outa, double2 *parta, const NsumPlan &pb,
                      const double2 *wb, double2 *outb, double2 *partb, int nrhs, int S, const double2 *sigma,
                      hipStream_t s);
// Fill plan.dense for the sources src (S of them); false (and nothing
// allocated) if it would take more than max_bytes or leave under 2 GiB free.
bool nsum_build_dense(NsumPlan &plan, double k, double ex, double ey, const double *src, int S,
                      size_t max_bytes, hipStream_t s);

// ------------------------------------------------- low-rank image blocks
// A_else on the surface (eq. (A)) as a sum over the eight neighbour images
// of K_e[t][s] = dG/dn_t(x_t - e, y_s), t = l M + m, s = l N + j.  Images
// that a rotation of the lattice about the body's axis carries into each
// other share one factorisation K_e ~ U X (U: T x ell with orthonormal
// columns, X = U^H K_e: ell x S): the rotation by 2 pi / nrot shifts the
// angle index l by P / nrot on both sides, so
// K_{R^r e}[t][s] = K_e[R^-r t][R^-r s].  Square lattices with P divisible
// by 4: the classes (1, 0) and (1, 1), four rotations each; otherwise the
// half-turn: four classes, two rotations each.
struct NearLowRank {
  int T = 0, S = 0, P = 0, M = 0, N = 0;
  int nrot = 0, ncls = 0;
  int shiftT = 0, shiftS = 0;   // index shifts of one rotation step
  double ex = 0.0, ey = 0.0, k = 0.0;
  struct Cls {
    int a = 0, b = 0;           // representative image (a e_x + b e_y)
    int ell = 0, ldu = 0;       // kept columns of U (a multiple of 16); leading dimension of U
    int img[4] = {0, 0, 0, 0};  // index of image R^r (a, b) in the surface group's image list
    double tail = 0.0;          // |R_ell,ell| / max |R_ii| of the sketch's QR at the kept width
    DevBuf U, X;                // U column-major [ell][ldu]; X source-major [S][ell]
  } cls[4];
  double build_ms = 0.0;
  size_t bytes = 0;
};
// Factors for the surface plan `psurf` of body b on lattice lat (nullptr if
// they would not fit in the free device memory).  Blocking.
std::shared_ptr<NearLowRank> build_near_lowrank(const BodyData &b, const NsumPlan &psurf, double ex, double ey,
                                                hipStream_t s);
// out[r][t] (r < nrhs, row stride ldo) = the eight images' phased sum of the
// point strengths sigma[r][S], weights w[img][nrhs] (the surface group's).
// work: device scratch of lowrank_work_bytes(lr, nrhs) bytes.
size_t lowrank_work_bytes(const NearLowRank &lr, int nrhs);
void lowrank_apply(const NearLowRank &lr, int nrhs, const double2 *sigma, const double2 *w, double2 *out,
                   size_t ldo, void *work, hipStream_t s);

// ----------------------------------------------------------- harmonics
// Fill rows of Q (S block and -W blocks) for one wave.
struct QFillArgs {
  double k, ex, ey, z0;
  int p, M1, nrb;
  double2 alpha, beta;
  const double *wall;     // SoA x y z of the 6 walls: R L F B T D, each M1^2
  const double *kx, *ky;  // [nrb]
  const double2 *kz;      // [nrb]
  double2 *Q;             // column-major [8 M1^2][ldq]
  int ldq;
};
// Q of every incidence of a batch (same wall grid and degree), zeroed then filled
void launch_qfill(const std::vector<QFillArgs> &h, hipStream_t s);
// Btilde: values dH_lm/dn (value = 0) or H_lm (value = 1) at the surface
// rings (phi = 0): out [NH][M]
void launch_bfill(int M, int p, double k, const double *rho, const double *z, const double *nrho,
                  const double *nz, double2 *out, hipStream_t s, int value = 0);
// out[r][bin][m] -= sum_{(l,mm): mm = bin mod P} B[(l,mm)][m] d[r][(l,mm)] ; d stride ldd;
// out has ldo entries per bin (M, or 2M with the value rows first)
void launch_bapply(int nrhs, int P, int M, int p, const double2 *B, const double2 *d, int ldd,
                   double2 *out, hipStream_t s, int ldo = 0);
// u[r][t] += sum_lm H_lm(x_t) d[r][lm]
void launch_harm_field(int nrhs, int nt, const double *xyz, int p, double k, const double2 *d,
                       int ldd, double2 *out, hipStream_t s);

// ------------------------------------------------------------- GMRES
void launch_dots(int nw, int nvec, int n, const double2 *V, size_t ldv_w, size_t ldv_i,
                 const double2 *z, double2 *h, hipStream_t s);
void launch_update(int nw, int nvec, int n, const double2 *V, size_t ldv_w, size_t ldv_i,
                   double2 *z, const double2 *h, int hstride, hipStream_t s);
void launch_axpby_op(int nw, int n, const double2 *x, const double2 *g, const double2 *bd,
                     double2 *out, hipStream_t s);
void launch_combine_walls(int nw, int M1sq, const double2 *in, double2 *out, hipStream_t s);

}  // namespace mfs
