// C ABI of libmfs: contexts, one-body operators and their factorisation,
// the solution-operator apply, right-hand sides, point-source transforms,
// neighbour sums and free-space field evaluation.  The periodic solve lives
// in solve.cpp.  Every entry point converts exceptions to an mfs_status.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "capi_impl.hpp"

namespace mfs {

static thread_local std::string g_error;
void set_error(const std::string &msg) { g_error = msg; }
const std::string &get_error() { return g_error; }

void progress(const char *fmt, ...) {
  static const bool on = std::getenv("MFS_PROGRESS") != nullptr;
  if (!on) return;
  va_list ap;
  va_start(ap, fmt);
  std::fprintf(stderr, "[mfs] ");
  std::vfprintf(stderr, fmt, ap);
  std::fprintf(stderr, "\n");
  va_end(ap);
  std::fflush(stderr);
}

static bool finite_all(const double *p, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

void upload(void *dst, const void *src, size_t bytes, hipStream_t s) {
  HIP_CHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
}

// Source points y_jl = (srho_j cos phi_l, srho_j sin phi_l, sz_j), phi_l = 2 pi l / qs,
// SoA x y z [qs*N], index l*N + j.
void source_points_of(const BodyData &b, const std::vector<double> &srho, const std::vector<double> &sz, int qs,
                      DevBuf &out, hipStream_t s) {
  std::vector<double> h((size_t)3 * qs * b.N);
  const size_t S = (size_t)qs * b.N;
  for (int l = 0; l < qs; ++l) {
    // exact reduction: cos/sin of 2 pi l / qs
    const double ang = 2.0 * kPi * l / qs;
    const double c = std::cos(ang), sn = std::sin(ang);
    for (int j = 0; j < b.N; ++j) {
      h[(size_t)l * b.N + j] = srho[j] * c;
      h[S + (size_t)l * b.N + j] = srho[j] * sn;
      h[2 * S + (size_t)l * b.N + j] = sz[j];
    }
  }
  out.alloc(h.size() * sizeof(double));
  upload(out.p, h.data(), h.size() * sizeof(double), s);
  HIP_CHECK(hipStreamSynchronize(s));
}

void source_points(const BodyData &b, int qs, DevBuf &out, hipStream_t s) {
  source_points_of(b, b.h_srho, b.h_sz, qs, out, s);
}

// Build a neighbour-sum plan from host target groups.
void build_plan(NsumPlan &plan, const std::vector<NsumGroup> &groups_in,
                const std::vector<std::vector<double>> &tg /* per group: x y z dx dy dz SoA */,
                hipStream_t s) {
  plan.groups = groups_in;
  int off = 0;
  for (auto &g : plan.groups) {
    g.t0 = off;
    off += round_up(std::max(g.nt, 1), 64);
  }
  plan.ntarget_pad = off;
  const int ntp = off;
  std::vector<double> soa((size_t)6 * ntp, 0.0);
  std::vector<int> tile_group(ntp / 64);
  for (size_t gi = 0; gi < plan.groups.size(); ++gi) {
    const auto &g = plan.groups[gi];
    const int padn = round_up(std::max(g.nt, 1), 64);
    for (int t = 0; t < padn; ++t) {
      const int dst = g.t0 + t;
      if (t < g.nt) {
        for (int c = 0; c < 6; ++c) soa[(size_t)c * ntp + dst] = tg[gi][(size_t)c * g.nt + t];
      } else {
        soa[(size_t)2 * ntp + dst] = 1e3;   // padding target far from every source
      }
    }
    for (int t = 0; t < padn / 64; ++t) tile_group[g.t0 / 64 + t] = (int)gi;
  }
  plan.tgt.alloc(soa.size() * sizeof(double));
  upload(plan.tgt.p, soa.data(), soa.size() * sizeof(double), s);
  plan.grp.alloc(plan.groups.size() * sizeof(NsumGroup));
  upload(plan.grp.p, plan.groups.data(), plan.groups.size() * sizeof(NsumGroup), s);
  plan.tile_group.alloc(tile_group.size() * sizeof(int));
  upload(plan.tile_group.p, tile_group.data(), tile_group.size() * sizeof(int), s);
  HIP_CHECK(hipStreamSynchronize(s));
}

// Surface targets of A_else: the P x M nodes (index l M + m) with their
// normals; one group of normal derivatives, and for a transmission body a
// second group of values at the same nodes.
void surface_plan(const BodyData &b, NsumPlan &plan, hipStream_t s) {
  NsumGroup g{};
  g.nt = b.P * b.M;
  g.deriv = 1;
  g.nimg = 0;
  for (int a = -1; a <= 1; ++a)
    for (int c = -1; c <= 1; ++c)
      if (a != 0 || c != 0) { g.ia[g.nimg] = a; g.ib[g.nimg] = c; ++g.nimg; }
  // The half-turn about the z axis maps the body onto itself, node (l, m)
  // onto (l + P/2, m), source (l, j) onto (l + P/2, j) (both at angles
  // 2 pi l / P, indices l M + m and l N + j) and the shift a e_x + b e_y onto
  // its negative; kernel values and normal derivatives are invariant under
  // it, so the images (a, b) and (-a, -b) share their kernel values (the
  // stored field uses the pairing when (P/2) M fills whole 64-target tiles).
  if (b.P % 2 == 0) {
    g.mt = (b.P / 2) * b.M;
    g.ms = (b.P / 2) * b.N;
    g.pkind = 1;
    g.pg = 0;
    g.psign = 1;
    for (int im = 0; im < g.nimg; ++im)
      for (int jm = 0; jm < g.nimg; ++jm)
        if (g.ia[jm] == -g.ia[im] && g.ib[jm] == -g.ib[im]) g.mir[im] = jm;
  }
  std::vector<double> t((size_t)6 * g.nt);
  const size_t n = g.nt;
  for (int l = 0; l < b.P; ++l) {
    const double ang = 2.0 * kPi * l / b.P;
    const double c = std::cos(ang), sn = std::sin(ang);
    for (int m = 0; m < b.M; ++m) {
      const size_t i = (size_t)l * b.M + m;
      t[i] = b.h_rho[m] * c;
      t[n + i] = b.h_rho[m] * sn;
      t[2 * n + i] = b.h_z[m];
      t[3 * n + i] = b.h_nrho[m] * c;
      t[4 * n + i] = b.h_nrho[m] * sn;
      t[5 * n + i] = b.h_nz[m];
    }
  }
  if (!b.trans()) {
    build_plan(plan, {g}, {t}, s);
  } else {
    NsumGroup gv = g;
    gv.deriv = 0;
    gv.pg = 1;   // its mirror weights are its own
    build_plan(plan, {g, gv}, {t, t}, s);
  }
}

// The 12 wall target groups R L Rx Lx F B Fy By T Tz D Dz (images and kinds).
// With P even (sources at the P angles of ring l N + j, mirror l + P/2) and
// M1 even, the half-turn about the z axis pairs the groups: R with L, F with
// B (wall node (a, b) with node (M1-1-a, b) of the other wall; the first of
// each pair keeps the stored values for both), the x and y derivative groups
// likewise with the sign reversed (their direction turns over), and T, Tz,
// D, Dz each with itself (node i with node M1^2-1-i).
void walls_plan(const mfs_lattice &lat, int P, int N, NsumPlan &plan, hipStream_t s) {
  std::vector<double> wall;
  wall_nodes(lat, wall);
  const int n = lat.M1 * lat.M1;
  std::vector<NsumGroup> groups;
  std::vector<std::vector<double>> tg;
  // wall index in SoA: R0 L1 F2 B3 T4 D5
  const int wall_of[12] = {0, 1, 0, 1, 2, 3, 2, 3, 4, 4, 5, 5};
  const int deriv_of[12] = {0, 0, 1, 1, 0, 0, 1, 1, 0, 1, 0, 1};
  for (int gi = 0; gi < 12; ++gi) {
    NsumGroup g{};
    g.nt = n;
    g.deriv = deriv_of[gi];
    g.nimg = 0;
    const int w = wall_of[gi];
    if (w == 0) { for (int c = -1; c <= 1; ++c) { g.ia[g.nimg] = -1; g.ib[g.nimg++] = c; } }
    else if (w == 1) { for (int c = -1; c <= 1; ++c) { g.ia[g.nimg] = 1; g.ib[g.nimg++] = c; } }
    else if (w == 2) { for (int a = -1; a <= 1; ++a) { g.ia[g.nimg] = a; g.ib[g.nimg++] = -1; } }
    else if (w == 3) { for (int a = -1; a <= 1; ++a) { g.ia[g.nimg] = a; g.ib[g.nimg++] = 1; } }
    else {
      for (int a = -1; a <= 1; ++a)
        for (int c = -1; c <= 1; ++c) { g.ia[g.nimg] = a; g.ib[g.nimg++] = c; }
    }
    std::vector<double> t((size_t)6 * n, 0.0);
    for (int i = 0; i < n; ++i)
      for (int c = 0; c < 3; ++c) t[(size_t)c * n + i] = wall[(size_t)(3 * w + c) * n + i];
    const int dircomp = (w <= 1) ? 0 : (w <= 3 ? 1 : 2);
    for (int i = 0; i < n; ++i) t[(size_t)(3 + dircomp) * n + i] = 1.0;
    groups.push_back(g);
    tg.push_back(std::move(t));
  }
  if (P % 2 == 0 && lat.M1 % 2 == 0) {
    const int partner[12] = {1, 0, 3, 2, 5, 4, 7, 6, 8, 9, 10, 11};
    const int sign[12] = {1, 1, -1, -1, 1, 1, -1, -1, 1, 1, 1, 1};
    for (int gi = 0; gi < 12; ++gi) {
      NsumGroup &g = groups[gi];
      const NsumGroup &q = groups[partner[gi]];
      g.ms = (P / 2) * N;
      g.pg = partner[gi];
      g.psign = sign[gi];
      g.m1 = lat.M1;
      g.pkind = partner[gi] == gi ? 4 : (gi % 2 == 0 ? 2 : 3);
      for (int im = 0; im < g.nimg; ++im)
        for (int jm = 0; jm < q.nimg; ++jm)
          if (q.ia[jm] == -g.ia[im] && q.ib[jm] == -g.ib[im]) g.mir[im] = jm;
    }
  }
  build_plan(plan, groups, tg, s);
}

// Per-rhs weights for the wall groups: w[g][img][r].
void walls_weights(const std::vector<std::complex<double>> &al, const std::vector<std::complex<double>> &be,
                   const NsumPlan &plan, std::vector<double2> &w) {
  const int nr = (int)al.size();
  w.assign((size_t)12 * 9 * nr, cz(0.0, 0.0));
  for (int gi = 0; gi < 12; ++gi) {
    const NsumGroup &g = plan.groups[gi];
    const int wall = gi < 4 ? (gi % 2) : (gi < 8 ? 2 + (gi % 2) : (gi < 10 ? 4 : 5));
    for (int im = 0; im < g.nimg; ++im)
      for (int r = 0; r < nr; ++r) {
        std::complex<double> v = std::pow(al[r], g.ia[im]) * std::pow(be[r], g.ib[im]);
        if (wall == 1) v *= -al[r];   // u_R - alpha u_L
        if (wall == 3) v *= -be[r];   // u_F - beta u_B
        w[((size_t)gi * 9 + im) * nr + r] = cz(v.real(), v.imag());
      }
  }
}

void image_weights(const std::vector<std::complex<double>> &al, const std::vector<std::complex<double>> &be,
                   const NsumPlan &plan, std::vector<double2> &w) {
  const int nr = (int)al.size();
  const int ng = (int)plan.groups.size();
  w.assign((size_t)ng * 9 * nr, cz(0.0, 0.0));
  for (int gi = 0; gi < ng; ++gi) {
    const NsumGroup &g = plan.groups[gi];
    for (int im = 0; im < g.nimg; ++im)
      for (int r = 0; r < nr; ++r) {
        const std::complex<double> v = std::pow(al[r], g.ia[im]) * std::pow(be[r], g.ib[im]);
        w[((size_t)gi * 9 + im) * nr + r] = cz(v.real(), v.imag());
      }
  }
}

void user_plan(const double *user, int nuser, int want, bool nine, NsumPlan &plan, hipStream_t s) {
  NsumGroup g{};
  g.nt = nuser;
  g.deriv = want;
  g.nimg = 0;
  if (nine) {
    for (int a = -1; a <= 1; ++a)
      for (int c = -1; c <= 1; ++c) { g.ia[g.nimg] = a; g.ib[g.nimg++] = c; }
  } else {
    g.ia[0] = 0; g.ib[0] = 0; g.nimg = 1;
  }
  std::vector<double> t((size_t)6 * nuser);
  for (int i = 0; i < nuser; ++i)
    for (int c = 0; c < 6; ++c) t[(size_t)c * nuser + i] = user[(size_t)6 * i + c];
  build_plan(plan, {g}, {t}, s);
}

// ---------------------------------------------------- operator set-up
static void validate_body(const mfs_body &b) {
  MFS_REQUIRE(b.M > 0 && b.N > 0, "M and N must be positive");
  MFS_REQUIRE(b.M >= b.N, "need M >= N (least squares)");
  MFS_REQUIRE(b.P >= 2 && b.P % 2 == 0, "P must be even and >= 2");
  MFS_REQUIRE(b.q >= b.P && b.q % 2 == 0, "q must be even and >= P");
  MFS_REQUIRE(b.k > 0 && std::isfinite(b.k), "k must be positive");
  MFS_REQUIRE(b.rho && b.z && b.nrho && b.nz && b.srho && b.sz, "null geometry pointer");
  MFS_REQUIRE(finite_all(b.rho, b.M) && finite_all(b.z, b.M) && finite_all(b.nrho, b.M) &&
                  finite_all(b.nz, b.M) && finite_all(b.srho, b.N) && finite_all(b.sz, b.N),
              "non-finite geometry");
  for (int j = 0; j < b.N; ++j) MFS_REQUIRE(b.srho[j] > 0.0, "source rho must be > 0");
  for (int m = 0; m < b.M; ++m) MFS_REQUIRE(b.rho[m] > 0.0, "collocation rho must be > 0");
  MFS_REQUIRE(b.km >= 0.0 && std::isfinite(b.km), "km must be 0 (sound-hard) or positive (transmission)");
  if (b.km > 0.0) {
    MFS_REQUIRE(b.srho_out && b.sz_out, "transmission needs the exterior sources srho_out, sz_out");
    MFS_REQUIRE(finite_all(b.srho_out, b.N) && finite_all(b.sz_out, b.N), "non-finite geometry");
    for (int j = 0; j < b.N; ++j) MFS_REQUIRE(b.srho_out[j] > 0.0, "source rho must be > 0");
  }
}

BodyData &body_of(const mfs_op *op, int body) {
  MFS_REQUIRE(op != nullptr, "null operator");
  MFS_REQUIRE(body >= 0 && body < (int)op->bodies.size(), "body index out of range");
  return *op->bodies[body];
}

double2 *op_workspace(const mfs_op *op, size_t bytes) {
  auto *o = const_cast<mfs_op *>(op);
  if (o->work.bytes < bytes) o->work.alloc(bytes);
  return o->work.as<double2>();
}

}  // namespace mfs

using namespace mfs;

#define MFS_API_BEGIN try {
#define MFS_API_END                                                               \
  return MFS_OK;                                                                  \
  }                                                                               \
  catch (const mfs::Error &e) {                                                   \
    mfs::set_error(e.msg);                                                        \
    return e.st;                                                                  \
  }                                                                               \
  catch (const std::exception &e) {                                               \
    mfs::set_error(e.what());                                                     \
    return MFS_ENOMEM;                                                            \
  }

extern "C" {

const char *mfs_last_error(void) { return mfs::get_error().c_str(); }
const char *mfs_version(void) { return "libmfs 0.1 (gfx950)"; }

mfs_status mfs_create(int device, mfs_ctx **out) {
  MFS_API_BEGIN
  MFS_REQUIRE(out != nullptr, "null output");
  int n = 0;
  HIP_CHECK(hipGetDeviceCount(&n));
  MFS_REQUIRE(device >= 0 && device < n, "no such HIP device");
  HIP_CHECK(hipSetDevice(device));
  auto *c = new mfs_ctx;
  c->device = device;
  *out = c;
  MFS_API_END
}

void mfs_destroy(mfs_ctx *ctx) { delete ctx; }

mfs_status mfs_memory_stats(int device, uint64_t *in_use, uint64_t *peak, uint64_t *cached) {
  MFS_API_BEGIN
  int n = 0;
  HIP_CHECK(hipGetDeviceCount(&n));
  MFS_REQUIRE(device >= 0 && device < n, "no such HIP device");
  size_t a = 0, b = 0, c = 0;
  pool_stats(device, &a, &b, &c);
  if (in_use) *in_use = a;
  if (peak) *peak = b;
  if (cached) *cached = c;
  MFS_API_END
}

mfs_status mfs_memory_reset_peak(int device) {
  MFS_API_BEGIN
  int n = 0;
  HIP_CHECK(hipGetDeviceCount(&n));
  MFS_REQUIRE(device >= 0 && device < n, "no such HIP device");
  pool_reset_peak(device);
  MFS_API_END
}

mfs_status mfs_release_cached_memory(int device) {
  MFS_API_BEGIN
  int n = 0;
  HIP_CHECK(hipGetDeviceCount(&n));
  MFS_REQUIRE(device >= 0 && device < n, "no such HIP device");
  pool_trim(device);
  MFS_API_END
}

mfs_status mfs_polar_geometry(const mfs_polar_spec *spec, double *rho, double *z, double *nrho,
                              double *nz, double *srho, double *sz) {
  MFS_API_BEGIN
  MFS_REQUIRE(spec && rho && z && nrho && nz && srho && sz, "null pointer");
  MFS_REQUIRE(spec->M > 0 && spec->N > 0 && spec->a > 0, "bad polar spec");
  MFS_REQUIRE(spec->colloc == 0 || spec->colloc == 1, "colloc must be 0 or 1");
  polar_geometry(*spec, rho, z, nrho, nz, srho, sz);
  MFS_API_END
}

mfs_status mfs_cup_geometry(const mfs_cup_spec *spec, double *rho, double *z, double *nrho, double *nz,
                            double *srho, double *sz) {
  MFS_API_BEGIN
  MFS_REQUIRE(spec && rho && z && nrho && nz && srho && sz, "null pointer");
  MFS_REQUIRE(spec->M > 0 && spec->N > 0, "bad cup spec: M and N must be positive");
  MFS_REQUIRE(spec->outer > 0 && spec->half > 0 && spec->half < 1 && spec->b > 0 && spec->b < kPi,
              "bad cup spec: need outer > 0, 0 < half < 1, 0 < b < pi");
  MFS_REQUIRE(std::fabs(spec->tau) <= spec->half, "bad cup spec: need |tau| <= half");
  MFS_REQUIRE(spec->colloc == 0 || spec->colloc == 1, "colloc must be 0 or 1");
  cup_geometry(*spec, rho, z, nrho, nz, srho, sz);
  MFS_API_END
}

mfs_status mfs_build_operator(mfs_ctx *ctx, const mfs_body *bodies, int32_t nbodies, void *stream,
                              mfs_op **out) {
  MFS_API_BEGIN
  MFS_REQUIRE(ctx && bodies && out && nbodies > 0, "bad arguments");
  for (int i = 0; i < nbodies; ++i) validate_body(bodies[i]);
  HIP_CHECK(hipSetDevice(ctx->device));
  auto op = std::make_unique<mfs_op>();
  op->ctx = ctx;
  op->stream = static_cast<hipStream_t>(stream);
  for (int i = 0; i < nbodies; ++i) {
    const mfs_body &src = bodies[i];
    auto b = std::make_unique<BodyData>();
    b->M = src.M; b->N = src.N; b->P = src.P; b->q = src.q; b->k = src.k; b->km = src.km;
    b->nd = src.P / 2 + 1;
    b->rows = b->trans() ? 2 * src.M : src.M;
    b->cols = b->trans() ? 2 * src.N : src.N;
    b->ldA = round_up(b->rows, 16);
    b->h_rho.assign(src.rho, src.rho + src.M);
    b->h_z.assign(src.z, src.z + src.M);
    b->h_nrho.assign(src.nrho, src.nrho + src.M);
    b->h_nz.assign(src.nz, src.nz + src.M);
    b->h_srho.assign(src.srho, src.srho + src.N);
    b->h_sz.assign(src.sz, src.sz + src.N);
    b->geom.alloc((size_t)(4 * src.M + 4 * src.N) * sizeof(double));
    double *g = b->geom.as<double>();
    b->rho = g; b->z = g + src.M; b->nrho = g + 2 * src.M; b->nz = g + 3 * src.M;
    b->srho = g + 4 * src.M; b->sz = g + 4 * src.M + src.N;
    if (b->trans()) {
      b->h_srho2.assign(src.srho_out, src.srho_out + src.N);
      b->h_sz2.assign(src.sz_out, src.sz_out + src.N);
      b->srho2 = g + 4 * src.M + 2 * src.N;
      b->sz2 = g + 4 * src.M + 3 * src.N;
      upload(b->srho2, src.srho_out, src.N * sizeof(double), op->stream);
      upload(b->sz2, src.sz_out, src.N * sizeof(double), op->stream);
    }
    upload(b->rho, src.rho, src.M * sizeof(double), op->stream);
    upload(b->z, src.z, src.M * sizeof(double), op->stream);
    upload(b->nrho, src.nrho, src.M * sizeof(double), op->stream);
    upload(b->nz, src.nz, src.M * sizeof(double), op->stream);
    upload(b->srho, src.srho, src.N * sizeof(double), op->stream);
    upload(b->sz, src.sz, src.N * sizeof(double), op->stream);
    b->blocks.alloc((size_t)b->nd * b->cols * b->ldA * sizeof(double2));
    source_points(*b, b->P, b->src_P, op->stream);
    op->bodies.push_back(std::move(b));
  }
  // every body's distinct blocks in one persistent launch
  std::vector<BodyData *> all;
  for (auto &bp : op->bodies) all.push_back(bp.get());
  hipEvent_t f0, f1;
  HIP_CHECK(hipEventCreate(&f0));
  HIP_CHECK(hipEventCreate(&f1));
  HIP_CHECK(hipEventRecord(f0, op->stream));
  launch_fill_all(all, op->stream);
  HIP_CHECK(hipEventRecord(f1, op->stream));
  HIP_CHECK(hipEventSynchronize(f1));
  float fms = 0.f;
  HIP_CHECK(hipEventElapsedTime(&fms, f0, f1));
  op->ms_fill = fms;
  (void)hipEventDestroy(f0);
  (void)hipEventDestroy(f1);
  HIP_CHECK(hipStreamSynchronize(op->stream));
  *out = op.release();
  MFS_API_END
}

void mfs_destroy_op(mfs_op *op) { delete op; }

mfs_status mfs_op_blocks(const mfs_op *op, int32_t body, mfs_c128 *out, void *stream) {
  MFS_API_BEGIN
  BodyData &b = body_of(op, body);
  if (op->factored) MFS_THROW(MFS_ESTATE, "blocks were overwritten by mfs_factor_modes");
  MFS_REQUIRE(out != nullptr, "null output");
  HIP_CHECK(hipMemcpy2DAsync(out, (size_t)b.rows * sizeof(double2), b.blocks.p, (size_t)b.ldA * sizeof(double2),
                             (size_t)b.rows * sizeof(double2), (size_t)b.nd * b.cols, hipMemcpyDeviceToDevice,
                             static_cast<hipStream_t>(stream)));
  MFS_API_END
}

mfs_status mfs_factor_modes(mfs_op *op, double rel_cutoff, int32_t *ranks) {
  MFS_API_BEGIN
  MFS_REQUIRE(op != nullptr, "null operator");
  MFS_REQUIRE(rel_cutoff >= 0.0 && rel_cutoff < 1.0, "rel_cutoff must be in [0, 1)");
  if (op->factored) MFS_THROW(MFS_ESTATE, "operator already factored");
  HIP_CHECK(hipSetDevice(op->ctx->device));
  hipStream_t s = op->stream;
  // every distinct block of every body, the widest first, in batched chunks
  // whose factorisation work fits in half of the free device memory
  struct Item {
    int body, d;
    MatDesc m;
    double bytes;
  };
  std::vector<Item> items;
  for (int bi = 0; bi < (int)op->bodies.size(); ++bi) {
    BodyData &b = *op->bodies[bi];
    for (int d = 0; d < b.nd; ++d) {
      Item it{};
      it.body = bi;
      it.d = d;
      it.m.a = b.blocks.as<double2>() + (size_t)d * b.cols * b.ldA;
      it.m.m = b.rows;
      it.m.n = b.cols;
      it.m.lda = b.ldA;
      // copies of the block and of U, the triangles and Jacobi factors, W
      it.bytes = (3.0 * b.ldA * b.cols + 8.0 * (double)b.cols * b.cols) * sizeof(double2);
      items.push_back(it);
    }
  }
  std::stable_sort(items.begin(), items.end(), [](const Item &x, const Item &y) { return x.m.n > y.m.n; });
  const size_t fr = device_free_bytes();
  const double budget = std::max(0.45 * (double)fr, (double)(1ull << 30));
  for (int i = 0; i < 3; ++i)
    if (!op->ev[i]) HIP_CHECK(hipEventCreate(&op->ev[i]));
  for (auto &bp : op->bodies) {
    bp->h_descs.assign(bp->nd, MatDesc{});
    bp->rank.assign(bp->nd, 0);
    bp->h_sv.assign((size_t)bp->nd * bp->cols, 0.0);
  }
  op->gps.clear();
  op->ms_qr = op->ms_svd = 0.0;
  int unconverged = 0;
  size_t c0 = 0;
  while (c0 < items.size()) {
    size_t c1 = c0 + 1;
    double used = items[c0].bytes;
    while (c1 < items.size() && c1 - c0 < 60000 && used + items[c1].bytes <= budget) used += items[c1++].bytes;
    std::vector<MatDesc> in;
    for (size_t i = c0; i < c1; ++i) in.push_back(items[i].m);
    auto g = std::make_unique<GradedPinv>();
    g->ev_qr_done = op->ev[1];
    HIP_CHECK(hipEventRecord(op->ev[0], s));
    graded_pinv(*g, in, rel_cutoff, 0, s);
    HIP_CHECK(hipEventRecord(op->ev[2], s));
    HIP_CHECK(hipStreamSynchronize(s));
    float ms_qr = 0, ms_svd = 0;
    HIP_CHECK(hipEventElapsedTime(&ms_qr, op->ev[0], op->ev[1]));
    HIP_CHECK(hipEventElapsedTime(&ms_svd, op->ev[1], op->ev[2]));
    op->ms_qr += ms_qr;
    op->ms_svd += ms_svd;
    int ldo = 0;
    for (size_t i = c0; i < c1; ++i) ldo = std::max(ldo, items[i].m.n);
    std::vector<double> sv;
    g->singular_values(ldo, sv, s);
    for (size_t i = c0; i < c1; ++i) {
      const Item &it = items[i];
      BodyData &b = *op->bodies[it.body];
      b.h_descs[it.d] = g->h_fin[i - c0];
      b.rank[it.d] = g->kept[i - c0];
      // the Jacobi factor holds the r leading singular values; the rest are
      // below 1e-15 of the largest and stay zero
      std::copy(sv.begin() + (i - c0) * ldo, sv.begin() + (i - c0) * ldo + std::min(ldo, b.cols),
                b.h_sv.begin() + (size_t)it.d * b.cols);
    }
    unconverged += g->jacobi_unconverged;
    g->release_work();
    op->gps.push_back(std::move(g));
    c0 = c1;
  }
  size_t off = 0;
  for (auto &bp : op->bodies) {
    BodyData &b = *bp;
    b.descs.alloc(b.nd * sizeof(MatDesc));
    upload(b.descs.p, b.h_descs.data(), b.nd * sizeof(MatDesc), s);
    if (ranks) std::copy(b.rank.begin(), b.rank.end(), ranks + off);
    off += b.nd;
  }
  HIP_CHECK(hipStreamSynchronize(s));
  // the factors are all the apply reads: the filled blocks are released
  for (auto &bp : op->bodies) bp->blocks.release();
  op->factored = true;
  op->cutoff = rel_cutoff;
  if (unconverged > 0) {
    set_error("mfs_factor_modes: the Jacobi SVD of " + std::to_string(unconverged) +
              " block(s) reached its sweep cap; their factors are those of the last sweep");
    return MFS_ENOTCONV;
  }
  MFS_API_END
}

mfs_status mfs_set_near_field_budget(mfs_op *op, uint64_t max_bytes) {
  MFS_API_BEGIN
  MFS_REQUIRE(op != nullptr, "null pointer");
  op->near_budget = max_bytes;
  MFS_API_END
}

mfs_status mfs_op_timing(const mfs_op *op, double *ms) {
  MFS_API_BEGIN
  MFS_REQUIRE(op != nullptr && ms != nullptr, "null pointer");
  ms[0] = op->ms_fill;
  ms[1] = op->ms_qr;
  ms[2] = op->ms_svd;
  MFS_API_END
}

mfs_status mfs_op_singular_values(const mfs_op *op, int32_t body, double *out) {
  MFS_API_BEGIN
  BodyData &b = body_of(op, body);
  if (!op->factored) MFS_THROW(MFS_ESTATE, "operator not factored");
  MFS_REQUIRE(out != nullptr, "null output");
  std::copy(b.h_sv.begin(), b.h_sv.end(), out);
  MFS_API_END
}

mfs_status mfs_apply_solution_op(const mfs_op *op, int32_t body, int32_t nrhs, const mfs_c128 *in,
                                 int32_t in_layout, mfs_c128 *out, int32_t out_layout, void *stream) {
  MFS_API_BEGIN
  BodyData &b = body_of(op, body);
  check_apply_args(op, nrhs, in, in_layout, out, out_layout);
  if (nrhs == 0) return MFS_OK;
  HIP_CHECK(hipSetDevice(op->ctx->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevBuf im, om;
  if (in_layout == MFS_LAYOUT_ANGLE) im.alloc((size_t)nrhs * b.P * b.rows * sizeof(double2));
  if (out_layout == MFS_LAYOUT_POINTS) om.alloc((size_t)nrhs * b.P * b.cols * sizeof(double2));
  apply_solution_layouts(op, b, nrhs, reinterpret_cast<const double2 *>(in), in_layout,
                         reinterpret_cast<double2 *>(out), out_layout, im.as<double2>(), om.as<double2>(), nullptr,
                         s);
  MFS_API_END
}

mfs_status mfs_rhs_modes(const mfs_op *op, int32_t body, int32_t nwaves, const double *kvec,
                         mfs_c128 *out, void *stream) {
  MFS_API_BEGIN
  BodyData &b = body_of(op, body);
  MFS_REQUIRE(nwaves >= 0 && (nwaves == 0 || (kvec && out)), "bad arguments");
  if (nwaves == 0) return MFS_OK;
  MFS_REQUIRE(finite_all(kvec, 3 * nwaves), "non-finite wave vector");
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevBuf kd((size_t)3 * nwaves * sizeof(double));
  upload(kd.p, kvec, 3 * nwaves * sizeof(double), s);
  launch_rhs(b, nwaves, kd.as<double>(), reinterpret_cast<double2 *>(out), s);
  HIP_CHECK(hipStreamSynchronize(s));
  MFS_API_END
}

mfs_status mfs_point_strengths(const mfs_op *op, int32_t body, int32_t nrhs, int32_t qs, const mfs_c128 *c,
                               mfs_c128 *sigma, void *stream) {
  MFS_API_BEGIN
  BodyData &b = body_of(op, body);
  MFS_REQUIRE(nrhs >= 0 && qs >= b.P && (nrhs == 0 || (c && sigma)), "bad arguments");
  if (nrhs == 0) return MFS_OK;
  launch_point_strengths(nrhs, b.P, qs, b.N, reinterpret_cast<const double2 *>(c),
                         reinterpret_cast<double2 *>(sigma), static_cast<hipStream_t>(stream), b.cols);
  MFS_API_END
}

mfs_status mfs_neighbour_sum(const mfs_op *op, int32_t body, const mfs_lattice *lat, int32_t nrhs,
                             int32_t qs, const mfs_c128 *sigma, const mfs_c128 *ab, int32_t target_set,
                             const double *user, int32_t nuser, int32_t want, mfs_c128 *out,
                             void *stream) {
  MFS_API_BEGIN
  BodyData &b = body_of(op, body);
  MFS_REQUIRE(lat != nullptr && ab != nullptr && sigma != nullptr && out != nullptr, "null pointer");
  MFS_REQUIRE(nrhs >= 1 && nrhs <= 16, "1 <= nrhs <= 16");
  MFS_REQUIRE(lat->ex > 0 && lat->ey > 0, "lattice periods must be positive");
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::vector<std::complex<double>> al(nrhs), be(nrhs);
  for (int r = 0; r < nrhs; ++r) {
    al[r] = {ab[2 * r].re, ab[2 * r].im};
    be[r] = {ab[2 * r + 1].re, ab[2 * r + 1].im};
  }
  NsumPlan plan;
  std::vector<double2> w;
  DevBuf srcbuf;
  const double *src;
  int S;
  if (target_set == MFS_TARGETS_SURFACE || target_set == MFS_TARGETS_WALLS) {
    MFS_REQUIRE(qs == b.P, "SURFACE and WALLS use qs = P");
    src = b.src_P.as<double>();
    S = b.P * b.N;
  } else {
    MFS_REQUIRE(qs >= b.P, "qs >= P");
    source_points(b, qs, srcbuf, s);
    src = srcbuf.as<double>();
    S = qs * b.N;
  }
  int nout = 0;
  if (target_set == MFS_TARGETS_SURFACE) {
    surface_plan(b, plan, s);
    image_weights(al, be, plan, w);
    nout = b.P * b.M;
  } else if (target_set == MFS_TARGETS_WALLS) {
    MFS_REQUIRE(lat->M1 > 0, "M1 > 0");
    walls_plan(*lat, b.P, b.N, plan, s);
    walls_weights(al, be, plan, w);
    nout = 8 * lat->M1 * lat->M1;
  } else if (target_set == MFS_TARGETS_USER) {
    MFS_REQUIRE(user != nullptr && nuser > 0, "user targets required");
    MFS_REQUIRE(want == 0 || want == 1, "want must be 0 or 1");
    user_plan(user, nuser, want, true, plan, s);
    image_weights(al, be, plan, w);
    nout = nuser;
  } else {
    MFS_THROW(MFS_EINVAL, "unknown target set");
  }
  DevBuf wd(w.size() * sizeof(double2));
  upload(wd.p, w.data(), w.size() * sizeof(double2), s);
  const int ntp = plan.ntarget_pad;
  const int nsplit = nsum_splits(plan, S);
  DevBuf tmp((size_t)nrhs * ntp * sizeof(double2) * (1 + nsplit));
  double2 *res = tmp.as<double2>();
  double2 *part = res + (size_t)nrhs * ntp;
  launch_nsum(plan, nrhs, b.k, lat->ex, lat->ey, src, S, reinterpret_cast<const double2 *>(sigma),
              wd.as<double2>(), res, part, s);
  double2 *o = reinterpret_cast<double2 *>(out);
  if (target_set == MFS_TARGETS_WALLS) {
    launch_combine_walls(nrhs, lat->M1 * lat->M1, res, o, s);
  } else {
    for (int r = 0; r < nrhs; ++r)
      HIP_CHECK(hipMemcpyAsync(o + (size_t)r * nout, res + (size_t)r * ntp, nout * sizeof(double2),
                               hipMemcpyDeviceToDevice, s));
  }
  HIP_CHECK(hipStreamSynchronize(s));
  MFS_API_END
}

namespace {
// u[r][t] = sum_{j,l} G_kk(x_t, y_jl) sigma_jl over the qs-node point form of
// the ring sources (srho, sz), the coefficients being columns [col0, col0 + N)
// of c [nrhs][P][cols].
void ring_field(const BodyData &b, double kk, const std::vector<double> &srho, const std::vector<double> &sz,
                int col0, int nrhs, int qs, const mfs_c128 *c, const double *targets, int ntargets, mfs_c128 *out,
                hipStream_t s) {
  DevBuf srcbuf;
  source_points_of(b, srho, sz, qs, srcbuf, s);
  const int S = qs * b.N;
  DevBuf sig((size_t)nrhs * S * sizeof(double2));
  launch_point_strengths(nrhs, b.P, qs, b.N, reinterpret_cast<const double2 *>(c) + col0, sig.as<double2>(), s,
                         b.cols);
  std::vector<double> u6((size_t)6 * ntargets, 0.0);
  for (int t = 0; t < ntargets; ++t)
    for (int k = 0; k < 3; ++k) u6[(size_t)6 * t + k] = targets[(size_t)3 * t + k];
  NsumPlan plan;
  user_plan(u6.data(), ntargets, 0, false, plan, s);
  std::vector<double2> w((size_t)9 * nrhs, cz(0.0, 0.0));
  for (int r = 0; r < nrhs; ++r) w[r] = cz(1.0, 0.0);
  DevBuf wd(w.size() * sizeof(double2));
  upload(wd.p, w.data(), w.size() * sizeof(double2), s);
  const int ntp = plan.ntarget_pad;
  const int nsplit = nsum_splits(plan, S);
  DevBuf tmp((size_t)nrhs * ntp * sizeof(double2) * (1 + nsplit));
  double2 *res = tmp.as<double2>();
  launch_nsum(plan, nrhs, kk, 1.0, 1.0, srcbuf.as<double>(), S, sig.as<double2>(), wd.as<double2>(), res,
              res + (size_t)nrhs * ntp, s);
  double2 *o = reinterpret_cast<double2 *>(out);
  for (int r = 0; r < nrhs; ++r)
    HIP_CHECK(hipMemcpyAsync(o + (size_t)r * ntargets, res + (size_t)r * ntp, ntargets * sizeof(double2),
                             hipMemcpyDeviceToDevice, s));
  HIP_CHECK(hipStreamSynchronize(s));
}
}  // namespace

mfs_status mfs_field_free(const mfs_op *op, int32_t body, int32_t nrhs, int32_t qs, const mfs_c128 *c,
                          const double *targets, int32_t ntargets, mfs_c128 *out, void *stream) {
  MFS_API_BEGIN
  BodyData &b = body_of(op, body);
  MFS_REQUIRE(nrhs >= 1 && nrhs <= 16, "1 <= nrhs <= 16");
  MFS_REQUIRE(qs >= b.P && c && targets && ntargets > 0 && out, "bad arguments");
  ring_field(b, b.k, b.h_srho, b.h_sz, 0, nrhs, qs, c, targets, ntargets, out, static_cast<hipStream_t>(stream));
  MFS_API_END
}

mfs_status mfs_field_interior(const mfs_op *op, int32_t body, int32_t nrhs, int32_t qs, const mfs_c128 *c,
                              const double *targets, int32_t ntargets, mfs_c128 *out, void *stream) {
  MFS_API_BEGIN
  BodyData &b = body_of(op, body);
  if (!b.trans()) MFS_THROW(MFS_EINVAL, "the body is sound-hard: no interior field");
  MFS_REQUIRE(nrhs >= 1 && nrhs <= 16, "1 <= nrhs <= 16");
  MFS_REQUIRE(qs >= b.P && c && targets && ntargets > 0 && out, "bad arguments");
  ring_field(b, b.km, b.h_srho2, b.h_sz2, b.N, nrhs, qs, c, targets, ntargets, out,
             static_cast<hipStream_t>(stream));
  MFS_API_END
}

}  // extern "C"
