// Periodic solve (Sec. 4.2 of the paper): per-incidence periodizer set-up,
// batched right-preconditioned GMRES on eq. (iter) and recovery of the
// Bragg amplitudes and fields, for up to 16 incident waves at once.
//
// Operator of eq. (iter) applied to a batch X [W][P][M] of surface
// unknowns (all on the GPU):
//   c  = A_0^+ X                     per-mode factors (apply.hip)
//   s  = point strengths of c        q = P angles (dft.hip)
//   g  = 8-image phased sum at the P x M surface nodes, normal derivative
//   Z  = X + FFT(g)/P                = X + A_else A_0^+ X
//   Cy = wall rows of C from s       (3x3 cancellation)
//   xi = Q^+ Cy                      per-wave truncated factors of Q
//   Z -= B~ xi_d                     harmonics' Neumann data, mode-sparse
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include <string>

#include "solver.hpp"

namespace mfs {

size_t apply_pinv_work_bytes(const BodyData &b) { return (size_t)b.nd * 32 * b.cols * sizeof(double2); }

void apply_pinv_body(const mfs_op *op, const BodyData &b, int nrhs, const double2 *x, double2 *out,
                     hipStream_t s, double2 *yw) {
  if (!yw) yw = op_workspace(op, apply_pinv_work_bytes(b));
  for (int r0 = 0; r0 < nrhs; r0 += 16) {
    const int nr = std::min(16, nrhs - r0);
    PinvJob j{};
    j.mode = 0;
    j.nmat = b.nd;
    j.P = b.P;
    j.nrhs = nr;
    j.maxcols = 2 * nr;
    j.maxr = b.cols;
    j.maxm = b.rows;
    j.maxn = b.cols;
    j.descs = b.descs.as<MatDesc>();
    j.x = x + (size_t)r0 * b.P * b.rows;
    j.out = out + (size_t)r0 * b.P * b.cols;
    j.ywork = yw;
    launch_pinv_apply(j, s);
  }
}

void check_apply_args(const mfs_op *op, int nrhs, const void *in, int in_layout, const void *out, int out_layout) {
  if (!op->factored) MFS_THROW(MFS_ESTATE, "mfs_factor_modes has not run");
  MFS_REQUIRE(nrhs >= 0 && (nrhs == 0 || (in && out)), "bad arguments");
  MFS_REQUIRE(in_layout == MFS_LAYOUT_MODES || in_layout == MFS_LAYOUT_ANGLE,
              "in_layout must be MFS_LAYOUT_MODES or MFS_LAYOUT_ANGLE");
  MFS_REQUIRE(out_layout == MFS_LAYOUT_MODES || out_layout == MFS_LAYOUT_POINTS,
              "out_layout must be MFS_LAYOUT_MODES or MFS_LAYOUT_POINTS");
}

void apply_solution_layouts(const mfs_op *op, const BodyData &b, int nrhs, const double2 *in, int in_layout,
                            double2 *out, int out_layout, double2 *in_modes, double2 *out_modes, double2 *yw,
                            hipStream_t s) {
  if (nrhs == 0) return;
  const double2 *x = in;
  if (in_layout == MFS_LAYOUT_ANGLE) {
    launch_angle_to_modes(nrhs, b.P, b.rows, in, in_modes, s);
    x = in_modes;
  }
  double2 *c = out_layout == MFS_LAYOUT_POINTS ? out_modes : out;
  apply_pinv_body(op, b, nrhs, x, c, s, yw);
  if (out_layout == MFS_LAYOUT_POINTS) launch_point_strengths(nrhs, b.P, b.P, b.N, c, out, s, b.cols);
}

}  // namespace mfs

using namespace mfs;

namespace {
// pinned host memory (hipHostMalloc), freed on every way out
struct PinnedBuf {
  void *p = nullptr;
  explicit PinnedBuf(size_t n) {
    if (hipHostMalloc(&p, n, hipHostMallocDefault) != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      throw Error{MFS_ENOMEM, "hipHostMalloc of " + std::to_string(n) + " bytes failed"};
    }
  }
  ~PinnedBuf() {
    if (p) (void)hipHostFree(p);
  }
  PinnedBuf(const PinnedBuf &) = delete;
  PinnedBuf &operator=(const PinnedBuf &) = delete;
};
}  // namespace

extern "C" mfs_status mfs_solve_incident(mfs_ctx *ctx, const mfs_op *op, int32_t body, const mfs_lattice *lat,
                                         int32_t nwaves, const mfs_wave *waves, double tol, int32_t maxit,
                                         double rel_cutoff, const double *targets, int32_t ntargets,
                                         int32_t q_field, mfs_result *res, mfs_solve_timing *timing) {
  try {
    MFS_REQUIRE(ctx && op && lat && waves && res, "null pointer");
    BodyData &b = body_of(op, body);
    if (!op->factored) MFS_THROW(MFS_ESTATE, "mfs_factor_modes has not run");
    MFS_REQUIRE(nwaves >= 1 && nwaves <= 16, "1 <= nwaves <= 16");
    MFS_REQUIRE(tol > 0 && maxit >= 1 && maxit <= 2000, "bad GMRES tolerance or maxit");
    MFS_REQUIRE(rel_cutoff >= 0 && rel_cutoff < 1, "bad cutoff");
    MFS_REQUIRE(lat->ex > 0 && lat->ey > 0 && lat->z0 > 0 && lat->N0 > 0, "bad lattice");
    MFS_REQUIRE(lat->p >= 1 && lat->p <= 96, "1 <= p <= 96");
    MFS_REQUIRE(lat->M1 >= 2 && lat->M1 % 2 == 0, "M1 must be even and >= 2");
    MFS_REQUIRE(ntargets >= 0 && (ntargets == 0 || (targets && q_field >= b.P)), "bad targets");
    HIP_CHECK(hipSetDevice(ctx->device));
    hipStream_t s = op->stream;
    const int W = nwaves;
    Solver S(op, b, *lat, W, maxit, s);
    // MFS_QPINV_REFLECT=1: a full-rank Q is applied from its QR's
    // reflectors, panel by panel, instead of forming U = Q_1 (measured on the
    // k = 10 workload: 31 us a panel launch, 41 launches an apply at 32-column
    // panels, more than forming U once and streaming it: not the default)
    {
      const char *e = std::getenv("MFS_QPINV_REFLECT");
      S.qreflect = e && std::string(e) == "1";
    }
    // host per-wave data
    S.al.resize(W); S.be.resize(W); S.kv.resize(3 * W); S.orders.resize(W);
    bool cap_ok = true;
    for (int w = 0; w < W; ++w) {
      const double th = waves[w].theta, ph = waves[w].phi;
      MFS_REQUIRE(std::isfinite(th) && std::isfinite(ph), "non-finite incidence");
      double *kv = &S.kv[3 * w];
      kv[0] = b.k * std::sin(th) * std::cos(ph);
      kv[1] = b.k * std::sin(th) * std::sin(ph);
      kv[2] = -b.k * std::cos(th);
      S.al[w] = std::exp(cplx(0.0, kv[0] * lat->ex));
      S.be[w] = std::exp(cplx(0.0, kv[1] * lat->ey));
      rb_orders(b.k, kv, *lat, S.orders[w]);
      res[w].norders = (int)S.orders[w].size();
      if (res[w].cap_orders < res[w].norders) cap_ok = false;
      bool has00 = false;
      for (auto &o : S.orders[w]) has00 |= (o.m == 0 && o.n == 0);
      MFS_REQUIRE(has00, "Rayleigh-Bloch cutoff excludes the (0,0) order");
    }
    if (!cap_ok) MFS_THROW(MFS_EINVAL, "result cap_orders too small (norders set)");

    hipEvent_t ev[5];
    for (auto &e : ev) HIP_CHECK(hipEventCreate(&e));
    HIP_CHECK(hipEventRecord(ev[0], s));
    // right-hand sides
    DevBuf kvd((size_t)3 * W * sizeof(double)), FH((size_t)W * S.MP * sizeof(double2));
    upload(kvd.p, S.kv.data(), 3 * W * sizeof(double), s);
    launch_rhs(b, W, kvd.as<double>(), FH.as<double2>(), s);
    HIP_CHECK(hipEventRecord(ev[1], s));
    S.setup_periodizer(rel_cutoff);
    HIP_CHECK(hipEventRecord(ev[2], s));
    S.setup_sums();
    progress("near sums ready (%s)", S.psurf.dense.p ? "stored" : "on the fly");

    // ---------------- GMRES (unrestarted, CGS2, lockstep over waves)
    const int MP = S.MP;
    const size_t ldw = (size_t)(maxit + 1) * MP;
    double2 *V = S.V.as<double2>();
    double2 *Zb = S.Z.as<double2>();
    double2 *Hd = S.H1.as<double2>();
    double *SCd = S.SC.as<double>();
    // host side of the per-iteration exchange in pinned memory (DMA copies, no staging)
    PinnedBuf hpin((size_t)W * (maxit + 2) * 2 * sizeof(double2) + (size_t)W * sizeof(double));
    double2 *hbuf = static_cast<double2 *>(hpin.p);
    double *scale = reinterpret_cast<double *>(hbuf + (size_t)W * (maxit + 2) * 2);
    // ||f||
    launch_dots(W, 1, MP, FH.as<double2>(), (size_t)MP, 0, FH.as<double2>(), Hd, s);
    HIP_CHECK(hipMemcpyAsync(hbuf, Hd, W * sizeof(double2), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    std::vector<double> beta0(W);
    for (int w = 0; w < W; ++w) {
      beta0[w] = std::sqrt(std::max(hbuf[w].x, 0.0));
      scale[w] = beta0[w] > 0 ? 1.0 / beta0[w] : 0.0;
    }
    upload(SCd, scale, W * sizeof(double), s);
    launch_scale2(W, MP, FH.as<double2>(), MP, V, ldw, S.XIN.as<double2>(), MP, SCd, s);
    std::vector<std::vector<cplx>> H(W, std::vector<cplx>((size_t)(maxit + 1) * maxit, 0.0));
    std::vector<std::vector<double>> cs(W, std::vector<double>(maxit, 0.0));
    std::vector<std::vector<cplx>> sn(W, std::vector<cplx>(maxit, 0.0)), g(W, std::vector<cplx>(maxit + 1, 0.0));
    std::vector<int> iters(W, 0);
    std::vector<char> active(W, 1);
    std::vector<double> resid(W, 0.0);
    std::vector<std::vector<cplx>> y(W);
    for (int w = 0; w < W; ++w) {
      g[w][0] = beta0[w];
      if (beta0[w] == 0.0) { active[w] = 0; iters[w] = 0; }
    }
    auto Hat = [&](int w, int i, int j) -> cplx & { return H[w][(size_t)j * (maxit + 1) + i]; };
    auto solve_y = [&](int w, int k) {
      y[w].assign(k, 0.0);
      for (int i = k - 1; i >= 0; --i) {
        cplx acc = g[w][i];
        for (int l = i + 1; l < k; ++l) acc -= Hat(w, i, l) * y[w][l];
        y[w][i] = acc / Hat(w, i, i);
      }
    };
    int jdone = 0;
    bool any_active = false;
    for (int w = 0; w < W; ++w) any_active |= active[w] != 0;
    for (int j = 0; j < maxit && any_active; ++j) {
      // z = Op(v_j): v_j of every wave is in XIN as well ([W][MP], written
      // with the basis vector)
      S.apply_op(S.XIN.as<double2>(), Zb);
      // CGS2
      const int nv = j + 1;
      double2 *h1 = Hd, *h2 = Hd + (size_t)W * nv;
      launch_dots(W, nv, MP, V, ldw, MP, Zb, h1, s);
      launch_update(W, nv, MP, V, ldw, MP, Zb, h1, nv, s);
      launch_dots(W, nv, MP, V, ldw, MP, Zb, h2, s);
      launch_update(W, nv, MP, V, ldw, MP, Zb, h2, nv, s);
      double2 *hn = h2 + (size_t)W * nv;
      launch_dots(W, 1, MP, Zb, (size_t)MP, 0, Zb, hn, s);
      HIP_CHECK(hipMemcpyAsync(hbuf, Hd, (size_t)W * (2 * nv + 1) * sizeof(double2),
                               hipMemcpyDeviceToHost, s));
      HIP_CHECK(hipStreamSynchronize(s));
      any_active = false;
      for (int w = 0; w < W; ++w) {
        scale[w] = 0.0;
        if (!active[w]) continue;
        for (int i = 0; i < nv; ++i) {
          const double2 a1 = hbuf[(size_t)w * nv + i], a2 = hbuf[(size_t)W * nv + (size_t)w * nv + i];
          Hat(w, i, j) = cplx(a1.x + a2.x, a1.y + a2.y);
        }
        const double hnext = std::sqrt(std::max(hbuf[(size_t)2 * W * nv + w].x, 0.0));
        Hat(w, j + 1, j) = hnext;
        // previous rotations
        for (int i = 0; i < j; ++i) {
          const cplx a = Hat(w, i, j), c2 = Hat(w, i + 1, j);
          Hat(w, i, j) = cs[w][i] * a + sn[w][i] * c2;
          Hat(w, i + 1, j) = -std::conj(sn[w][i]) * a + cs[w][i] * c2;
        }
        const cplx a = Hat(w, j, j);
        const double bb = std::abs(Hat(w, j + 1, j));
        const double r = std::hypot(std::abs(a), bb);
        if (r == 0.0) { cs[w][j] = 1.0; sn[w][j] = 0.0; }
        else if (std::abs(a) == 0.0) { cs[w][j] = 0.0; sn[w][j] = 1.0; Hat(w, j, j) = r; }
        else {
          const cplx ph = a / std::abs(a);
          cs[w][j] = std::abs(a) / r;
          sn[w][j] = ph * bb / r;
          Hat(w, j, j) = ph * r;
        }
        Hat(w, j + 1, j) = 0.0;
        g[w][j + 1] = -std::conj(sn[w][j]) * g[w][j];
        g[w][j] = cs[w][j] * g[w][j];
        resid[w] = std::abs(g[w][j + 1]) / beta0[w];
        if (resid[w] <= tol || hnext <= 1e-300) {
          active[w] = 0;
          iters[w] = j + 1;
          solve_y(w, j + 1);
        } else {
          any_active = true;
          scale[w] = 1.0 / hnext;
        }
      }
      jdone = j + 1;
      if (j % 5 == 4 || !any_active) {
        double worst = 0.0;
        for (int w = 0; w < W; ++w) worst = std::max(worst, resid[w]);
        progress("GMRES iteration %d: largest relative residual %.2e", j + 1, worst);
      }
      if (any_active) {
        upload(SCd, scale, W * sizeof(double), s);
        launch_scale2(W, MP, Zb, MP, V + (size_t)(j + 1) * MP, ldw, S.XIN.as<double2>(), MP, SCd, s);
      }
    }
    bool notconv = false;
    for (int w = 0; w < W; ++w)
      if (active[w]) {
        notconv = true;
        iters[w] = jdone;
        solve_y(w, jdone);
      }
    HIP_CHECK(hipEventRecord(ev[3], s));

    // ---------------- recovery: eta~ = V y, eta = A_0^+ eta~, xi = -Q^+ C eta
    std::vector<double2> xi, uf;
    S.recover(V, ldw, y, iters, targets, ntargets, q_field, xi, uf);
    HIP_CHECK(hipEventRecord(ev[4], s));
    HIP_CHECK(hipStreamSynchronize(s));
    for (int w = 0; w < W; ++w) {
      mfs_result &r = res[w];
      r.iters = iters[w];
      r.resid = resid[w];
      for (int t = 0; t < ntargets; ++t)
        r.field[t] = mfs_c128{uf[(size_t)w * ntargets + t].x, uf[(size_t)w * ntargets + t].y};
      S.amplitudes(w, xi.data() + (size_t)w * S.NQmax, r);
    }
    if (timing) {
      float t01, t12, t23, t34, t04;
      HIP_CHECK(hipEventElapsedTime(&t01, ev[0], ev[1]));
      HIP_CHECK(hipEventElapsedTime(&t12, ev[1], ev[2]));
      HIP_CHECK(hipEventElapsedTime(&t23, ev[2], ev[3]));
      HIP_CHECK(hipEventElapsedTime(&t34, ev[3], ev[4]));
      HIP_CHECK(hipEventElapsedTime(&t04, ev[0], ev[4]));
      timing->rhs = t01;
      timing->periodizer = t12;
      timing->gmres = t23;
      timing->recover = t34;
      timing->total = t04;
      timing->nsum_avg = S.nsum_avg_ms();
      timing->nsum_launches = (int)(S.nsum_ev.size() / 2);
      timing->jacobi_ms = S.gp.jacobi_ms;
      timing->jacobi_launches = S.gp.jacobi_launches;
      timing->jacobi_bytes = S.gp.jacobi_bytes;
      timing->jacobi_flops = S.gp.jacobi_flops;
      timing->near_fill_ms = S.near_fill_ms;
      double nb = 0.0;
      for (double x : S.nsum_bytes) nb += x;
      timing->near_bytes = S.nsum_bytes.empty() ? 0.0 : nb / (double)S.nsum_bytes.size();
      double na = 0.0;
      for (double x : S.nsum_alg_bytes) na += x;
      timing->near_alg_bytes = S.nsum_alg_bytes.empty() ? 0.0 : na / (double)S.nsum_alg_bytes.size();
      timing->near_mode = S.near_mode;
      timing->q_qr_ms = S.gp.qr_ms;
      timing->q_qr_flops = S.gp.qr_flops;
      timing->q_post_ms = S.gp.post_ms;
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    if (notconv) {
      set_error("GMRES reached maxit before the tolerance");
      return MFS_ENOTCONV;
    }
    if (S.gp.jacobi_unconverged > 0) {
      set_error("the Jacobi SVD of the periodizer Q of " + std::to_string(S.gp.jacobi_unconverged) +
                " wave(s) reached its sweep cap; the results use the factors of the last sweep");
      return MFS_ENOTCONV;
    }
    return MFS_OK;
  } catch (const Error &e) {
    set_error(e.msg);
    return e.st;
  } catch (const std::exception &e) {
    set_error(e.what());
    return MFS_ENOMEM;
  }
}
