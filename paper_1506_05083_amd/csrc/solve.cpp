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

#include "capi_impl.hpp"
#include "gpinv.hpp"

namespace mfs {

void qr_factor(const MatDesc *descs, const std::vector<MatDesc> &h, hipStream_t s);
void launch_dft_ld(int nr, int P, int X, const double2 *in, size_t ld_in, double2 *out, int sgn,
                   double scale, hipStream_t s);

void apply_pinv_body(const mfs_op *op, const BodyData &b, int nrhs, const double2 *x, double2 *out,
                     hipStream_t s) {
  const size_t need = (size_t)b.nd * 32 * b.N * sizeof(double2);
  double2 *yw = op_workspace(op, need);
  for (int r0 = 0; r0 < nrhs; r0 += 16) {
    const int nr = std::min(16, nrhs - r0);
    PinvJob j{};
    j.mode = 0;
    j.nmat = b.nd;
    j.P = b.P;
    j.nrhs = nr;
    j.maxcols = 2 * nr;
    j.maxr = b.N;
    j.maxm = b.M;
    j.maxn = b.N;
    j.descs = b.descs.as<MatDesc>();
    j.x = x + (size_t)r0 * b.P * b.M;
    j.out = out + (size_t)r0 * b.P * b.N;
    j.ywork = yw;
    launch_pinv_apply(j, s);
  }
}

namespace {

using cplx = std::complex<double>;

struct QStore {
  DevBuf a, fac;
  MatDesc d{};
};

struct Solver {
  const mfs_op *op;
  BodyData &b;
  mfs_lattice lat;
  int W, P, M, N, MP, NH, rows, ldq, NQmax, maxit;
  hipStream_t s;
  std::vector<cplx> al, be;
  std::vector<double> kv;
  std::vector<std::vector<RBOrder>> orders;
  // periodizer
  std::vector<QStore> Q;
  DevBuf qflags, qdescs, Bvals, walls_soa;
  std::vector<MatDesc> h_qdescs;
  std::vector<int> qrank;
  GradedPinv gp;
  // plans
  NsumPlan psurf, pwalls;
  DevBuf wsurf, wwalls;
  // work
  DevBuf V, Z, XIN, C, SIG, GS, GH, WR, CY, XI, PART, YW, H1, SC;
  int nsplit_s = 1, nsplit_w = 1;
  // timing: events around every neighbour-sum launch, the dense bytes each streamed
  std::vector<hipEvent_t> nsum_ev;
  std::vector<double> nsum_bytes;
  bool time_nsum = true;
  double near_fill_ms = 0.0;

  Solver(const mfs_op *o, BodyData &body, const mfs_lattice &l, int nw, int mi, hipStream_t st)
      : op(o), b(body), lat(l), W(nw), maxit(mi), s(st) {
    P = b.P; M = b.M; N = b.N; MP = P * M;
    NH = (lat.p + 1) * (lat.p + 1);
    rows = 8 * lat.M1 * lat.M1;
    ldq = round_up(rows, 16);
  }
  ~Solver() {
    for (auto e : nsum_ev) (void)hipEventDestroy(e);
  }

  void setup_periodizer(double rel_cutoff) {
    // walls
    std::vector<double> wall;
    wall_nodes(lat, wall);
    walls_soa.alloc(wall.size() * sizeof(double));
    upload(walls_soa.p, wall.data(), wall.size() * sizeof(double), s);
    qflags.alloc((size_t)2 * W * sizeof(int));
    int *flags = qflags.as<int>();
    Q.resize(W);
    h_qdescs.resize(W);
    NQmax = 0;
    std::vector<DevBuf> ordbufs(W);
    for (int w = 0; w < W; ++w) {
      const int nrb = (int)orders[w].size();
      const int NQ = NH + 2 * nrb;
      NQmax = std::max(NQmax, NQ);
      MFS_REQUIRE(NQ <= rows, "periodizer: Q has more columns than rows (raise M1)");
      QStore &q = Q[w];
      q.a.alloc((size_t)ldq * NQ * sizeof(double2));
      MatDesc &d = q.d;
      d = MatDesc{};
      d.a = q.a.as<double2>(); d.m = rows; d.n = NQ; d.lda = ldq;
      d.flag = flags + w;
      d.rank = flags + W + w;
      h_qdescs[w] = d;
      // Rayleigh-Bloch data
      std::vector<double> kx(nrb), ky(nrb);
      std::vector<double2> kz(nrb);
      for (int o = 0; o < nrb; ++o) {
        kx[o] = orders[w][o].kx;
        ky[o] = orders[w][o].ky;
        kz[o] = cz(orders[w][o].kz.real(), orders[w][o].kz.imag());
      }
      ordbufs[w].alloc((size_t)std::max(1, nrb) * (2 * sizeof(double) + sizeof(double2)));
      double *kxd = ordbufs[w].as<double>();
      double *kyd = kxd + nrb;
      double2 *kzd = reinterpret_cast<double2 *>(kyd + nrb);
      if (nrb > 0) {
        upload(kxd, kx.data(), nrb * sizeof(double), s);
        upload(kyd, ky.data(), nrb * sizeof(double), s);
        upload(kzd, kz.data(), nrb * sizeof(double2), s);
      }
      QFillArgs a{};
      a.k = b.k; a.ex = lat.ex; a.ey = lat.ey; a.z0 = lat.z0;
      a.p = lat.p; a.M1 = lat.M1; a.nrb = nrb;
      a.alpha = cz(al[w].real(), al[w].imag());
      a.beta = cz(be[w].real(), be[w].imag());
      a.wall = walls_soa.as<double>();
      a.kx = kxd; a.ky = kyd; a.kz = kzd;
      a.Q = d.a; a.ldq = ldq;
      launch_qfill(a, s);
    }
    qdescs.alloc(W * sizeof(MatDesc));
    upload(qdescs.p, h_qdescs.data(), W * sizeof(MatDesc), s);
    HIP_CHECK(hipStreamSynchronize(s));   // ordbufs are released on return
    graded_pinv(gp, h_qdescs, rel_cutoff, s);
    qrank = gp.kept;
    // harmonics' Neumann data on the surface rings
    Bvals.alloc((size_t)NH * M * sizeof(double2));
    launch_bfill(M, lat.p, b.k, b.rho, b.z, b.nrho, b.nz, Bvals.as<double2>(), s);
  }

  void setup_sums() {
    surface_plan(b, psurf, s);
    walls_plan(lat, pwalls, s);
    std::vector<double2> w1, w2;
    image_weights(al, be, psurf, w1);
    walls_weights(al, be, pwalls, w2);
    wsurf.alloc(w1.size() * sizeof(double2));
    upload(wsurf.p, w1.data(), w1.size() * sizeof(double2), s);
    wwalls.alloc(w2.size() * sizeof(double2));
    upload(wwalls.p, w2.data(), w2.size() * sizeof(double2), s);
    const int S = P * N;
    nsplit_s = nsum_splits(psurf, S);
    nsplit_w = nsum_splits(pwalls, S);
    // dense near field, surface first (the larger share of the iteration)
    if (op->near_budget > 0) {
      hipEvent_t f0, f1;
      HIP_CHECK(hipEventCreate(&f0));
      HIP_CHECK(hipEventCreate(&f1));
      HIP_CHECK(hipEventRecord(f0, s));
      const size_t budget = (size_t)std::min<uint64_t>(op->near_budget, (uint64_t)SIZE_MAX);
      if (nsum_build_dense(psurf, b.k, lat.ex, lat.ey, b.src_P.as<double>(), S, budget, s))
        nsum_build_dense(pwalls, b.k, lat.ex, lat.ey, b.src_P.as<double>(), S, budget - psurf.dense_bytes, s);
      HIP_CHECK(hipEventRecord(f1, s));
      HIP_CHECK(hipEventSynchronize(f1));
      float ms = 0.f;
      HIP_CHECK(hipEventElapsedTime(&ms, f0, f1));
      near_fill_ms = (psurf.dense.p || pwalls.dense.p) ? ms : 0.0;
      (void)hipEventDestroy(f0);
      (void)hipEventDestroy(f1);
    }
    // work buffers
    V.alloc((size_t)W * (maxit + 1) * MP * sizeof(double2));
    Z.alloc((size_t)W * MP * sizeof(double2));
    XIN.alloc((size_t)W * MP * sizeof(double2));
    C.alloc((size_t)W * P * N * sizeof(double2));
    SIG.alloc((size_t)W * P * N * sizeof(double2));
    GS.alloc((size_t)W * psurf.ntarget_pad * sizeof(double2));
    GH.alloc((size_t)W * MP * sizeof(double2));
    WR.alloc((size_t)W * pwalls.ntarget_pad * sizeof(double2));
    CY.alloc((size_t)W * rows * sizeof(double2));
    XI.alloc((size_t)W * NQmax * sizeof(double2));
    const size_t part = std::max((size_t)nsplit_s * W * psurf.ntarget_pad, (size_t)nsplit_w * W * pwalls.ntarget_pad);
    PART.alloc(part * sizeof(double2));
    YW.alloc(std::max((size_t)b.nd * 2 * W * N, (size_t)W * NQmax) * sizeof(double2));
    H1.alloc((size_t)W * (maxit + 2) * 2 * sizeof(double2));
    SC.alloc((size_t)W * sizeof(double));
  }

  void pinv_A0(const double2 *x, double2 *out) {
    PinvJob j{};
    j.mode = 0; j.nmat = b.nd; j.P = P; j.nrhs = W; j.maxcols = 2 * W; j.maxr = N; j.maxm = M; j.maxn = N;
    j.descs = b.descs.as<MatDesc>(); j.x = x; j.out = out; j.ywork = YW.as<double2>();
    launch_pinv_apply(j, s);
  }

  // neighbour sum of the point strengths in SIG over plan (weights w) into out
  void nsum(const NsumPlan &plan, const DevBuf &w, double2 *out) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (time_nsum) {
      HIP_CHECK(hipEventCreate(&e0));
      HIP_CHECK(hipEventCreate(&e1));
      HIP_CHECK(hipEventRecord(e0, s));
    }
    launch_nsum(plan, W, b.k, lat.ex, lat.ey, b.src_P.as<double>(), P * N, SIG.as<double2>(), w.as<double2>(), out,
                PART.as<double2>(), s);
    if (time_nsum) {
      HIP_CHECK(hipEventRecord(e1, s));
      nsum_ev.push_back(e0);
      nsum_ev.push_back(e1);
      nsum_bytes.push_back((double)plan.dense_bytes);
    }
  }

  // XI = Q^+ (C c) for mode coefficients in C
  void c_then_qpinv(const double2 *cmodes) {
    launch_point_strengths(W, P, P, N, cmodes, SIG.as<double2>(), s);
    nsum(pwalls, wwalls, WR.as<double2>());
    launch_combine_walls(W, lat.M1 * lat.M1, WR.as<double2>(), CY.as<double2>(), s);
    PinvJob j{};
    j.mode = 1; j.nmat = W; j.P = P; j.nrhs = 1; j.ldx = rows; j.ldo = NQmax; j.maxcols = 1;
    j.maxr = NQmax; j.maxm = rows; j.maxn = NQmax;
    j.descs = gp.apply_descs(); j.x = CY.as<double2>(); j.out = XI.as<double2>(); j.ywork = YW.as<double2>();
    launch_pinv_apply(j, s);
  }

  // out = (I + A_else A_0^+ - B Q^+ C A_0^+) x
  void apply_op(const double2 *x, double2 *out) {
    pinv_A0(x, C.as<double2>());
    launch_point_strengths(W, P, P, N, C.as<double2>(), SIG.as<double2>(), s);
    nsum(psurf, wsurf, GS.as<double2>());
    launch_dft_ld(W, P, M, GS.as<double2>(), psurf.ntarget_pad, GH.as<double2>(), -1, 1.0 / P, s);
    launch_axpby_op(W, MP, x, GH.as<double2>(), nullptr, out, s);
    // the wall rows reuse SIG computed above
    nsum(pwalls, wwalls, WR.as<double2>());
    launch_combine_walls(W, lat.M1 * lat.M1, WR.as<double2>(), CY.as<double2>(), s);
    PinvJob j{};
    j.mode = 1; j.nmat = W; j.P = P; j.nrhs = 1; j.ldx = rows; j.ldo = NQmax; j.maxcols = 1;
    j.maxr = NQmax; j.maxm = rows; j.maxn = NQmax;
    j.descs = gp.apply_descs(); j.x = CY.as<double2>(); j.out = XI.as<double2>(); j.ywork = YW.as<double2>();
    launch_pinv_apply(j, s);
    launch_bapply(W, P, M, lat.p, Bvals.as<double2>(), XI.as<double2>(), NQmax, out, s);
  }

  double nsum_avg_ms() {
    if (nsum_ev.empty()) return 0.0;
    double tot = 0.0;
    for (size_t i = 0; i + 1 < nsum_ev.size(); i += 2) {
      float ms = 0.f;
      HIP_CHECK(hipEventElapsedTime(&ms, nsum_ev[i], nsum_ev[i + 1]));
      tot += ms;
    }
    return tot / (nsum_ev.size() / 2);
  }
};

}  // namespace
}  // namespace mfs

using namespace mfs;

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

    // ---------------- GMRES (unrestarted, CGS2, lockstep over waves)
    const int MP = S.MP;
    const size_t ldw = (size_t)(maxit + 1) * MP;
    double2 *V = S.V.as<double2>();
    double2 *Zb = S.Z.as<double2>();
    double2 *Hd = S.H1.as<double2>();
    double *SCd = S.SC.as<double>();
    std::vector<double2> hbuf((size_t)W * (maxit + 2) * 2);
    // ||f||
    launch_dots(W, 1, MP, FH.as<double2>(), (size_t)MP, 0, FH.as<double2>(), Hd, s);
    HIP_CHECK(hipMemcpyAsync(hbuf.data(), Hd, W * sizeof(double2), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    std::vector<double> beta0(W), scale(W);
    for (int w = 0; w < W; ++w) {
      beta0[w] = std::sqrt(std::max(hbuf[w].x, 0.0));
      scale[w] = beta0[w] > 0 ? 1.0 / beta0[w] : 0.0;
    }
    upload(SCd, scale.data(), W * sizeof(double), s);
    launch_scale(W, MP, FH.as<double2>(), MP, V, ldw, SCd, s);
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
      const double2 *vj = V + (size_t)j * MP;
      // z = Op(v_j): v_j of wave w is at V + w*ldw + j*MP; Op works on [W][MP] so gather
      for (int w = 0; w < W; ++w)
        HIP_CHECK(hipMemcpyAsync(Zb + (size_t)w * MP, vj + w * ldw, MP * sizeof(double2),
                                 hipMemcpyDeviceToDevice, s));
      HIP_CHECK(hipMemcpyAsync(S.XIN.p, Zb, (size_t)W * MP * sizeof(double2), hipMemcpyDeviceToDevice, s));
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
      HIP_CHECK(hipMemcpyAsync(hbuf.data(), Hd, (size_t)W * (2 * nv + 1) * sizeof(double2),
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
      if (any_active) {
        upload(SCd, scale.data(), W * sizeof(double), s);
        launch_scale(W, MP, Zb, MP, V + (size_t)(j + 1) * MP, ldw, SCd, s);
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
    int kmax = 0;
    for (int w = 0; w < W; ++w) kmax = std::max(kmax, iters[w]);
    std::vector<double2> ny((size_t)W * std::max(kmax, 1), cz(0.0, 0.0));
    for (int w = 0; w < W; ++w)
      for (int i = 0; i < iters[w]; ++i) ny[(size_t)w * kmax + i] = cz(-y[w][i].real(), -y[w][i].imag());
    DevBuf X((size_t)W * MP * sizeof(double2)), Yd(ny.size() * sizeof(double2));
    launch_zero(X.as<double2>(), (long)W * MP, s);
    upload(Yd.p, ny.data(), ny.size() * sizeof(double2), s);
    if (kmax > 0) launch_update(W, kmax, MP, V, ldw, MP, X.as<double2>(), Yd.as<double2>(), kmax, s);
    S.pinv_A0(X.as<double2>(), S.C.as<double2>());
    S.c_then_qpinv(S.C.as<double2>());
    std::vector<double2> xi((size_t)W * S.NQmax);
    HIP_CHECK(hipMemcpyAsync(xi.data(), S.XI.p, xi.size() * sizeof(double2), hipMemcpyDeviceToHost, s));
    // fields at targets
    std::vector<double2> unear, uh;
    if (ntargets > 0) {
      DevBuf srcf, sigf((size_t)W * q_field * b.N * sizeof(double2));
      source_points(b, q_field, srcf, s);
      launch_point_strengths(W, b.P, q_field, b.N, S.C.as<double2>(), sigf.as<double2>(), s);
      std::vector<double> u6((size_t)6 * ntargets, 0.0);
      for (int t = 0; t < ntargets; ++t)
        for (int k = 0; k < 3; ++k) u6[(size_t)6 * t + k] = targets[(size_t)3 * t + k];
      NsumPlan pu;
      user_plan(u6.data(), ntargets, 0, true, pu, s);
      std::vector<double2> wu;
      image_weights(S.al, S.be, pu, wu);
      DevBuf wud(wu.size() * sizeof(double2));
      upload(wud.p, wu.data(), wu.size() * sizeof(double2), s);
      const int Sf = q_field * b.N;
      const int ns = nsum_splits(pu, Sf);
      DevBuf ur((size_t)W * pu.ntarget_pad * (1 + ns) * sizeof(double2));
      launch_nsum(pu, W, b.k, lat->ex, lat->ey, srcf.as<double>(), Sf, sigf.as<double2>(), wud.as<double2>(),
                  ur.as<double2>(), ur.as<double2>() + (size_t)W * pu.ntarget_pad, s);
      DevBuf hf((size_t)W * ntargets * sizeof(double2)), tx((size_t)3 * ntargets * sizeof(double));
      launch_zero(hf.as<double2>(), (long)W * ntargets, s);
      upload(tx.p, targets, (size_t)3 * ntargets * sizeof(double), s);
      launch_harm_field(W, ntargets, tx.as<double>(), lat->p, b.k, S.XI.as<double2>(), S.NQmax,
                        hf.as<double2>(), s);
      unear.resize((size_t)W * pu.ntarget_pad);
      uh.resize((size_t)W * ntargets);
      HIP_CHECK(hipMemcpyAsync(unear.data(), ur.p, unear.size() * sizeof(double2), hipMemcpyDeviceToHost, s));
      HIP_CHECK(hipMemcpyAsync(uh.data(), hf.p, uh.size() * sizeof(double2), hipMemcpyDeviceToHost, s));
      HIP_CHECK(hipStreamSynchronize(s));
      for (int w = 0; w < W; ++w)
        for (int t = 0; t < ntargets; ++t) {
          const double2 a = unear[(size_t)w * pu.ntarget_pad + t], h = uh[(size_t)w * ntargets + t];
          // d = -xi_d
          res[w].field[t] = mfs_c128{a.x - h.x, a.y - h.y};
        }
    }
    HIP_CHECK(hipEventRecord(ev[4], s));
    HIP_CHECK(hipStreamSynchronize(s));
    const int NH = S.NH;
    for (int w = 0; w < W; ++w) {
      const auto &o = S.orders[w];
      const int nrb = (int)o.size();
      mfs_result &r = res[w];
      r.iters = iters[w];
      r.resid = resid[w];
      r.q_rank = S.qrank[w];
      r.nq_cols = NH + 2 * nrb;
      double flux = 0.0, kz00 = 0.0;
      for (int i = 0; i < nrb; ++i) {
        const double2 av = xi[(size_t)w * S.NQmax + NH + i];
        const double2 bv = xi[(size_t)w * S.NQmax + NH + nrb + i];
        if (r.m) r.m[i] = o[i].m;
        if (r.n) r.n[i] = o[i].n;
        if (r.kz) r.kz[i] = mfs_c128{o[i].kz.real(), o[i].kz.imag()};
        const cplx a(-av.x, -av.y), bcoef(-bv.x, -bv.y);
        if (r.a) r.a[i] = mfs_c128{a.real(), a.imag()};
        if (r.b) r.b[i] = mfs_c128{bcoef.real(), bcoef.imag()};
        if (o[i].kz.imag() == 0.0 && o[i].kz.real() > 0.0) {
          cplx bb = bcoef;
          if (o[i].m == 0 && o[i].n == 0) {
            bb += std::exp(cplx(0.0, -S.kv[3 * w + 2] * lat->z0));
            kz00 = o[i].kz.real();
          }
          flux += o[i].kz.real() * (std::norm(a) + std::norm(bb));
        }
      }
      r.eps_flux = std::fabs(flux - kz00);
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
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    if (notconv) {
      set_error("GMRES reached maxit before the tolerance");
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
