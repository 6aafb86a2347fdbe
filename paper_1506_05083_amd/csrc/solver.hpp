// Batched periodic solver of eq. (iter) (Sec. 4.2): per-incidence
// periodizer set-up, the operator (I + A_else A_0^+ - B Q^+ C A_0^+) applied
// to a batch of right-hand sides, and the pieces of the recovery.  Used by
// mfs_solve_incident (one batch) and by the serving loop (a fixed pool of
// slots that incident waves enter and leave between GMRES iterations).
#pragma once

#include <algorithm>
#include <cmath>
#include <complex>
#include <memory>
#include <vector>

#include "capi_impl.hpp"
#include "gpinv.hpp"

namespace mfs {

// launch_dft with the input rows ld_in apart and the output bins ldo apart
// (ldo <= 0: X)
void launch_dft_ld(int nr, int P, int X, const double2 *in, size_t ld_in, double2 *out, int sgn,
                   double scale, hipStream_t s, int ldo = 0);

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
  int Mr, Nc;   // per-mode system rows and columns (2M x 2N for transmission)
  hipStream_t s;
  std::vector<cplx> al, be;
  std::vector<double> kv;
  std::vector<std::vector<RBOrder>> orders;
  // periodizer
  std::vector<QStore> Q;
  DevBuf qflags, qdescs, Bvals, Bvals_v, walls_soa;
  std::vector<MatDesc> h_qdescs;
  std::vector<int> qrank;
  GradedPinv gp;
  bool qreflect = false;            // let a full-rank Q keep its QR's reflectors instead of forming U = Q_1
  DevBuf QHW;                       // work of the reflector apply
  const MatDesc *qdesc = nullptr;   // Q^+ factors of every wave (default: gp's)
  size_t near_limit = SIZE_MAX;     // bound on the stored near field besides the operator's
  // plans
  NsumPlan psurf, pwalls;
  DevBuf wsurf, wwalls;
  // low-rank image blocks of the surface sums (when their stored values do not fit)
  std::shared_ptr<NearLowRank> lowrank;
  DevBuf LRW;
  // work
  DevBuf V, Z, XIN, C, SIG, GS, GH, WR, CY, XI, PART, PART2, YW, H1, SC;
  int nsplit_s = 1, nsplit_w = 1;
  // timing: events around every neighbour-sum launch, the dense bytes each streamed
  std::vector<hipEvent_t> nsum_ev;
  std::vector<double> nsum_bytes, nsum_alg_bytes;
  // where the neighbour sums' kernel values come from: 0 evaluated on the fly
  // (near-field budget 0), 1 stored, 2 on the fly because the stored field
  // did not fit the budget or the free device memory
  int near_mode = 0;
  bool time_nsum = true;
  double near_fill_ms = 0.0;

  Solver(const mfs_op *o, BodyData &body, const mfs_lattice &l, int nw, int mi, hipStream_t st)
      : op(o), b(body), lat(l), W(nw), maxit(mi), s(st) {
    P = b.P; M = b.M; N = b.N; Mr = b.rows; Nc = b.cols; MP = P * Mr;
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
    std::vector<QFillArgs> qargs(W);
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
      qargs[w] = a;
    }
    launch_qfill(qargs, s);
    qdescs.alloc(W * sizeof(MatDesc));
    upload(qdescs.p, h_qdescs.data(), W * sizeof(MatDesc), s);
    HIP_CHECK(hipStreamSynchronize(s));   // ordbufs are released on return
    progress("periodizer: Q filled for %d waves, %d x %d at most; factoring", W, rows, NQmax);
    // Q's columns equilibrated: the harmonics of high degree are smaller than
    // the low ones by far more than the cutoff on the walls, and would
    // otherwise be dropped whatever their use
    graded_pinv(gp, h_qdescs, rel_cutoff, kQPivotMinCols, s, true, qreflect);
    if (gp.reflect) QHW.alloc(qh_apply_work(W, rows, rows));
    qrank = gp.kept;
    progress("periodizer: factored (%s; Jacobi %.0f ms, %d launches)",
             gp.direct ? "full rank, no SVD"
             : gp.cod  ? "pivoted triangle, truncated complete orthogonal decomposition"
             : gp.pivoted ? "pivoted triangle" : "ordered triangle",
             gp.jacobi_ms, gp.jacobi_launches);
    setup_bvals();
  }

  void setup_sums() {
    surface_plan(b, psurf, s);
    walls_plan(lat, b.P, b.N, pwalls, s);
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
    const uint64_t near_budget = std::min<uint64_t>(op->near_budget, (uint64_t)near_limit);
    if (near_budget > 0) {
      hipEvent_t f0, f1;
      HIP_CHECK(hipEventCreate(&f0));
      HIP_CHECK(hipEventCreate(&f1));
      HIP_CHECK(hipEventRecord(f0, s));
      const size_t budget = (size_t)std::min<uint64_t>(near_budget, (uint64_t)SIZE_MAX);
      if (nsum_build_dense(psurf, b.k, lat.ex, lat.ey, b.src_P.as<double>(), S, budget, s))
        nsum_build_dense(pwalls, b.k, lat.ex, lat.ey, b.src_P.as<double>(), S, budget - psurf.dense_bytes, s);
      HIP_CHECK(hipEventRecord(f1, s));
      HIP_CHECK(hipEventSynchronize(f1));
      float ms = 0.f;
      HIP_CHECK(hipEventElapsedTime(&ms, f0, f1));
      near_fill_ms = (psurf.dense.p || pwalls.dense.p) ? ms : 0.0;
      near_mode = (psurf.dense.p && pwalls.dense.p) ? 1 : 2;
      if (near_mode == 2)
        progress("near field: %s stored; the other sums run on the fly (budget or free memory too small)",
                 psurf.dense.p ? "surface sums" : "nothing");
      (void)hipEventDestroy(f0);
      (void)hipEventDestroy(f1);
    }
    // Surface sums from low-rank factors of the image blocks when their
    // stored values did not fit (MFS_NEAR_LOWRANK: 0 never, 1 then
    // (default), 2 whenever the surface values are not stored).  The factors
    // depend on the body and the lattice only and stay with the operator.
    {
      const char *e = std::getenv("MFS_NEAR_LOWRANK");
      const int mode = e ? std::atoi(e) : 1;
      if (!psurf.dense.p && !b.trans() && W <= 16 && mode > 0 && (near_mode == 2 || mode == 2)) {
        auto &c = b.lowrank;
        if (!(c && c->ex == lat.ex && c->ey == lat.ey && c->k == b.k && c->P == P && c->M == M && c->N == N)) {
          c.reset();
          c = build_near_lowrank(b, psurf, lat.ex, lat.ey, s);
          near_fill_ms = c ? c->build_ms : 0.0;
        } else {
          near_fill_ms = 0.0;
        }
        lowrank = c;
        if (lowrank) {
          LRW.alloc(lowrank_work_bytes(*lowrank, W));
          near_mode = 3;
          progress("near field: surface sums from low-rank image blocks (%.2f GB, built in %.0f ms)",
                   lowrank->bytes / 1e9, lowrank->build_ms);
        }
      }
    }
    // work buffers
    V.alloc((size_t)W * (maxit + 1) * MP * sizeof(double2));
    Z.alloc((size_t)W * MP * sizeof(double2));
    XIN.alloc((size_t)W * MP * sizeof(double2));
    C.alloc((size_t)W * P * Nc * sizeof(double2));
    SIG.alloc((size_t)W * P * N * sizeof(double2));
    GS.alloc((size_t)W * psurf.ntarget_pad * sizeof(double2));
    GH.alloc((size_t)W * MP * sizeof(double2));
    WR.alloc((size_t)W * pwalls.ntarget_pad * sizeof(double2));
    CY.alloc((size_t)W * rows * sizeof(double2));
    XI.alloc((size_t)W * NQmax * sizeof(double2));
    const size_t part = std::max((size_t)nsplit_s * W * psurf.ntarget_pad, (size_t)nsplit_w * W * pwalls.ntarget_pad);
    PART.alloc(part * sizeof(double2));
    // the wall sums' slices when they run in the surface sums' launch
    if (nsum_pair_fusable(psurf, pwalls, b.k, b.src_P.as<double>(), P * N, W))
      PART2.alloc((size_t)nsplit_w * W * pwalls.ntarget_pad * sizeof(double2));
    YW.alloc(std::max((size_t)b.nd * 2 * W * Nc, (size_t)W * NQmax) * sizeof(double2));
    H1.alloc((size_t)W * (maxit + 2) * 2 * sizeof(double2));
    SC.alloc((size_t)W * sizeof(double));
  }

  const MatDesc *qpinv_descs() const { return qdesc ? qdesc : gp.apply_descs(); }

  // XI = Q^+ CY for every wave: U^H then W, or, when the factorisation kept
  // the QR's reflectors in place of U = Q_1 (the direct form), Q^H from the
  // reflectors panel by panel, then W
  void apply_qpinv() {
    PinvJob j{};
    j.mode = 1; j.nmat = W; j.P = P; j.nrhs = 1; j.ldx = rows; j.ldo = NQmax; j.maxcols = 1;
    j.maxr = NQmax; j.maxm = rows; j.maxn = NQmax;
    j.descs = qpinv_descs(); j.x = CY.as<double2>(); j.out = XI.as<double2>(); j.ywork = YW.as<double2>();
    if (!qdesc && gp.reflect) {
      launch_qh_apply(gp.qr_descs(), W, rows, NQmax, gp.qr_nb, CY.as<double2>(), rows, QHW.as<double2>(),
                      YW.as<double2>(), NQmax, s);
      launch_pinv_apply_w(j, s);
    } else {
      launch_pinv_apply(j, s);
    }
  }

  // phase weights of the neighbour sums from al, be (after a wave changes)
  void upload_weights() {
    std::vector<double2> w1, w2;
    image_weights(al, be, psurf, w1);
    walls_weights(al, be, pwalls, w2);
    upload(wsurf.p, w1.data(), w1.size() * sizeof(double2), s);
    upload(wwalls.p, w2.data(), w2.size() * sizeof(double2), s);
  }

  // B~ (the harmonics' Neumann data on the surface rings, and for a
  // transmission body their values), wave independent
  void setup_bvals() {
    Bvals.alloc((size_t)NH * M * sizeof(double2));
    launch_bfill(M, lat.p, b.k, b.rho, b.z, b.nrho, b.nz, Bvals.as<double2>(), s, 0);
    if (b.trans()) {
      Bvals_v.alloc((size_t)NH * M * sizeof(double2));
      launch_bfill(M, lat.p, b.k, b.rho, b.z, b.nrho, b.nz, Bvals_v.as<double2>(), s, 1);
    }
  }

  // Recovery of the waves w with iters[w] > 0 from their GMRES coefficients
  // y[w] (eta~ = V y): eta = A_0^+ eta~, xi = -Q^+ C eta, and the field at the
  // targets (near sum of the q_field-node point sources + harmonics).
  // xi: host [W][NQmax]; u: host [W][ntargets].  Blocking.
  void recover(const double2 *Vb, size_t ldw, const std::vector<std::vector<cplx>> &y,
               const std::vector<int> &iters, const double *targets, int ntargets, int q_field,
               std::vector<double2> &xi, std::vector<double2> &u) {
    int kmax = 0;
    for (int w = 0; w < W; ++w) kmax = std::max(kmax, iters[w]);
    std::vector<double2> ny((size_t)W * std::max(kmax, 1), cz(0.0, 0.0));
    for (int w = 0; w < W; ++w)
      for (int i = 0; i < iters[w]; ++i) ny[(size_t)w * kmax + i] = cz(-y[w][i].real(), -y[w][i].imag());
    DevBuf X((size_t)W * MP * sizeof(double2)), Yd(ny.size() * sizeof(double2));
    launch_zero(X.as<double2>(), (long)W * MP, s);
    upload(Yd.p, ny.data(), ny.size() * sizeof(double2), s);
    if (kmax > 0) launch_update(W, kmax, MP, Vb, ldw, MP, X.as<double2>(), Yd.as<double2>(), kmax, s);
    pinv_A0(X.as<double2>(), C.as<double2>());
    c_then_qpinv(C.as<double2>());
    xi.assign((size_t)W * NQmax, cz(0.0, 0.0));
    HIP_CHECK(hipMemcpyAsync(xi.data(), XI.p, xi.size() * sizeof(double2), hipMemcpyDeviceToHost, s));
    u.assign((size_t)W * ntargets, cz(0.0, 0.0));
    if (ntargets > 0) {
      DevBuf srcf, sigf((size_t)W * q_field * b.N * sizeof(double2));
      source_points(b, q_field, srcf, s);
      launch_point_strengths(W, b.P, q_field, b.N, C.as<double2>(), sigf.as<double2>(), s, Nc);
      std::vector<double> u6((size_t)6 * ntargets, 0.0);
      for (int t = 0; t < ntargets; ++t)
        for (int k = 0; k < 3; ++k) u6[(size_t)6 * t + k] = targets[(size_t)3 * t + k];
      NsumPlan pu;
      user_plan(u6.data(), ntargets, 0, true, pu, s);
      std::vector<double2> wu;
      image_weights(al, be, pu, wu);
      DevBuf wud(wu.size() * sizeof(double2));
      upload(wud.p, wu.data(), wu.size() * sizeof(double2), s);
      const int Sf = q_field * b.N;
      const int ns = nsum_splits(pu, Sf);
      DevBuf ur((size_t)W * pu.ntarget_pad * (1 + ns) * sizeof(double2));
      launch_nsum(pu, W, b.k, lat.ex, lat.ey, srcf.as<double>(), Sf, sigf.as<double2>(), wud.as<double2>(),
                  ur.as<double2>(), ur.as<double2>() + (size_t)W * pu.ntarget_pad, s);
      DevBuf hf((size_t)W * ntargets * sizeof(double2)), tx((size_t)3 * ntargets * sizeof(double));
      launch_zero(hf.as<double2>(), (long)W * ntargets, s);
      upload(tx.p, targets, (size_t)3 * ntargets * sizeof(double), s);
      launch_harm_field(W, ntargets, tx.as<double>(), lat.p, b.k, XI.as<double2>(), NQmax, hf.as<double2>(), s);
      std::vector<double2> unear((size_t)W * pu.ntarget_pad), uh((size_t)W * ntargets);
      HIP_CHECK(hipMemcpyAsync(unear.data(), ur.p, unear.size() * sizeof(double2), hipMemcpyDeviceToHost, s));
      HIP_CHECK(hipMemcpyAsync(uh.data(), hf.p, uh.size() * sizeof(double2), hipMemcpyDeviceToHost, s));
      HIP_CHECK(hipStreamSynchronize(s));
      for (int w = 0; w < W; ++w)
        for (int t = 0; t < ntargets; ++t) {
          const double2 a = unear[(size_t)w * pu.ntarget_pad + t], h = uh[(size_t)w * ntargets + t];
          u[(size_t)w * ntargets + t] = cz(a.x - h.x, a.y - h.y);   // d = -xi_d
        }
    }
    HIP_CHECK(hipStreamSynchronize(s));
  }

  // Bragg amplitudes a = -xi_a, b = -xi_b of wave w, its orders and eps_flux
  void amplitudes(int w, const double2 *xw, mfs_result &r) const {
    const auto &o = orders[w];
    const int nrb = (int)o.size();
    r.q_rank = qrank.empty() ? 0 : qrank[w];
    r.nq_cols = NH + 2 * nrb;
    double flux = 0.0, kz00 = 0.0;
    for (int i = 0; i < nrb; ++i) {
      const double2 av = xw[NH + i];
      const double2 bv = xw[NH + nrb + i];
      if (r.m) r.m[i] = o[i].m;
      if (r.n) r.n[i] = o[i].n;
      if (r.kz) r.kz[i] = mfs_c128{o[i].kz.real(), o[i].kz.imag()};
      const cplx a(-av.x, -av.y), bcoef(-bv.x, -bv.y);
      if (r.a) r.a[i] = mfs_c128{a.real(), a.imag()};
      if (r.b) r.b[i] = mfs_c128{bcoef.real(), bcoef.imag()};
      if (o[i].kz.imag() == 0.0 && o[i].kz.real() > 0.0) {
        cplx bb = bcoef;
        if (o[i].m == 0 && o[i].n == 0) {
          bb += std::exp(cplx(0.0, -kv[3 * w + 2] * lat.z0));
          kz00 = o[i].kz.real();
        }
        flux += o[i].kz.real() * (std::norm(a) + std::norm(bb));
      }
    }
    r.eps_flux = std::fabs(flux - kz00);
  }

  void pinv_A0(const double2 *x, double2 *out) {
    PinvJob j{};
    j.mode = 0; j.nmat = b.nd; j.P = P; j.nrhs = W; j.maxcols = 2 * W; j.maxr = Nc; j.maxm = Mr; j.maxn = Nc;
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
      nsum_alg_bytes.push_back((double)plan.dense_alg_bytes);
    }
  }

  // the surface sums into GS and the wall sums into WR in one launch over
  // both stored fields, timed like one neighbour sum (bytes: both fields)
  void nsum_surface_and_walls() {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (time_nsum) {
      HIP_CHECK(hipEventCreate(&e0));
      HIP_CHECK(hipEventCreate(&e1));
      HIP_CHECK(hipEventRecord(e0, s));
    }
    launch_nsum_pair(psurf, wsurf.as<double2>(), GS.as<double2>(), PART.as<double2>(), pwalls,
                     wwalls.as<double2>(), WR.as<double2>(), PART2.as<double2>(), W, P * N, SIG.as<double2>(), s);
    if (time_nsum) {
      HIP_CHECK(hipEventRecord(e1, s));
      nsum_ev.push_back(e0);
      nsum_ev.push_back(e1);
      nsum_bytes.push_back((double)(psurf.dense_bytes + pwalls.dense_bytes));
      nsum_alg_bytes.push_back((double)(psurf.dense_alg_bytes + pwalls.dense_alg_bytes));
    }
  }

  // the surface sums of the point strengths in SIG from the low-rank image
  // blocks, timed like the direct sums (bytes: the factors streamed)
  void surface_sum_lowrank(double2 *out) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (time_nsum) {
      HIP_CHECK(hipEventCreate(&e0));
      HIP_CHECK(hipEventCreate(&e1));
      HIP_CHECK(hipEventRecord(e0, s));
    }
    lowrank_apply(*lowrank, W, SIG.as<double2>(), wsurf.as<double2>(), out, psurf.ntarget_pad, LRW.p, s);
    if (time_nsum) {
      HIP_CHECK(hipEventRecord(e1, s));
      nsum_ev.push_back(e0);
      nsum_ev.push_back(e1);
      nsum_bytes.push_back((double)lowrank->bytes);
      nsum_alg_bytes.push_back((double)lowrank->bytes);
    }
  }

  // XI = Q^+ (C c) for mode coefficients in C
  void c_then_qpinv(const double2 *cmodes) {
    launch_point_strengths(W, P, P, N, cmodes, SIG.as<double2>(), s, Nc);
    nsum(pwalls, wwalls, WR.as<double2>());
    launch_combine_walls(W, lat.M1 * lat.M1, WR.as<double2>(), CY.as<double2>(), s);
    apply_qpinv();
  }

  // out = (I + A_else A_0^+ - B Q^+ C A_0^+) x
  void apply_op(const double2 *x, double2 *out) {
    pinv_A0(x, C.as<double2>());
    launch_point_strengths(W, P, P, N, C.as<double2>(), SIG.as<double2>(), s, Nc);
    // both stored fields in one launch when they can (the wall rows read the
    // same strengths), else the surface sums now and the wall sums below
    const bool fused = !lowrank && PART2.p && nsum_pair_fusable(psurf, pwalls, b.k, b.src_P.as<double>(), P * N, W);
    if (fused) nsum_surface_and_walls();
    else if (lowrank) surface_sum_lowrank(GS.as<double2>());
    else nsum(psurf, wsurf, GS.as<double2>());
    if (!b.trans()) {
      launch_dft_ld(W, P, M, GS.as<double2>(), psurf.ntarget_pad, GH.as<double2>(), -1, 1.0 / P, s, M);
    } else {
      // values (second target group) into rows [0, M), normal derivatives into [M, 2M)
      launch_dft_ld(W, P, M, GS.as<double2>() + psurf.groups[1].t0, psurf.ntarget_pad, GH.as<double2>(), -1,
                    1.0 / P, s, Mr);
      launch_dft_ld(W, P, M, GS.as<double2>() + psurf.groups[0].t0, psurf.ntarget_pad, GH.as<double2>() + M, -1,
                    1.0 / P, s, Mr);
    }
    launch_axpby_op(W, MP, x, GH.as<double2>(), nullptr, out, s);
    // the wall rows reuse SIG computed above
    if (!fused) nsum(pwalls, wwalls, WR.as<double2>());
    launch_combine_walls(W, lat.M1 * lat.M1, WR.as<double2>(), CY.as<double2>(), s);
    apply_qpinv();
    if (!b.trans()) {
      launch_bapply(W, P, M, lat.p, Bvals.as<double2>(), XI.as<double2>(), NQmax, out, s, M);
    } else {
      launch_bapply(W, P, M, lat.p, Bvals_v.as<double2>(), XI.as<double2>(), NQmax, out, s, Mr);
      launch_bapply(W, P, M, lat.p, Bvals.as<double2>(), XI.as<double2>(), NQmax, out + M, s, Mr);
    }
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


}  // namespace mfs
