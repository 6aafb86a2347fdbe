// Serving loop: continuous batching of incident-wave solves (Sec. 4.2) on a
// resident factored operator.
//
// Two host threads, two HIP streams:
//   * the admission thread takes waiting requests as slots and the memory
//     budget allow (up to admit_batch at once), fills and factors their Q
//     (the per-incidence part of Sec. 4.2), computes their right-hand sides
//     and writes the first Krylov vector into the slot's basis;
//   * the iteration thread runs lockstep GMRES over the slot pool: per
//     iteration one batched application of the operator of eq. (iter) to the
//     current vector of every iterating slot, CGS2 against each slot's own
//     basis (bases are zeroed on admission, so slots at different iteration
//     counts share the launches), Givens rotations on the host; slots whose
//     factorisation finished join at the next iteration, converged slots are
//     recovered and leave.
// Every slot's arithmetic reads only its own data, so a request's result
// does not depend on the others in flight.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>

#include "solver.hpp"

namespace mfs {
namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  uint64_t ticket = 0;
  mfs_wave wave{};
  Clock::time_point t_submit;
};

struct Finished {
  mfs_status st = MFS_OK;
  int iters = 0, q_rank = 0, nq_cols = 0;
  double resid = 0.0, eps_flux = 0.0, latency_ms = 0.0;
  std::vector<int32_t> m, n;
  std::vector<mfs_c128> kz, a, b, field;
};

struct Slot {
  int state = 0;   // 0 free, 1 admitting, 2 factored (joins at the next iteration), 3 iterating
  Request req;
  MatDesc qd{};   // Q^+ factors in the slot's own storage (slot_fac)
  cplx al = 1.0, be = 1.0;
  double kv[3] = {0.0, 0.0, 0.0};
  std::vector<RBOrder> orders;
  int qrank = 0;
  bool q_converged = true;   // the Jacobi SVD of the wave's Q (if one ran) converged
  // GMRES
  int j = 0;
  double beta0 = 0.0, resid = 0.0;
  std::vector<cplx> H, g, sn;
  std::vector<double> cs;
};

}  // namespace
}  // namespace mfs

struct mfs_server {
  mfs_ctx *ctx = nullptr;
  const mfs_op *op = nullptr;
  int body = 0;
  mfs_lattice lat{};
  mfs_server_config cfg{};
  std::vector<double> targets;
  hipStream_t s_it = nullptr, s_ad = nullptr;
  std::unique_ptr<mfs::Solver> it;      // the slot pool: plans, near field, B~, bases, work
  mfs::DevBuf qd, zero;                 // Q^+ descriptors of the slots; zeros for empty ones
  // every slot's Q^+ factors, U (rows x NQb, leading dimension ldq) then W
  // (round_up(NQb, 16) x NQb), and the slots' kept ranks: allocated with the
  // server, so the factors of the waves in flight never add memory
  mfs::DevBuf slot_fac, slot_rank;
  size_t slot_stride = 0;
  std::vector<mfs::MatDesc> hq;
  std::vector<mfs::Slot> slots;
  std::mutex mu;
  std::condition_variable cv_ad, cv_it;
  std::deque<mfs::Request> pending;
  std::map<uint64_t, mfs::Finished> done;
  uint64_t next = 1;
  bool stop = false, failed = false;
  std::string fail_msg;
  int admitting = 0;
  // memory: fixed_bytes (stored near field, Krylov bases, the slots' factor
  // storage) is held for the server's life; an admission group of g waves
  // holds g * wave_work_bytes more while it is factored
  double wave_work_bytes = 0.0, fixed_bytes = 0.0;
  std::thread t_ad, t_it;
};

namespace mfs {
namespace {

MatDesc empty_desc(mfs_server *sv) {
  MatDesc e{};
  e.m = 0;
  e.n = sv->it->NQmax;
  e.lda = 1;
  e.ldg = 1;
  e.u = sv->zero.as<double2>();
  e.w = sv->zero.as<double2>();
  e.rank = reinterpret_cast<int *>(sv->zero.p);
  return e;
}

void fail(mfs_server *sv, const std::string &msg) {
  std::lock_guard<std::mutex> lk(sv->mu);
  sv->failed = true;
  sv->fail_msg = msg;
  sv->cv_ad.notify_all();
  sv->cv_it.notify_all();
}

// waves the admission thread may take now (mu held)
int admissible(mfs_server *sv) {
  int freeslots = 0;
  for (auto &s : sv->slots)
    if (s.state == 0) ++freeslots;
  int g = std::min({(int)sv->pending.size(), freeslots, sv->cfg.admit_batch});
  while (g > 0 && sv->fixed_bytes + g * sv->wave_work_bytes > (double)sv->cfg.hbm_budget) --g;
  return g;
}

void wave_host_data(const BodyData &b, const mfs_lattice &lat, const mfs_wave &w, cplx &al, cplx &be, double kv[3],
                    std::vector<RBOrder> &orders) {
  MFS_REQUIRE(std::isfinite(w.theta) && std::isfinite(w.phi), "non-finite incidence");
  kv[0] = b.k * std::sin(w.theta) * std::cos(w.phi);
  kv[1] = b.k * std::sin(w.theta) * std::sin(w.phi);
  kv[2] = -b.k * std::cos(w.theta);
  al = std::exp(cplx(0.0, kv[0] * lat.ex));
  be = std::exp(cplx(0.0, kv[1] * lat.ey));
  rb_orders(b.k, kv, lat, orders);
  bool has00 = false;
  for (auto &o : orders) has00 |= (o.m == 0 && o.n == 0);
  MFS_REQUIRE(has00, "Rayleigh-Bloch cutoff excludes the (0,0) order");
}

void admit(mfs_server *sv, const std::vector<int> &ks, const std::vector<Request> &reqs) {
  BodyData &b = body_of(sv->op, sv->body);
  const int g = (int)ks.size();
  hipStream_t s = sv->s_ad;
  std::unique_ptr<Solver> As(new Solver(sv->op, b, sv->lat, g, sv->cfg.maxit, s));
  Solver &A = *As;
  A.al.resize(g);
  A.be.resize(g);
  A.kv.resize(3 * g);
  A.orders.resize(g);
  for (int i = 0; i < g; ++i)
    wave_host_data(b, sv->lat, reqs[i].wave, A.al[i], A.be[i], &A.kv[3 * i], A.orders[i]);
  A.setup_periodizer(sv->cfg.rel_cutoff);
  MFS_REQUIRE(A.NQmax <= sv->it->NQmax, "server: Q wider than the pool's bound");
  A.Q.clear();
  A.gp.release_work();
  // the factors move into the slots' own storage; the group's arenas go
  // when A does, at the end of this call
  std::vector<MatDesc> sq(g);
  for (int i = 0; i < g; ++i) {
    const MatDesc &f = A.gp.h_fin[i];
    const int kept = A.qrank[i];
    char *base = static_cast<char *>(sv->slot_fac.p) + (size_t)ks[i] * sv->slot_stride;
    MatDesc d = f;
    d.u = reinterpret_cast<double2 *>(base);
    d.w = reinterpret_cast<double2 *>(base + (size_t)f.lda * sv->it->NQmax * sizeof(double2));
    d.rank = sv->slot_rank.as<int>() + ks[i];
    MFS_REQUIRE(f.lda == sv->it->ldq && f.ldg <= round_up(sv->it->NQmax, 16) && kept <= sv->it->NQmax,
                "server: factors larger than a slot's storage");
    if (kept > 0) {
      HIP_CHECK(hipMemcpyAsync(d.u, f.u, (size_t)f.lda * kept * sizeof(double2), hipMemcpyDeviceToDevice, s));
      HIP_CHECK(hipMemcpyAsync(d.w, f.w, (size_t)f.ldg * kept * sizeof(double2), hipMemcpyDeviceToDevice, s));
    }
    HIP_CHECK(hipMemcpyAsync(d.rank, &A.qrank[i], sizeof(int), hipMemcpyHostToDevice, s));
    sq[i] = d;
  }
  // right-hand sides and the first Krylov vector of every wave in its slot
  Solver &P = *sv->it;
  const int MP = P.MP;
  const size_t ldw = (size_t)(sv->cfg.maxit + 1) * MP;
  DevBuf kvd((size_t)3 * g * sizeof(double)), FH((size_t)g * MP * sizeof(double2)),
      hn((size_t)g * sizeof(double2)), sc((size_t)g * sizeof(double));
  upload(kvd.p, A.kv.data(), 3 * g * sizeof(double), s);
  launch_rhs(b, g, kvd.as<double>(), FH.as<double2>(), s);
  launch_dots(g, 1, MP, FH.as<double2>(), (size_t)MP, 0, FH.as<double2>(), hn.as<double2>(), s);
  std::vector<double2> h(g);
  HIP_CHECK(hipMemcpyAsync(h.data(), hn.p, g * sizeof(double2), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipStreamSynchronize(s));
  std::vector<double> beta0(g), scale(g);
  for (int i = 0; i < g; ++i) {
    beta0[i] = std::sqrt(std::max(h[i].x, 0.0));
    scale[i] = beta0[i] > 0 ? 1.0 / beta0[i] : 0.0;
  }
  upload(sc.p, scale.data(), g * sizeof(double), s);
  for (int i = 0; i < g; ++i) {
    double2 *Vk = P.V.as<double2>() + (size_t)ks[i] * ldw;
    launch_zero(Vk, (long)ldw, s);
    launch_scale(1, MP, FH.as<double2>() + (size_t)i * MP, MP, Vk, ldw, sc.as<double>() + i, s);
  }
  HIP_CHECK(hipStreamSynchronize(s));
  std::lock_guard<std::mutex> lk(sv->mu);
  for (int i = 0; i < g; ++i) {
    Slot &sl = sv->slots[ks[i]];
    sl.qd = sq[i];
    sl.al = A.al[i];
    sl.be = A.be[i];
    for (int c = 0; c < 3; ++c) sl.kv[c] = A.kv[3 * i + c];
    sl.orders = A.orders[i];
    sl.qrank = A.qrank[i];
    sl.q_converged = A.gp.jacobi_unconverged == 0;
    sl.j = 0;
    sl.beta0 = beta0[i];
    sl.resid = beta0[i] > 0 ? 1.0 : 0.0;
    const int mi = sv->cfg.maxit;
    sl.H.assign((size_t)(mi + 1) * mi, 0.0);
    sl.g.assign(mi + 1, 0.0);
    sl.g[0] = beta0[i];
    sl.cs.assign(mi, 0.0);
    sl.sn.assign(mi, 0.0);
    sl.state = 2;
  }
  sv->admitting -= g;
  sv->cv_it.notify_all();
}

void admit_loop(mfs_server *sv) {
  try {
    HIP_CHECK(hipSetDevice(sv->ctx->device));
    for (;;) {
      std::vector<int> ks;
      std::vector<Request> reqs;
      {
        std::unique_lock<std::mutex> lk(sv->mu);
        sv->cv_ad.wait(lk, [&] { return sv->stop || sv->failed || admissible(sv) > 0; });
        if (sv->stop || sv->failed) return;
        const int g = admissible(sv);
        for (int k = 0; k < (int)sv->slots.size() && (int)ks.size() < g; ++k) {
          if (sv->slots[k].state != 0) continue;
          sv->slots[k].state = 1;
          sv->slots[k].req = sv->pending.front();
          ks.push_back(k);
          reqs.push_back(sv->pending.front());
          sv->pending.pop_front();
        }
        sv->admitting += (int)ks.size();
      }
      admit(sv, ks, reqs);
    }
  } catch (const Error &e) {
    fail(sv, e.msg);
  } catch (const std::exception &e) {
    fail(sv, e.what());
  }
}

// finish slot k from its GMRES state (iteration thread; results recorded by the caller)
void solve_y(const Slot &sl, int k, int maxit, std::vector<cplx> &y) {
  y.assign(k, 0.0);
  auto Hat = [&](int i, int c) { return sl.H[(size_t)c * (maxit + 1) + i]; };
  for (int i = k - 1; i >= 0; --i) {
    cplx acc = sl.g[i];
    for (int l = i + 1; l < k; ++l) acc -= Hat(i, l) * y[l];
    y[i] = acc / Hat(i, i);
  }
}

void iter_loop(mfs_server *sv) {
  try {
    HIP_CHECK(hipSetDevice(sv->ctx->device));
    Solver &S = *sv->it;
    const int W = S.W, MP = S.MP, maxit = sv->cfg.maxit;
    const size_t ldw = (size_t)(maxit + 1) * MP;
    hipStream_t s = sv->s_it;
    double2 *V = S.V.as<double2>();
    double2 *Zb = S.Z.as<double2>();
    double2 *Hd = S.H1.as<double2>();
    double *SCd = S.SC.as<double>();
    std::vector<double2> hbuf((size_t)W * (maxit + 2) * 2);
    std::vector<double> scale(W, 0.0);
    bool descs_dirty = true;
    for (;;) {
      std::vector<int> act;
      bool joined = false;
      {
        std::unique_lock<std::mutex> lk(sv->mu);
        sv->cv_it.wait(lk, [&] {
          if (sv->stop || sv->failed) return true;
          for (auto &sl : sv->slots)
            if (sl.state >= 2) return true;
          return false;
        });
        if (sv->stop || sv->failed) return;
        for (int k = 0; k < W; ++k) {
          Slot &sl = sv->slots[k];
          if (sl.state == 2) {
            sl.state = 3;
            S.al[k] = sl.al;
            S.be[k] = sl.be;
            for (int c = 0; c < 3; ++c) S.kv[3 * k + c] = sl.kv[c];
            S.orders[k] = sl.orders;
            S.qrank[k] = sl.qrank;
            sv->hq[k] = sl.qd;
            joined = true;
          }
          if (sl.state == 3) act.push_back(k);
        }
      }
      if (joined || descs_dirty) {
        S.upload_weights();
        upload(sv->qd.p, sv->hq.data(), W * sizeof(MatDesc), s);
        descs_dirty = false;
      }
      // current vector of every iterating slot (zero elsewhere) -> operator
      launch_zero(S.XIN.as<double2>(), (long)W * MP, s);
      int jmax = 0;
      for (int k : act) {
        const Slot &sl = sv->slots[k];
        jmax = std::max(jmax, sl.j);
        HIP_CHECK(hipMemcpyAsync(S.XIN.as<double2>() + (size_t)k * MP, V + (size_t)k * ldw + (size_t)sl.j * MP,
                                 MP * sizeof(double2), hipMemcpyDeviceToDevice, s));
      }
      S.apply_op(S.XIN.as<double2>(), Zb);
      // CGS2 against each slot's basis (columns past a slot's count are zero)
      const int nv = jmax + 1;
      double2 *h1 = Hd, *h2 = Hd + (size_t)W * nv;
      launch_dots(W, nv, MP, V, ldw, MP, Zb, h1, s);
      launch_update(W, nv, MP, V, ldw, MP, Zb, h1, nv, s);
      launch_dots(W, nv, MP, V, ldw, MP, Zb, h2, s);
      launch_update(W, nv, MP, V, ldw, MP, Zb, h2, nv, s);
      double2 *hnp = h2 + (size_t)W * nv;
      launch_dots(W, 1, MP, Zb, (size_t)MP, 0, Zb, hnp, s);
      HIP_CHECK(hipMemcpyAsync(hbuf.data(), Hd, (size_t)W * (2 * nv + 1) * sizeof(double2), hipMemcpyDeviceToHost,
                               s));
      HIP_CHECK(hipStreamSynchronize(s));
      std::vector<int> fin;
      std::fill(scale.begin(), scale.end(), 0.0);
      for (int k : act) {
        Slot &sl = sv->slots[k];
        const int j = sl.j;
        auto Hat = [&](int i, int c) -> cplx & { return sl.H[(size_t)c * (maxit + 1) + i]; };
        if (sl.beta0 == 0.0) {   // zero right-hand side: zero solution
          fin.push_back(k);
          continue;
        }
        for (int i = 0; i <= j; ++i) {
          const double2 a1 = hbuf[(size_t)k * nv + i], a2 = hbuf[(size_t)W * nv + (size_t)k * nv + i];
          Hat(i, j) = cplx(a1.x + a2.x, a1.y + a2.y);
        }
        const double hnext = std::sqrt(std::max(hbuf[(size_t)2 * W * nv + k].x, 0.0));
        Hat(j + 1, j) = hnext;
        for (int i = 0; i < j; ++i) {
          const cplx a = Hat(i, j), c2 = Hat(i + 1, j);
          Hat(i, j) = sl.cs[i] * a + sl.sn[i] * c2;
          Hat(i + 1, j) = -std::conj(sl.sn[i]) * a + sl.cs[i] * c2;
        }
        const cplx a = Hat(j, j);
        const double bb = std::abs(Hat(j + 1, j));
        const double r = std::hypot(std::abs(a), bb);
        if (r == 0.0) {
          sl.cs[j] = 1.0;
          sl.sn[j] = 0.0;
        } else if (std::abs(a) == 0.0) {
          sl.cs[j] = 0.0;
          sl.sn[j] = 1.0;
          Hat(j, j) = r;
        } else {
          const cplx ph = a / std::abs(a);
          sl.cs[j] = std::abs(a) / r;
          sl.sn[j] = ph * bb / r;
          Hat(j, j) = ph * r;
        }
        Hat(j + 1, j) = 0.0;
        sl.g[j + 1] = -std::conj(sl.sn[j]) * sl.g[j];
        sl.g[j] = sl.cs[j] * sl.g[j];
        sl.resid = std::abs(sl.g[j + 1]) / sl.beta0;
        sl.j = j + 1;
        if (sl.resid <= sv->cfg.tol || hnext <= 1e-300 || sl.j >= maxit) fin.push_back(k);
        else scale[k] = 1.0 / hnext;
      }
      upload(SCd, scale.data(), W * sizeof(double), s);
      for (int k : act)
        if (scale[k] != 0.0) {
          const Slot &sl = sv->slots[k];
          launch_scale(1, MP, Zb + (size_t)k * MP, MP, V + (size_t)k * ldw + (size_t)sl.j * MP, ldw, SCd + k, s);
        }
      if (fin.empty()) continue;
      // recovery of the finished slots (the others ride along with zero coefficients)
      std::vector<std::vector<cplx>> y(W);
      std::vector<int> iters(W, 0);
      for (int k : fin) {
        const Slot &sl = sv->slots[k];
        iters[k] = sl.beta0 == 0.0 ? 0 : sl.j;
        solve_y(sl, iters[k], maxit, y[k]);
      }
      std::vector<double2> xi, uf;
      const int nt = sv->cfg.ntargets;
      S.recover(V, ldw, y, iters, sv->targets.data(), nt, sv->cfg.q_field, xi, uf);
      const auto t_done = Clock::now();
      std::vector<std::pair<uint64_t, Finished>> out;
      for (int k : fin) {
        const Slot &sl = sv->slots[k];
        Finished f;
        const int no = (int)sl.orders.size();
        f.m.resize(no);
        f.n.resize(no);
        f.kz.resize(no);
        f.a.resize(no);
        f.b.resize(no);
        f.field.resize(nt);
        mfs_result r{};
        r.m = f.m.data();
        r.n = f.n.data();
        r.kz = f.kz.data();
        r.a = f.a.data();
        r.b = f.b.data();
        r.cap_orders = no;
        S.amplitudes(k, xi.data() + (size_t)k * S.NQmax, r);
        for (int t = 0; t < nt; ++t) f.field[t] = mfs_c128{uf[(size_t)k * nt + t].x, uf[(size_t)k * nt + t].y};
        f.iters = iters[k];
        f.resid = sl.resid;
        f.eps_flux = r.eps_flux;
        f.q_rank = r.q_rank;
        f.nq_cols = r.nq_cols;
        f.st = ((sl.resid <= sv->cfg.tol || sl.beta0 == 0.0) && sl.q_converged) ? MFS_OK : MFS_ENOTCONV;
        f.latency_ms = std::chrono::duration<double, std::milli>(t_done - sl.req.t_submit).count();
        out.emplace_back(sl.req.ticket, std::move(f));
      }
      {
        std::lock_guard<std::mutex> lk(sv->mu);
        for (auto &p : out) sv->done[p.first] = std::move(p.second);
        for (int k : fin) {
          sv->slots[k].state = 0;
          sv->hq[k] = empty_desc(sv);
        }
        descs_dirty = true;
        sv->cv_ad.notify_all();
      }
    }
  } catch (const Error &e) {
    fail(sv, e.msg);
  } catch (const std::exception &e) {
    fail(sv, e.what());
  }
}

}  // namespace
}  // namespace mfs

using namespace mfs;

extern "C" {

mfs_status mfs_server_create(mfs_ctx *ctx, const mfs_op *op, int32_t body, const mfs_lattice *lat,
                             const mfs_server_config *cfg, mfs_server **out) {
  mfs_server *sv = nullptr;
  try {
    MFS_REQUIRE(ctx && op && lat && cfg && out, "null pointer");
    BodyData &b = body_of(op, body);
    if (!op->factored) MFS_THROW(MFS_ESTATE, "mfs_factor_modes has not run");
    MFS_REQUIRE(cfg->slots >= 1 && cfg->slots <= 16, "1 <= slots <= 16");
    MFS_REQUIRE(cfg->admit_batch >= 1 && cfg->admit_batch <= cfg->slots, "1 <= admit_batch <= slots");
    MFS_REQUIRE(cfg->queue_cap >= 1, "queue_cap >= 1");
    MFS_REQUIRE(cfg->tol > 0 && cfg->maxit >= 1 && cfg->maxit <= 2000, "bad GMRES tolerance or maxit");
    MFS_REQUIRE(cfg->rel_cutoff >= 0 && cfg->rel_cutoff < 1, "bad cutoff");
    MFS_REQUIRE(lat->ex > 0 && lat->ey > 0 && lat->z0 > 0 && lat->N0 > 0, "bad lattice");
    MFS_REQUIRE(lat->p >= 1 && lat->p <= 96, "1 <= p <= 96");
    MFS_REQUIRE(lat->M1 >= 2 && lat->M1 % 2 == 0, "M1 must be even and >= 2");
    MFS_REQUIRE(cfg->ntargets >= 0 && (cfg->ntargets == 0 || (cfg->targets && cfg->q_field >= b.P)),
                "bad targets");
    HIP_CHECK(hipSetDevice(ctx->device));
    sv = new mfs_server();
    sv->ctx = ctx;
    sv->op = op;
    sv->body = body;
    sv->lat = *lat;
    sv->cfg = *cfg;
    if (cfg->ntargets > 0) sv->targets.assign(cfg->targets, cfg->targets + (size_t)3 * cfg->ntargets);
    sv->cfg.targets = nullptr;
    HIP_CHECK(hipStreamCreate(&sv->s_it));
    HIP_CHECK(hipStreamCreate(&sv->s_ad));
    const int W = cfg->slots;
    // widest Q of any incidence: (p+1)^2 harmonics + 2 x the Rayleigh-Bloch
    // orders, at most the lattice points of a disc of radius pi N0
    const int NH = (lat->p + 1) * (lat->p + 1);
    const int ob = ((int)std::ceil(lat->N0 * lat->ex) + 3) * ((int)std::ceil(lat->N0 * lat->ey) + 3);
    const int NQb = NH + 2 * ob;
    const double rows = 8.0 * lat->M1 * lat->M1;
    sv->wave_work_bytes = (4.0 * rows * NQb + 8.0 * (double)NQb * NQb) * sizeof(double2);
    const double basis = (double)W * (cfg->maxit + 1) * b.P * b.rows * sizeof(double2);
    const int ldq = round_up((int)rows, 16);
    sv->slot_stride = ((size_t)ldq * NQb + (size_t)round_up(NQb, 16) * NQb) * sizeof(double2);
    const double need = basis + (double)W * sv->slot_stride + sv->wave_work_bytes;
    if ((double)cfg->hbm_budget < need)
      MFS_THROW(MFS_ENOMEM, "server: hbm_budget below the slots' storage and one wave's factorisation");
    size_t in0 = 0, in1 = 0;
    pool_stats(ctx->device, &in0, nullptr, nullptr);
    sv->it.reset(new Solver(op, b, *lat, W, cfg->maxit, sv->s_it));
    Solver &S = *sv->it;
    S.NQmax = NQb;
    S.al.assign(W, 1.0);
    S.be.assign(W, 1.0);
    S.kv.assign(3 * W, 0.0);
    S.orders.assign(W, {});
    S.qrank.assign(W, 0);
    S.near_limit = (size_t)std::max(0.0, (double)cfg->hbm_budget - need);
    S.setup_bvals();
    S.setup_sums();
    S.time_nsum = false;
    sv->slot_fac.alloc((size_t)W * sv->slot_stride);
    sv->slot_rank.alloc((size_t)W * sizeof(int));
    sv->zero.alloc(4096);
    HIP_CHECK(hipMemsetAsync(sv->zero.p, 0, 4096, sv->s_it));
    sv->qd.alloc((size_t)W * sizeof(MatDesc));
    sv->hq.assign(W, empty_desc(sv));
    S.qdesc = sv->qd.as<MatDesc>();
    upload(sv->qd.p, sv->hq.data(), W * sizeof(MatDesc), sv->s_it);
    HIP_CHECK(hipStreamSynchronize(sv->s_it));
    // held for the server's life: what the set-up above allocated (measured;
    // at least the bases, the slots' storage and the stored near field), and
    // the buffers of one recovery of `slots` waves (the iteration thread
    // forms their amplitudes and fields: eta, the q_field-node strengths and
    // the target sums with up to 51 partial slices)
    pool_stats(ctx->device, &in1, nullptr, nullptr);
    const double listed = basis + (double)W * sv->slot_stride + (double)S.psurf.dense_bytes +
                          (double)S.pwalls.dense_bytes;
    const double ntp = (double)round_up(std::max(cfg->ntargets, 1), 64);
    const double recover = 16.0 * W * ((double)b.P * b.rows + (double)cfg->q_field * b.N + 51.0 * ntp) +
                           24.0 * cfg->q_field * b.N;
    sv->fixed_bytes = std::max(in1 > in0 ? (double)(in1 - in0) : 0.0, listed) + recover;
    if (sv->fixed_bytes + sv->wave_work_bytes > (double)cfg->hbm_budget)
      MFS_THROW(MFS_ENOMEM, "server: hbm_budget below the resident storage and one wave's factorisation");
    sv->slots.resize(W);
    sv->t_ad = std::thread(admit_loop, sv);
    sv->t_it = std::thread(iter_loop, sv);
    *out = sv;
    return MFS_OK;
  } catch (const Error &e) {
    set_error(e.msg);
    if (sv) mfs_server_destroy(sv);
    return e.st;
  } catch (const std::exception &e) {
    set_error(e.what());
    if (sv) mfs_server_destroy(sv);
    return MFS_ENOMEM;
  }
}

mfs_status mfs_server_submit(mfs_server *sv, const mfs_wave *wave, uint64_t *ticket) {
  if (!sv || !wave || !ticket) {
    set_error("null pointer");
    return MFS_EINVAL;
  }
  if (!std::isfinite(wave->theta) || !std::isfinite(wave->phi)) {
    set_error("non-finite incidence");
    return MFS_EINVAL;
  }
  std::lock_guard<std::mutex> lk(sv->mu);
  if (sv->failed) {
    set_error(sv->fail_msg);
    return MFS_EDEVICE;
  }
  if ((int)sv->pending.size() >= sv->cfg.queue_cap) {
    set_error("server queue full");
    return MFS_EBUSY;
  }
  Request r;
  r.ticket = sv->next++;
  r.wave = *wave;
  r.t_submit = Clock::now();
  sv->pending.push_back(r);
  *ticket = r.ticket;
  sv->cv_ad.notify_all();
  return MFS_OK;
}

mfs_status mfs_server_poll(mfs_server *sv, uint64_t ticket, mfs_result *res, double *latency_ms) {
  if (!sv || !res) {
    set_error("null pointer");
    return MFS_EINVAL;
  }
  std::lock_guard<std::mutex> lk(sv->mu);
  auto itd = sv->done.find(ticket);
  if (itd == sv->done.end()) {
    if (sv->failed) {
      set_error(sv->fail_msg);
      return MFS_EDEVICE;
    }
    bool known = ticket >= 1 && ticket < sv->next;
    bool waiting = false;
    for (auto &r : sv->pending) waiting |= r.ticket == ticket;
    for (auto &sl : sv->slots) waiting |= (sl.state != 0 && sl.req.ticket == ticket);
    if (known && waiting) return MFS_EBUSY;
    set_error("unknown or already collected ticket");
    return MFS_EINVAL;
  }
  const Finished &f = itd->second;
  const int no = (int)f.m.size();
  res->norders = no;
  if (res->cap_orders < no) {
    set_error("result cap_orders too small (norders set)");
    return MFS_EINVAL;
  }
  for (int i = 0; i < no; ++i) {
    if (res->m) res->m[i] = f.m[i];
    if (res->n) res->n[i] = f.n[i];
    if (res->kz) res->kz[i] = f.kz[i];
    if (res->a) res->a[i] = f.a[i];
    if (res->b) res->b[i] = f.b[i];
  }
  if (res->field)
    for (size_t t = 0; t < f.field.size(); ++t) res->field[t] = f.field[t];
  res->iters = f.iters;
  res->resid = f.resid;
  res->eps_flux = f.eps_flux;
  res->q_rank = f.q_rank;
  res->nq_cols = f.nq_cols;
  if (latency_ms) *latency_ms = f.latency_ms;
  const mfs_status st = f.st;
  sv->done.erase(itd);
  if (st == MFS_ENOTCONV) set_error("GMRES reached maxit before the tolerance");
  return st;
}

mfs_status mfs_server_stats(mfs_server *sv, int32_t *pending, int32_t *admitting, int32_t *iterating,
                            int32_t *finished) {
  if (!sv) {
    set_error("null pointer");
    return MFS_EINVAL;
  }
  std::lock_guard<std::mutex> lk(sv->mu);
  int it = 0;
  for (auto &sl : sv->slots) it += sl.state >= 2;
  if (pending) *pending = (int32_t)sv->pending.size();
  if (admitting) *admitting = sv->admitting;
  if (iterating) *iterating = it;
  if (finished) *finished = (int32_t)sv->done.size();
  if (sv->failed) {
    set_error(sv->fail_msg);
    return MFS_EDEVICE;
  }
  return MFS_OK;
}

void mfs_server_destroy(mfs_server *sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
    sv->cv_ad.notify_all();
    sv->cv_it.notify_all();
  }
  if (sv->t_ad.joinable()) sv->t_ad.join();
  if (sv->t_it.joinable()) sv->t_it.join();
  (void)hipSetDevice(sv->ctx ? sv->ctx->device : 0);
  if (sv->s_ad) (void)hipStreamSynchronize(sv->s_ad);
  if (sv->s_it) (void)hipStreamSynchronize(sv->s_it);
  sv->slots.clear();
  sv->it.reset();
  sv->qd.release();
  sv->zero.release();
  if (sv->s_ad) (void)hipStreamDestroy(sv->s_ad);
  if (sv->s_it) (void)hipStreamDestroy(sv->s_it);
  delete sv;
}

}  // extern "C"
