// Truncated pseudoinverse of graded matrices (see gpinv.hip).
#pragma once

#include <vector>

#include "internal.hpp"

namespace mfs {

struct GradedPinv {
  DevBuf d_in, d_qc, d_rq, d_rqu, d_lq, d_fin, perm, piv, small;
  DevBuf colscale;   // [W][nmax] 1 / column norm of each kept column (equilibrated factorisations)
  // one allocation per kind for all matrices of the batch (per-matrix pieces
  // at aligned offsets): the QR'd copies and their tau, T and U, the pivoted
  // triangles, the LQ/Jacobi factors, and W
  DevBuf qc_a, qc_fac, rq_a, rq_fac, lq_a, lq_fac, fin_w;
  std::vector<MatDesc> h_qc, h_rq, h_rqu, h_lq, h_fin;
  std::vector<double> maxcol;
  std::vector<int> cols, rows, kept;
  hipEvent_t ev_qr_done = nullptr;   // if set, recorded after the unpivoted blocked QR
  bool pivoted = false;              // the triangle went through the pivoted QR
  bool direct = false;               // every singular value kept: U = Q_1, W = D P R^{-1} (no SVD)
  bool reflect = false;              // direct, with U = Q_1 applied from the QR's reflectors (d_qc) instead of formed
  bool cod = false;                  // truncated complete orthogonal decomposition in place of the SVD
  int qr_nb = kQRNB;                 // panel width of the QR of the ordered columns
  double jacobi_ms = 0.0;            // Jacobi sweeps: time, launches, algorithmic bytes and flops
  int jacobi_launches = 0;
  double jacobi_bytes = 0.0;
  double jacobi_flops = 0.0;
  int jacobi_unconverged = 0;        // matrices whose Jacobi reached the sweep cap
  // the unpivoted blocked QR of the ordered columns: time (HIP events) and
  // algorithmic flops, sum over matrices of 8 m n^2 - 8 n^3 / 3
  double qr_ms = 0.0, qr_flops = 0.0;
  // everything after that QR (triangle inverse or pivoted QR, LQ, Jacobi, and
  // the explicit factors U and W), HIP events
  double post_ms = 0.0;
  // descriptors for launch_pinv_apply (mode 1): u (m x kept), w (n x kept)
  const MatDesc *apply_descs() const { return d_fin.as<MatDesc>(); }
  // free the factorisation's work, keeping what the apply reads (U in
  // qc_fac, W in fin_w, the kept ranks in small)
  void release_work() {
    d_in.release(); d_rq.release(); d_rqu.release(); d_lq.release();
    perm.release(); piv.release(); colscale.release();
    rq_a.release(); rq_fac.release(); lq_a.release(); lq_fac.release();
    if (!reflect) {
      d_qc.release();
      qc_a.release();
    }
  }
  // the QR'd matrices whose reflectors stand for U (reflect)
  const MatDesc *qr_descs() const { return d_qc.as<MatDesc>(); }
  // singular values of every matrix, [W][ldo] (descending, zero past n);
  // before release_work.  Blocking.
  void singular_values(int ldo, std::vector<double> &out, hipStream_t s) const;
};

// in[w]: matrix w (a, m, n, lda) only.  Fills g; blocking.  The
// column-pivoted QR of the triangle is taken before the LQ when the widest
// kept triangle has at least pivot_min_cols columns (0: always); below that
// the norm ordering alone preconditions Jacobi.
// equilibrate: factor A D instead of A, D scaling every kept column to unit
// norm, so that the relative cutoff judges linear dependence rather than
// column size; W then holds D V S^+ and the pseudoinverse is D (A D)^+.
// keep_reflectors: when every singular value is kept (the direct form), U =
// Q_1 is not formed; the QR's reflectors stay for launch_qh_apply (g.reflect).
void graded_pinv(GradedPinv &g, const std::vector<MatDesc> &in, double rel_cutoff, int pivot_min_cols,
                 hipStream_t s, bool equilibrate = false, bool keep_reflectors = false);

// Widest periodizer triangle factored without the pivoted QR (measured:
// 1257 columns at k = 10 gain nothing from it, 9701 at k = 2 pi 13 gain 30%).
constexpr int kQPivotMinCols = 2048;

}  // namespace mfs
