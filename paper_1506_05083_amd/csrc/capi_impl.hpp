// Objects behind the opaque C handles, and helpers shared by capi.cpp and
// solve.cpp.
#pragma once

#include <complex>
#include <memory>
#include <vector>

#include "geometry.hpp"
#include "gpinv.hpp"
#include "internal.hpp"

struct mfs_ctx {
  int device = 0;
};

struct mfs_op {
  mfs_ctx *ctx = nullptr;
  hipStream_t stream = nullptr;
  std::vector<std::unique_ptr<mfs::BodyData>> bodies;
  bool factored = false;
  double cutoff = 1e-10;
  std::vector<std::unique_ptr<mfs::GradedPinv>> gps;   // factors of the distinct blocks, by chunk
  mfs::DevBuf work;
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
  double ms_fill = 0.0, ms_qr = 0.0, ms_svd = 0.0;
  uint64_t near_budget = UINT64_MAX;   // dense near-field storage limit (bytes)
  ~mfs_op() {
    for (auto &e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

namespace mfs {

void upload(void *dst, const void *src, size_t bytes, hipStream_t s);
void source_points(const BodyData &b, int qs, DevBuf &out, hipStream_t s);
// the same for a given source set (the exterior sources of a transmission body)
void source_points_of(const BodyData &b, const std::vector<double> &srho, const std::vector<double> &sz, int qs,
                      DevBuf &out, hipStream_t s);
void build_plan(NsumPlan &plan, const std::vector<NsumGroup> &groups,
                const std::vector<std::vector<double>> &tg, hipStream_t s);
void surface_plan(const BodyData &b, NsumPlan &plan, hipStream_t s);
void walls_plan(const mfs_lattice &lat, int P, int N, NsumPlan &plan, hipStream_t s);
void user_plan(const double *user, int nuser, int want, bool nine, NsumPlan &plan, hipStream_t s);
void walls_weights(const std::vector<std::complex<double>> &al, const std::vector<std::complex<double>> &be,
                   const NsumPlan &plan, std::vector<double2> &w);
void image_weights(const std::vector<std::complex<double>> &al, const std::vector<std::complex<double>> &be,
                   const NsumPlan &plan, std::vector<double2> &w);
BodyData &body_of(const mfs_op *op, int body);
double2 *op_workspace(const mfs_op *op, size_t bytes);
// c = A0^+ x for nrhs right-hand sides in mode layout (chunks of 16); yw is
// a work buffer of apply_pinv_work_bytes(b) bytes (null: the operator's own)
void apply_pinv_body(const mfs_op *op, const BodyData &b, int nrhs, const double2 *x, double2 *out,
                     hipStream_t s, double2 *yw = nullptr);
size_t apply_pinv_work_bytes(const BodyData &b);
// The solution-operator apply with its input and output layouts (MFS_LAYOUT_*):
// an ANGLE input goes through the forward angle DFT into in_modes
// ([nrhs][P][rows]), a POINTS output is formed from out_modes
// ([nrhs][P][cols]) by the inverse DFT; yw as for apply_pinv_body.  The
// buffers are the caller's (the library's cache, or the no-allocation entry
// point's static scratch).
void apply_solution_layouts(const mfs_op *op, const BodyData &b, int nrhs, const double2 *in, int in_layout,
                            double2 *out, int out_layout, double2 *in_modes, double2 *out_modes, double2 *yw,
                            hipStream_t s);
void check_apply_args(const mfs_op *op, int nrhs, const void *in, int in_layout, const void *out, int out_layout);
void launch_zero(double2 *p, long n, hipStream_t s);
void launch_scale(int nw, int n, const double2 *src, size_t lds, double2 *dst, size_t ldd,
                  const double *sdev, hipStream_t s);
// the same into dst and dst2 (ld2 apart per wave) at once
void launch_scale2(int nw, int n, const double2 *src, size_t lds, double2 *dst, size_t ldd, double2 *dst2,
                   size_t ld2, const double *sdev, hipStream_t s);

}  // namespace mfs
