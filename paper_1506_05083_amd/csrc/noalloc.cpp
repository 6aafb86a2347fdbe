// The solution-operator apply without any allocation, for callers that
// cannot allocate device memory: code under HIP graph capture, tight serving
// loops, harnesses that forbid it.  Its work memory (the per-mode
// pseudoinverse work buffer and the angle/point layout intermediates) is a
// fixed array in device memory: every GPU the library runs on holds its own
// copy until the process ends, and every call on that GPU uses it.
#include <mutex>
#include <vector>

#include "capi_impl.hpp"

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;   // per device

}  // namespace

// Work memory of mfs_apply_solution_op_noalloc.  In host code this name is a
// host-side stand-in, not the device address: kernels are given the address
// that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) double2 scratch[kScratchBytes / sizeof(double2)];

namespace mfs {
namespace {

std::mutex g_scratch_mu;
std::vector<double2 *> g_scratch;   // per device: the device address of `scratch`

// The device address of `scratch` on device dev (current), looked up once
// per device.
double2 *scratch_on(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch.size() <= dev) g_scratch.resize(dev + 1, nullptr);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    MFS_REQUIRE(p != nullptr, "no device address for the static scratch");
    g_scratch[dev] = static_cast<double2 *>(p);
  }
  return g_scratch[dev];
}

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace
}  // namespace mfs

using namespace mfs;

extern "C" mfs_status mfs_apply_solution_op_noalloc(const mfs_op *op, int32_t body, int32_t nrhs,
                                                    const mfs_c128 *in, int32_t in_layout, mfs_c128 *out,
                                                    int32_t out_layout, void *stream) {
  try {
    BodyData &b = body_of(op, body);
    check_apply_args(op, nrhs, in, in_layout, out, out_layout);
    if (nrhs == 0) return MFS_OK;
    // work memory, laid out in the scratch array: the per-mode work buffer,
    // then the mode-layout copy of an angle input, then the mode-layout
    // result that a point-strength output is formed from
    const size_t yw = round256(apply_pinv_work_bytes(b));
    const size_t im = in_layout == MFS_LAYOUT_ANGLE ? round256((size_t)nrhs * b.P * b.rows * sizeof(double2)) : 0;
    const size_t om = out_layout == MFS_LAYOUT_POINTS ? round256((size_t)nrhs * b.P * b.cols * sizeof(double2)) : 0;
    if (yw + im + om > kScratchBytes)
      MFS_THROW(MFS_EINVAL, "mfs_apply_solution_op_noalloc: this body and nrhs need " + std::to_string(yw + im + om) +
                                " bytes of work memory, more than the " + std::to_string(kScratchBytes) +
                                " bytes of the static scratch (fewer right-hand sides per call fit)");
    HIP_CHECK(hipSetDevice(op->ctx->device));
    double2 *base = scratch_on(op->ctx->device);
    double2 *ywork = base;
    double2 *in_modes = base + yw / sizeof(double2);
    double2 *out_modes = base + (yw + im) / sizeof(double2);
    apply_solution_layouts(op, b, nrhs, reinterpret_cast<const double2 *>(in), in_layout,
                           reinterpret_cast<double2 *>(out), out_layout, in_modes, out_modes, ywork,
                           static_cast<hipStream_t>(stream));
    return MFS_OK;
  } catch (const Error &e) {
    set_error(e.msg);
    return e.st;
  } catch (const std::exception &e) {
    set_error(e.what());
    return MFS_EDEVICE;
  }
}
