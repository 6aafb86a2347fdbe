// Shared helpers of libmfs: complex double arithmetic on double2, error
// reporting across the C ABI, and small device utilities (wave64 reductions).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/mfs.h"

namespace mfs {

// ------------------------------------------------------------ errors
void set_error(const std::string &msg);
const std::string &get_error();

struct Error {
  mfs_status st;
  std::string msg;
};

#define MFS_THROW(code, msg_expr)                                                 \
  do {                                                                            \
    throw ::mfs::Error{(code), std::string(msg_expr)};                            \
  } while (0)

#define HIP_CHECK(expr)                                                           \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess)                                                         \
      throw ::mfs::Error{MFS_EDEVICE, std::string(#expr) + ": " +                 \
                                          hipGetErrorString(e_)};                 \
  } while (0)

#define MFS_REQUIRE(cond, msg_expr)                                               \
  do {                                                                            \
    if (!(cond)) MFS_THROW(MFS_EINVAL, msg_expr);                                 \
  } while (0)

// --------------------------------------------------------- complex
__host__ __device__ inline double2 cz(double re, double im = 0.0) {
  double2 r;
  r.x = re;
  r.y = im;
  return r;
}
__host__ __device__ inline double2 cadd(double2 a, double2 b) { return cz(a.x + b.x, a.y + b.y); }
__host__ __device__ inline double2 csub(double2 a, double2 b) { return cz(a.x - b.x, a.y - b.y); }
__host__ __device__ inline double2 cmul(double2 a, double2 b) {
  return cz(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__host__ __device__ inline double2 cmulc(double2 a, double2 b) {
  return cz(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__host__ __device__ inline double2 cscale(double2 a, double s) { return cz(a.x * s, a.y * s); }
__host__ __device__ inline double2 cconj(double2 a) { return cz(a.x, -a.y); }
__host__ __device__ inline double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
// acc += a * b
__host__ __device__ inline void cfma(double2 &acc, double2 a, double2 b) {
  acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
  acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
}
// acc += conj(a) * b
__host__ __device__ inline void cfmac(double2 &acc, double2 a, double2 b) {
  acc.x = fma(a.x, b.x, fma(a.y, b.y, acc.x));
  acc.y = fma(a.x, b.y, fma(-a.y, b.x, acc.y));
}

// ----------------------------------------------------- reductions
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline double2 wave_sum(double2 v) {
  v.x = wave_sum(v.x);
  v.y = wave_sum(v.y);
  return v;
}
__device__ inline double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

inline int cdiv(int a, int b) { return (a + b - 1) / b; }
inline int round_up(int a, int b) { return cdiv(a, b) * b; }

constexpr double kPi = 3.14159265358979323846;

}  // namespace mfs
