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

// Stage progress on stderr when the environment sets MFS_PROGRESS (long
// solves report what they are doing; printf-style, one line, flushed).
void progress(const char *fmt, ...);

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

// cond ? a : b component by component (a select of the whole struct can be
// lowered through private memory)
__host__ __device__ inline double2 csel(bool cond, double2 a, double2 b) {
  return cz(cond ? a.x : b.x, cond ? a.y : b.y);
}

// p[i] if ok, else 0.  The load itself is unconditional (index 0 when !ok,
// so p must point at valid memory) and its bits are masked, not selected, so
// that the compiler cannot move it under a branch: a run of these is issued
// back to back instead of one branch and one wait per element.
__device__ inline double2 ld_or0(const double2 *p, size_t i, bool ok) {
  const double2 v = p[ok ? i : 0];
  const long long m = ok ? -1LL : 0LL;
  return cz(__longlong_as_double(__double_as_longlong(v.x) & m),
            __longlong_as_double(__double_as_longlong(v.y) & m));
}

// ----------------------------------------------------- FP64 matrix cores
// One v_mfma_f64_16x16x4f64: D = A B + C with A 16 x 4 (lane i + 16 k holds
// A[i][k]), B 4 x 16 (lane j + 16 k holds B[k][j]) and C, D 16 x 16 (lane
// j + 16 g holds D[g + 4 v][j] in its v-th element; checked on gfx950 with
// a one-instruction probe).  Every lane of the wave must be active.
typedef double dx4 __attribute__((ext_vector_type(4)));

__device__ inline dx4 mfma_f64(double a, double b, dx4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ----------------------------------------------------- reductions
// DPP lane move of a double (both 32-bit halves with the same pattern);
// lanes whose source is outside the pattern, or whose row is masked off,
// receive 0.
template <int CTRL, int ROW_MASK>
__device__ inline double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ inline double lane63(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
// Sum over the 64 lanes of a wave, returned to every lane.  An inclusive
// scan inside each row of 16 lanes (row_shr 1, 2, 4, 8), then row_bcast 15
// (rows 1 and 3 add the last lane of the row before) and row_bcast 31 (rows
// 2 and 3 add lane 31) leave the total in lane 63.  All 64 lanes must be
// active.
// Column sums of a lane-distributed block: every lane holds v[0..NB) (its
// row's terms of NB columns); on return lane l holds in v[0] the sum over
// all 64 lanes of column l % NB.  Plain sums over the lane bits above
// log2(NB), then a butterfly over the others that halves the values a lane
// keeps at each stage (63 exchanges for 64 columns instead of 6 a column).
// The stages are template recursions so that every index is a constant
// (the array stays in registers).
template <int O, int NB>
__device__ inline void plain_stages(double2 (&v)[NB]) {
  if constexpr (O >= NB) {
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      v[j].x += __shfl_xor(v[j].x, O, 64);
      v[j].y += __shfl_xor(v[j].y, O, 64);
    }
    plain_stages<O / 2, NB>(v);
  }
}
template <int H, int NB>
__device__ inline void butterfly_stages(double2 (&v)[NB], int lane) {
  if constexpr (H >= 1) {
    const bool hi = (lane & H) != 0;
#pragma unroll
    for (int j = 0; j < H; ++j) {
      const double2 send = hi ? v[j] : v[j + H], keep = hi ? v[j + H] : v[j];
      v[j] = cz(keep.x + __shfl_xor(send.x, H, 64), keep.y + __shfl_xor(send.y, H, 64));
    }
    butterfly_stages<H / 2, NB>(v, lane);
  }
}
template <int NB>
__device__ inline void lane_column_sums(double2 (&v)[NB], int lane) {
  plain_stages<32, NB>(v);
  butterfly_stages<NB / 2, NB>(v, lane);
}

constexpr int QHR = 128;   // rows a workgroup in the reflector apply

__device__ inline double wave_sum(double v) {
  v += dpp_move<0x111, 0xf>(v);
  v += dpp_move<0x112, 0xf>(v);
  v += dpp_move<0x114, 0xf>(v);
  v += dpp_move<0x118, 0xf>(v);
  v += dpp_move<0x142, 0xa>(v);
  v += dpp_move<0x143, 0xc>(v);
  return lane63(v);
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
