// Azimuthal transforms between angle samples and Fourier modes.
//
//  forward  (eq. (fhatquad) with q = P, and the final FFT of the A_else
//            action, Sec. 4.1):  out[b] = (1/P) sum_l in[l] e^{-2 pi i b l/P}
//  strengths (point-source form of the ring sources, Sec. 4.1):
//            sigma_l = (1/qs) sum_n c_n e^{+2 pi i n l/qs},  n = mode of bin b
//
// Both are dense DFTs along the middle axis of [nr][len][X] arrays (X the
// ring index, contiguous); the forward one also takes angle samples laid out
// [nr][X][P] (the angle index contiguous).  The lengths here are P <= 256 and qs <= 1024, so
// a direct O(len^2) transform staged through LDS (a 16-wide x tile, exact
// twiddle table indexed by (n l mod Q)) costs less than the HBM traffic of
// the arrays it transforms.
#include "internal.hpp"

namespace mfs {
namespace {

constexpr int XT = 16;

// out[r][o][x] = scale * sum_{i < Pin} in[r][i][x] * exp(sgn 2 pi i (ni(i) o mod Q) / Q)
// with ni(i) = i, or the signed mode of bin i (period Pin) when in_modes;
// in[r][i][x] at r ld_in + i ldi + x xs, out[r][o][x] at r ld_out + o ldo + x.
__global__ __launch_bounds__(256) void dft_kernel(int Pin, int Pout, int Q, int X, int in_modes,
                                                  int sgn, double scale,
                                                  const double2 *__restrict__ in, size_t ld_in, int ldi, int xs,
                                                  double2 *__restrict__ out, size_t ld_out, int ldo) {
  extern __shared__ double2 sh[];
  double2 *tw = sh;            // [Q]
  double2 *tile = sh + Q;      // [Pin][XT]
  const int r = blockIdx.y;
  const int x0 = blockIdx.x * XT;
  for (int i = threadIdx.x; i < Q; i += blockDim.x) {
    double s, c;
    sincospi(2.0 * i / Q, &s, &c);
    tw[i] = cz(c, sgn * s);
  }
  for (int idx = threadIdx.x; idx < Pin * XT; idx += blockDim.x) {
    const int i = idx / XT, xx = idx % XT;
    const int x = x0 + xx;
    tile[idx] = (x < X) ? in[(size_t)r * ld_in + (size_t)i * ldi + (size_t)x * xs] : cz(0.0, 0.0);
  }
  __syncthreads();
  const int xx = threadIdx.x % XT;
  const int x = x0 + xx;
  for (int o = threadIdx.x / XT; o < Pout; o += blockDim.x / XT) {
    double2 acc = cz(0.0, 0.0);
    // ph = (ni(i) o) mod Q, stepped by o (o < Q) and set afresh where ni(i)
    // turns negative (the first negative mode of in_modes)
    const int ohalf = in_modes ? Pin / 2 + 1 : Pin;
    const int oq = o % Q;
    int ph = 0;
    for (int i = 0; i < Pin; ++i) {
      if (i == ohalf) {
        long t = ((long)(i - Pin) * o) % Q;
        ph = (int)(t < 0 ? t + Q : t);
      }
      cfma(acc, tile[i * XT + xx], tw[ph]);
      ph += oq;
      if (ph >= Q) ph -= Q;
    }
    if (x < X) out[(size_t)r * ld_out + (size_t)o * ldo + x] = cscale(acc, scale);
  }
}

}  // namespace

void launch_dft_ld(int nr, int P, int X, const double2 *in, size_t ld_in, double2 *out, int sgn,
                   double scale, hipStream_t s, int ldo) {
  const size_t sh = (size_t)(P + P * XT) * sizeof(double2);
  MFS_REQUIRE(sh <= 64 * 1024, "P too large for the angle transform");
  if (ldo <= 0) ldo = X;
  hipLaunchKernelGGL(dft_kernel, dim3(cdiv(X, XT), nr), dim3(256), sh, s, P, P, P, X, 0, sgn,
                     scale, in, ld_in, X, 1, out, (size_t)P * ldo, ldo);
  HIP_CHECK(hipGetLastError());
}

void launch_angle_to_modes(int nr, int P, int X, const double2 *in, double2 *out, hipStream_t s) {
  const size_t sh = (size_t)(P + P * XT) * sizeof(double2);
  MFS_REQUIRE(sh <= 64 * 1024, "P too large for the angle transform");
  // in[r][x][l]: angle index l contiguous, ring index x strided by P
  hipLaunchKernelGGL(dft_kernel, dim3(cdiv(X, XT), nr), dim3(256), sh, s, P, P, P, X, 0, -1,
                     1.0 / P, in, (size_t)X * P, 1, P, out, (size_t)P * X, X);
  HIP_CHECK(hipGetLastError());
}

void launch_dft(int nr, int P, int X, const double2 *in, double2 *out, int sgn, double scale,
                hipStream_t s) {
  launch_dft_ld(nr, P, X, in, (size_t)P * X, out, sgn, scale, s, X);
}

void launch_point_strengths(int nr, int P, int qs, int N, const double2 *c, double2 *sigma,
                            hipStream_t s, int ldc) {
  MFS_REQUIRE(qs >= P, "point strengths need qs >= P");
  const size_t sh = (size_t)(qs + P * XT) * sizeof(double2);
  MFS_REQUIRE(sh <= 64 * 1024, "qs too large for the strengths transform");
  if (ldc <= 0) ldc = N;
  hipLaunchKernelGGL(dft_kernel, dim3(cdiv(N, XT), nr), dim3(256), sh, s, P, qs, qs, N, 1, +1,
                     1.0 / qs, c, (size_t)P * ldc, ldc, 1, sigma, (size_t)qs * N, N);
  HIP_CHECK(hipGetLastError());
}

}  // namespace mfs
