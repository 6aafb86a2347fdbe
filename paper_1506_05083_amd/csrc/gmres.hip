// Vector kernels of the batched GMRES on eq. (iter): one Krylov basis per
// incident wave, all waves advanced in lockstep.  CGS2 orthogonalisation is
// dots (h = V^H z) followed by an update (z -= V h), done twice.
#include "internal.hpp"

namespace mfs {
namespace {

// h[w][i] = sum_t conj(V[w][i][t]) z[w][t], one workgroup per (i, w)
__global__ __launch_bounds__(256) void dots_kernel(int n, const double2 *__restrict__ V,
                                                   size_t ldw, size_t ldi,
                                                   const double2 *__restrict__ z, size_t ldz,
                                                   double2 *__restrict__ h, int hstride) {
  const int i = blockIdx.x, w = blockIdx.y;
  const double2 *v = V + w * ldw + i * ldi;
  const double2 *zz = z + w * ldz;
  double2 acc = cz(0.0, 0.0);
  for (int t = threadIdx.x; t < n; t += 256) cfmac(acc, v[t], zz[t]);
  acc = wave_sum(acc);
  __shared__ double2 red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) h[(size_t)w * hstride + i] = cadd(cadd(red[0], red[1]), cadd(red[2], red[3]));
}

// z[w][t] -= sum_{i < nvec} V[w][i][t] h[w][i]
__global__ void update_kernel(int n, int nvec, const double2 *__restrict__ V, size_t ldw, size_t ldi,
                              double2 *__restrict__ z, size_t ldz, const double2 *__restrict__ h,
                              int hstride) {
  const int w = blockIdx.y;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  double2 acc = z[w * ldz + t];
  const double2 *hw = h + (size_t)w * hstride;
  for (int i = 0; i < nvec; ++i) {
    const double2 hv = hw[i];
    const double2 v = V[w * ldw + i * ldi + t];
    acc.x -= v.x * hv.x - v.y * hv.y;
    acc.y -= v.x * hv.y + v.y * hv.x;
  }
  z[w * ldz + t] = acc;
}

// out = x + g
__global__ void add_kernel(long n, const double2 *__restrict__ x, const double2 *__restrict__ g,
                           double2 *__restrict__ out) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    out[i] = cadd(x[i], g[i]);
}

// dst[w][t] = src[w][t] * s[w]
__global__ void scale_kernel(int n, const double2 *__restrict__ src, size_t lds,
                             double2 *__restrict__ dst, size_t ldd, const double *__restrict__ s) {
  const int w = blockIdx.y;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  dst[w * ldd + t] = cscale(src[w * lds + t], s[w]);
}

// dst[w][t] = dst2[w][t] = src[w][t] * s[w] (the next Krylov vector into the
// basis and into the operator's input at once)
__global__ void scale2_kernel(int n, const double2 *__restrict__ src, size_t lds, double2 *__restrict__ dst,
                              size_t ldd, double2 *__restrict__ dst2, size_t ld2, const double *__restrict__ s) {
  const int w = blockIdx.y;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const double2 v = cscale(src[w * lds + t], s[w]);
  dst[w * ldd + t] = v;
  dst2[w * ld2 + t] = v;
}

__global__ void zero2_kernel(double2 *p, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    p[i] = cz(0.0, 0.0);
}

}  // namespace

void launch_zero(double2 *p, long n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(zero2_kernel, dim3((unsigned)std::min<long>(2048, (n + 255) / 256)), dim3(256), 0, s, p, n);
  HIP_CHECK(hipGetLastError());
}

void launch_dots(int nw, int nvec, int n, const double2 *V, size_t ldv_w, size_t ldv_i,
                 const double2 *z, double2 *h, hipStream_t s) {
  // z has the same per-wave stride as one basis vector block: caller passes ldz via ldv_w
  hipLaunchKernelGGL(dots_kernel, dim3(nvec, nw), dim3(256), 0, s, n, V, ldv_w, ldv_i, z,
                     (size_t)n, h, nvec);
  HIP_CHECK(hipGetLastError());
}

void launch_update(int nw, int nvec, int n, const double2 *V, size_t ldv_w, size_t ldv_i, double2 *z,
                   const double2 *h, int hstride, hipStream_t s) {
  hipLaunchKernelGGL(update_kernel, dim3(cdiv(n, 256), nw), dim3(256), 0, s, n, nvec, V, ldv_w, ldv_i, z,
                     (size_t)n, h, hstride);
  HIP_CHECK(hipGetLastError());
}

void launch_axpby_op(int nw, int n, const double2 *x, const double2 *g, const double2 *bd,
                     double2 *out, hipStream_t s) {
  (void)bd;
  const long tot = (long)nw * n;
  hipLaunchKernelGGL(add_kernel, dim3((unsigned)std::min<long>(2048, (tot + 255) / 256)), dim3(256), 0, s,
                     tot, x, g, out);
  HIP_CHECK(hipGetLastError());
}

void launch_scale(int nw, int n, const double2 *src, size_t lds, double2 *dst, size_t ldd,
                  const double *sdev, hipStream_t s) {
  hipLaunchKernelGGL(scale_kernel, dim3(cdiv(n, 256), nw), dim3(256), 0, s, n, src, lds, dst, ldd, sdev);
  HIP_CHECK(hipGetLastError());
}

void launch_scale2(int nw, int n, const double2 *src, size_t lds, double2 *dst, size_t ldd, double2 *dst2,
                   size_t ld2, const double *sdev, hipStream_t s) {
  hipLaunchKernelGGL(scale2_kernel, dim3(cdiv(n, 256), nw), dim3(256), 0, s, n, src, lds, dst, ldd, dst2, ld2, sdev);
  HIP_CHECK(hipGetLastError());
}

}  // namespace mfs
