// Vector kernels of the Krylov driver: multi-dot products with FP64 accumulation (classical
// Gram-Schmidt of FGMRES, Sec. 4.2), basis combinations, axpby, diagonal scaling, conversion.
// Reductions are two-stage with a fixed order, so results are deterministic.
#include <hip/hip_runtime.h>

#include "nsmf_internal.h"

namespace nsmf {

constexpr int BLAS_NT = 256;
constexpr int DOT_BLOCKS = 1024;

// partial[b][i] = sum over the block's chunk of V[i][r] * w[r], i < k  (k <= MAX_DOTS)
template <typename T>
__global__ void __launch_bounds__(BLAS_NT)
k_dots_partial(int64_t n, int k, const T *__restrict__ V, int64_t ldv, const T *__restrict__ w,
               double *__restrict__ partial) {
  __shared__ double red[BLAS_NT];
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * chunk, r1 = r0 + chunk < n ? r0 + chunk : n;
  for (int i = 0; i < k; ++i) {
    double s = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += BLAS_NT) s += (double)V[i * ldv + r] * (double)w[r];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = BLAS_NT / 2; h > 0; h >>= 1) {
      if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[(size_t)blockIdx.x * MAX_DOTS + i] = red[0];
    __syncthreads();
  }
}

__global__ void k_dots_final(int nb, int k, const double *__restrict__ partial, double *__restrict__ h) {
  const int i = threadIdx.x;
  if (i >= k) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += partial[(size_t)b * MAX_DOTS + i];
  h[i] = s;
}

// w[r] += alpha * sum_i V[i][r] h[i]
template <typename T>
__global__ void k_gemv(int64_t n, int k, const T *__restrict__ V, int64_t ldv, const double *__restrict__ h,
                       double alpha, T *__restrict__ w) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double s = 0.0;
  for (int i = 0; i < k; ++i) s += (double)V[i * ldv + r] * h[i];
  w[r] = (T)((double)w[r] + alpha * s);
}

// y = a x + b y; with b == 0 the old y is not read (BLAS convention), so y may hold any bits
template <typename T>
__global__ void k_axpby(int64_t n, double a, const T *__restrict__ x, double b, T *__restrict__ y) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) y[r] = (T)(b == 0.0 ? a * (double)x[r] : a * (double)x[r] + b * (double)y[r]);
}

// z = d * x (elementwise), d in FP64
template <typename T>
__global__ void k_mul(int64_t n, const double *__restrict__ d, const T *__restrict__ x, T *__restrict__ z) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) z[r] = (T)(d[r] * (double)x[r]);
}

__global__ void k_recip(int64_t n, double *__restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 1.0 / x[i];
}

__global__ void k_f2d(const float *in, double *out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (double)in[i];
}

static inline int nblk(int64_t n) { return (int)((n + BLAS_NT - 1) / BLAS_NT); }

hipError_t launch_dots(hipStream_t s, int prec, int64_t n, int k, const void *V, int64_t ldv, const void *w,
                       double *partial, double *h) {
  const int nb = n < (int64_t)DOT_BLOCKS * BLAS_NT ? nblk(n) : DOT_BLOCKS;
  if (prec == 0)
    hipLaunchKernelGGL(k_dots_partial<double>, dim3(nb), dim3(BLAS_NT), 0, s, n, k, (const double *)V, ldv,
                       (const double *)w, partial);
  else
    hipLaunchKernelGGL(k_dots_partial<float>, dim3(nb), dim3(BLAS_NT), 0, s, n, k, (const float *)V, ldv,
                       (const float *)w, partial);
  hipLaunchKernelGGL(k_dots_final, dim3(1), dim3(MAX_DOTS), 0, s, nb, k, partial, h);
  return hipGetLastError();
}

hipError_t launch_gemv(hipStream_t s, int prec, int64_t n, int k, const void *V, int64_t ldv, const double *h,
                       double alpha, void *w) {
  if (prec == 0)
    hipLaunchKernelGGL(k_gemv<double>, dim3(nblk(n)), dim3(BLAS_NT), 0, s, n, k, (const double *)V, ldv, h, alpha,
                       (double *)w);
  else
    hipLaunchKernelGGL(k_gemv<float>, dim3(nblk(n)), dim3(BLAS_NT), 0, s, n, k, (const float *)V, ldv, h, alpha,
                       (float *)w);
  return hipGetLastError();
}

hipError_t launch_axpby(hipStream_t s, int prec, int64_t n, double a, const void *x, double b, void *y) {
  if (prec == 0)
    hipLaunchKernelGGL(k_axpby<double>, dim3(nblk(n)), dim3(BLAS_NT), 0, s, n, a, (const double *)x, b, (double *)y);
  else
    hipLaunchKernelGGL(k_axpby<float>, dim3(nblk(n)), dim3(BLAS_NT), 0, s, n, a, (const float *)x, b, (float *)y);
  return hipGetLastError();
}

hipError_t launch_mul(hipStream_t s, int prec, int64_t n, const double *d, const void *x, void *z) {
  if (prec == 0)
    hipLaunchKernelGGL(k_mul<double>, dim3(nblk(n)), dim3(BLAS_NT), 0, s, n, d, (const double *)x, (double *)z);
  else
    hipLaunchKernelGGL(k_mul<float>, dim3(nblk(n)), dim3(BLAS_NT), 0, s, n, d, (const float *)x, (float *)z);
  return hipGetLastError();
}

hipError_t launch_recip(hipStream_t s, int64_t n, double *x) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_recip, dim3(nblk(n)), dim3(BLAS_NT), 0, s, n, x);
  return hipGetLastError();
}

hipError_t launch_f2d(hipStream_t s, const float *in, double *out, int64_t n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_f2d, dim3(nblk(n)), dim3(BLAS_NT), 0, s, in, out, n);
  return hipGetLastError();
}

}  // namespace nsmf
