// Vector kernels of the Krylov driver: multi-dot products with FP64 accumulation (classical
// Gram-Schmidt of FGMRES, Sec. 4.2), basis combinations, axpby, diagonal scaling, conversion.
// Reductions are two-stage with a fixed order, so results are deterministic.
#include <hip/hip_runtime.h>

#include "nsmf_internal.h"

namespace nsmf {

constexpr int BLAS_NT = 256;

// 16-byte vectors of T (4 floats or 2 doubles) for the aligned paths below
template <typename T> struct Vec16;
template <> struct Vec16<float> { typedef float type __attribute__((ext_vector_type(4))); static constexpr int W = 4; };
template <> struct Vec16<double> { typedef double type __attribute__((ext_vector_type(2))); static constexpr int W = 2; };
template <typename T> __host__ __device__ inline bool aligned16(const T *p) { return ((uintptr_t)p & 15u) == 0; }

// partial[b][i] = sum over the block's chunk of V[i][r] * w[r], i < k  (k <= MAX_DOTS).  The basis
// vectors are taken DOT_GROUP at a time, so w is read once per group rather than once per vector;
// each thread's sums run in a fixed order and are combined by a fixed tree, so the result does not
// depend on timing.  VEC: V, its row stride and w allow 16-byte loads; the chunks then cover whole
// vectors of Vec16<T>::W entries, and the last block also takes the n mod W trailing entries.
constexpr int DOT_GROUP = 8, DOT_ROWS = 2;
template <typename T, bool VEC>
__global__ void __launch_bounds__(BLAS_NT)
k_dots_partial(int64_t n, int k, const T *__restrict__ V, int64_t ldv, const T *__restrict__ w,
               double *__restrict__ partial, const int32_t *__restrict__ flag) {
  __shared__ double red[DOT_GROUP][BLAS_NT];
  if (flag != nullptr && flag[0] == 0) return;   // conditional call not taken (k_dots_final zeroes h)
  constexpr int VW = VEC ? Vec16<T>::W : 1;
  typedef typename Vec16<T>::type vec;
  const int64_t nv = n / VW;   // whole vectors (VEC) or entries
  const int64_t chunk = (nv + gridDim.x - 1) / gridDim.x;
  const int64_t q0 = (int64_t)blockIdx.x * chunk, q1 = q0 + chunk < nv ? q0 + chunk : nv;
  for (int i0 = 0; i0 < k; i0 += DOT_GROUP) {
    double s[DOT_GROUP];
#pragma unroll
    for (int g = 0; g < DOT_GROUP; ++g) s[g] = 0.0;
    // DOT_ROWS steps per iteration: that many times the independent loads in flight per thread
    for (int64_t q = q0 + threadIdx.x; q < q1; q += DOT_ROWS * BLAS_NT) {
#pragma unroll
      for (int u = 0; u < DOT_ROWS; ++u) {
        const int64_t qu = q + (int64_t)u * BLAS_NT;
        if (qu >= q1) break;
        if constexpr (VEC) {
          const vec wv = *reinterpret_cast<const vec *>(w + qu * VW);
          vec v[DOT_GROUP];
#pragma unroll
          for (int g = 0; g < DOT_GROUP; ++g)
            if (i0 + g < k) v[g] = *reinterpret_cast<const vec *>(V + (int64_t)(i0 + g) * ldv + qu * VW);
#pragma unroll
          for (int g = 0; g < DOT_GROUP; ++g)
            if (i0 + g < k)
#pragma unroll
              for (int e = 0; e < VW; ++e) s[g] += (double)v[g][e] * (double)wv[e];
        } else {
          const double wr = (double)w[qu];
          T v[DOT_GROUP];
#pragma unroll
          for (int g = 0; g < DOT_GROUP; ++g) v[g] = i0 + g < k ? V[(int64_t)(i0 + g) * ldv + qu] : T(0);
#pragma unroll
          for (int g = 0; g < DOT_GROUP; ++g) s[g] += (double)v[g] * wr;
        }
      }
    }
    if (VEC && blockIdx.x == gridDim.x - 1) {   // trailing entries
      const int64_t r = nv * VW + threadIdx.x;
      if (r < n)
#pragma unroll
        for (int g = 0; g < DOT_GROUP; ++g)
          if (i0 + g < k) s[g] += (double)V[(int64_t)(i0 + g) * ldv + r] * (double)w[r];
    }
#pragma unroll
    for (int g = 0; g < DOT_GROUP; ++g) red[g][threadIdx.x] = s[g];
    __syncthreads();
    for (int h = BLAS_NT / 2; h > 0; h >>= 1) {
      if ((int)threadIdx.x < h)
#pragma unroll
        for (int g = 0; g < DOT_GROUP; ++g) red[g][threadIdx.x] += red[g][threadIdx.x + h];
      __syncthreads();
    }
    if ((int)threadIdx.x < DOT_GROUP && i0 + (int)threadIdx.x < k)
      partial[(size_t)blockIdx.x * MAX_DOTS + i0 + threadIdx.x] = red[threadIdx.x][0];
    __syncthreads();
  }
}

// h[i] = sum over the nb blocks of partial[b][i]: one block per dot, a fixed-order strided sum per
// thread and a fixed tree across the block
__global__ void __launch_bounds__(BLAS_NT) k_dots_final(int nb, const double *__restrict__ partial,
                                                        double *__restrict__ h, const int32_t *__restrict__ flag) {
  __shared__ double red[BLAS_NT];
  const int i = blockIdx.x;
  if (flag != nullptr && flag[0] == 0) {   // conditional call not taken: h[i] = 0
    if (threadIdx.x == 0) h[i] = 0.0;
    return;
  }
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += BLAS_NT) s += partial[(size_t)b * MAX_DOTS + i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int hh = BLAS_NT / 2; hh > 0; hh >>= 1) {
    if ((int)threadIdx.x < hh) red[threadIdx.x] += red[threadIdx.x + hh];
    __syncthreads();
  }
  if (threadIdx.x == 0) h[i] = red[0];
}

// w[r] += alpha * sum_i V[i][r] h[i]; the basis entries are loaded GEMV_GROUP at a time ahead of the
// (fixed-order) accumulation, so that a thread has that many independent loads in flight.  VEC: each
// thread takes Vec16<T>::W consecutive entries with 16-byte loads (V, its row stride and w aligned);
// the threads past the whole vectors take the trailing entries one each.
constexpr int GEMV_GROUP = 8;
template <typename T, bool VEC>
__global__ void k_gemv(int64_t n, int k, const T *__restrict__ V, int64_t ldv, const double *__restrict__ h,
                       double alpha, T *__restrict__ w, const int32_t *__restrict__ flag) {
  if (flag != nullptr && flag[0] == 0) return;   // conditional call not taken
  constexpr int VW = VEC ? Vec16<T>::W : 1;
  typedef typename Vec16<T>::type vec;
  const int64_t nv = n / VW;
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (VEC && q < nv) {
    double s[VW];
#pragma unroll
    for (int e = 0; e < VW; ++e) s[e] = 0.0;
    for (int i0 = 0; i0 < k; i0 += GEMV_GROUP) {
      vec v[GEMV_GROUP];
#pragma unroll
      for (int g = 0; g < GEMV_GROUP; ++g)
        if (i0 + g < k) v[g] = *reinterpret_cast<const vec *>(V + (int64_t)(i0 + g) * ldv + q * VW);
#pragma unroll
      for (int g = 0; g < GEMV_GROUP; ++g)
        if (i0 + g < k)
#pragma unroll
          for (int e = 0; e < VW; ++e) s[e] += (double)v[g][e] * h[i0 + g];
    }
    vec wv = *reinterpret_cast<const vec *>(w + q * VW);
#pragma unroll
    for (int e = 0; e < VW; ++e) wv[e] = (T)((double)wv[e] + alpha * s[e]);
    *reinterpret_cast<vec *>(w + q * VW) = wv;
    return;
  }
  const int64_t r = VEC ? nv * VW + (q - nv) : q;
  if (r >= n) return;
  double s = 0.0;
  for (int i0 = 0; i0 < k; i0 += GEMV_GROUP) {
    T v[GEMV_GROUP];
#pragma unroll
    for (int g = 0; g < GEMV_GROUP; ++g) v[g] = i0 + g < k ? V[(int64_t)(i0 + g) * ldv + r] : T(0);
#pragma unroll
    for (int g = 0; g < GEMV_GROUP; ++g)
      if (i0 + g < k) s += (double)v[g] * h[i0 + g];
  }
  w[r] = (T)((double)w[r] + alpha * s);
}

// y = a x + b y; with b == 0 the old y is not read (BLAS convention), so y may hold any bits
template <typename T>
__global__ void k_axpby(int64_t n, double a, const T *__restrict__ x, double b, T *__restrict__ y) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) y[r] = (T)(b == 0.0 ? a * (double)x[r] : a * (double)x[r] + b * (double)y[r]);
}

// x = x / sqrt(nrm2[0]) with the squared norm read on the device (0 when nrm2[0] <= 0): the Arnoldi
// normalisation without a round trip of the norm through the host
template <typename T>
__global__ void k_normalize(int64_t n, const double *__restrict__ nrm2, T *__restrict__ x) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double s = nrm2[0];
  const double f = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
  if (r < n) x[r] = (T)((double)x[r] * f);
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

// the 16-byte paths need V, w and (for more than one row) the row stride 16-byte aligned
template <typename T>
static bool vec_ok(const T *V, int64_t ldv, int k, const T *w) {
  return aligned16(V) && aligned16(w) && (k == 1 || (ldv * (int64_t)sizeof(T)) % 16 == 0);
}

template <typename T>
static void dots_t(hipStream_t s, int64_t n, int k, const T *V, int64_t ldv, const T *w, double *partial, int nb,
                   const int32_t *flag) {
  if (vec_ok(V, ldv, k, w))
    hipLaunchKernelGGL((k_dots_partial<T, true>), dim3(nb), dim3(BLAS_NT), 0, s, n, k, V, ldv, w, partial, flag);
  else
    hipLaunchKernelGGL((k_dots_partial<T, false>), dim3(nb), dim3(BLAS_NT), 0, s, n, k, V, ldv, w, partial, flag);
}

hipError_t launch_dots(hipStream_t s, int prec, int64_t n, int k, const void *V, int64_t ldv, const void *w,
                       double *partial, double *h, const int32_t *flag) {
  const int nb = n < (int64_t)DOT_BLOCKS * BLAS_NT ? nblk(n) : DOT_BLOCKS;
  if (prec == 0) dots_t<double>(s, n, k, (const double *)V, ldv, (const double *)w, partial, nb, flag);
  else dots_t<float>(s, n, k, (const float *)V, ldv, (const float *)w, partial, nb, flag);
  hipLaunchKernelGGL(k_dots_final, dim3(k), dim3(BLAS_NT), 0, s, nb, partial, h, flag);
  return hipGetLastError();
}

template <typename T>
static void gemv_t(hipStream_t s, int64_t n, int k, const T *V, int64_t ldv, const double *h, double alpha, T *w,
                   const int32_t *flag) {
  if (vec_ok(V, ldv, k, (const T *)w)) {
    constexpr int VW = Vec16<T>::W;
    const int64_t items = n / VW + n % VW;
    hipLaunchKernelGGL((k_gemv<T, true>), dim3(nblk(items)), dim3(BLAS_NT), 0, s, n, k, V, ldv, h, alpha, w, flag);
  } else {
    hipLaunchKernelGGL((k_gemv<T, false>), dim3(nblk(n)), dim3(BLAS_NT), 0, s, n, k, V, ldv, h, alpha, w, flag);
  }
}

hipError_t launch_gemv(hipStream_t s, int prec, int64_t n, int k, const void *V, int64_t ldv, const double *h,
                       double alpha, void *w, const int32_t *flag) {
  if (prec == 0) gemv_t<double>(s, n, k, (const double *)V, ldv, h, alpha, (double *)w, flag);
  else gemv_t<float>(s, n, k, (const float *)V, ldv, h, alpha, (float *)w, flag);
  return hipGetLastError();
}

// Squared norm after the projection w -= V h, from the dots of the rows and of w itself (h[k] = |w|^2):
// nrm2 = h[k] - sum_{i<k} h[i]^2 (exact when the rows are orthonormal), summed in a fixed order, and
// the test for a second Gram-Schmidt pass, nrm2 < eta2 h[k] (the criterion of Daniel, Gragg, Kaufman
// and Stewart, 1976).  A flag_in of 0 leaves everything unchanged.
__global__ void k_gs_norm(int k, const double *__restrict__ h, double eta2, const int32_t *__restrict__ flag_in,
                          int32_t *__restrict__ flag_out, double *__restrict__ nrm2) {
  if (flag_in != nullptr && flag_in[0] == 0) return;
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < k; ++i) s += h[i] * h[i];
  const double est = h[k] - s;
  nrm2[0] = est;
  if (flag_out != nullptr) flag_out[0] = est < eta2 * h[k] ? 1 : 0;
}

hipError_t launch_gs_norm(hipStream_t s, int k, const double *h, double eta2, const int32_t *flag_in, int32_t *flag_out,
                          double *nrm2) {
  hipLaunchKernelGGL(k_gs_norm, dim3(1), dim3(64), 0, s, k, h, eta2, flag_in, flag_out, nrm2);
  return hipGetLastError();
}

hipError_t launch_axpby(hipStream_t s, int prec, int64_t n, double a, const void *x, double b, void *y) {
  if (prec == 0)
    hipLaunchKernelGGL(k_axpby<double>, dim3(nblk(n)), dim3(BLAS_NT), 0, s, n, a, (const double *)x, b, (double *)y);
  else
    hipLaunchKernelGGL(k_axpby<float>, dim3(nblk(n)), dim3(BLAS_NT), 0, s, n, a, (const float *)x, b, (float *)y);
  return hipGetLastError();
}

hipError_t launch_normalize(hipStream_t s, int prec, int64_t n, const double *nrm2, void *x) {
  if (n <= 0) return hipSuccess;
  if (prec == 0)
    hipLaunchKernelGGL(k_normalize<double>, dim3(nblk(n)), dim3(BLAS_NT), 0, s, n, nrm2, (double *)x);
  else
    hipLaunchKernelGGL(k_normalize<float>, dim3(nblk(n)), dim3(BLAS_NT), 0, s, n, nrm2, (float *)x);
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


// ---------------------------------------------------------------- horizontal coarse space
// Coarse functions of the two-level velocity preconditioner: a bilinear hat of a coarse lattice point
// in (x, y) times one of NCZ profiles in the node's relative height zeta (1 - zeta, zeta, 4 zeta (1 -
// zeta)), per velocity component.  Coarse vectors are FP64 [3][n_cpts][NCZ].  Node n belongs to the
// coarse cell whose corners are cpt[n][0..3] with bilinear weights w[n][0..3]; masked components are
// zero (the coarse functions are prolongated into the Dirichlet-eliminated space).
constexpr int NCZ = 3;
__device__ __forceinline__ void zprof(double z, double (&l)[NCZ]) {
  l[0] = 1.0 - z;
  l[1] = z;
  l[2] = 4.0 * z * (1.0 - z);
}

template <typename T>
__global__ void k_prolong(int64_t N, int64_t nc, const int32_t *__restrict__ cpt, const double *__restrict__ cw,
                          const double *__restrict__ zeta, const uint8_t *__restrict__ dm, const double *__restrict__ xc,
                          T *__restrict__ x) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  // node inputs first (unsigned corner ids: widening them needs no wait for the load)
  uint32_t cj[4];
  double wj[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    cj[j] = (uint32_t)cpt[4 * n + j];
    wj[j] = cw[4 * n + j];
  }
  int dv[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) dv[c] = dm[(size_t)c * N + n];
  double l[NCZ];
  zprof(zeta[n], l);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double v = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double *p = xc + ((size_t)c * nc + cj[j]) * NCZ;
      v += wj[j] * (l[0] * p[0] + l[1] * p[1] + l[2] * p[2]);
    }
    x[(size_t)c * N + n] = dv[c] ? T(0) : (T)v;
  }
}

// rc[c][J][m] = sum over the nodes n of coarse point J (list cptr/cnode/cwt, fixed order) of
// w_J(n) l_m(zeta_n) (P r)[c][n]: one block per coarse point, FP64 accumulation, fixed reduction order.
constexpr int RST_NT = 256;
template <typename T>
__global__ void __launch_bounds__(RST_NT)
k_restrict(int64_t N, int64_t nc, const int64_t *__restrict__ cptr, const int32_t *__restrict__ cnode,
           const double *__restrict__ cwt, const double *__restrict__ zeta, const uint8_t *__restrict__ dm,
           const T *__restrict__ r, double *__restrict__ rc) {
  __shared__ double red[3 * NCZ][RST_NT];
  const int64_t J = blockIdx.x;
  double acc[3][NCZ] = {};
  // each thread takes list entries k = k0 + tid + RST_NT i in increasing i, UB at a time: all their
  // loads are requested before any is used (entries past the end read entry k0, in bounds, and add
  // zero: a conditional accumulation lets the compiler move the loads into the branches)
  constexpr int UB = 4;
  const int64_t k0 = cptr[J], k1 = cptr[J + 1];
  for (int64_t kb = k0 + threadIdx.x; kb < k1; kb += UB * RST_NT) {
    uint32_t nn[UB];   // unsigned: widening it to an address needs no wait for the loaded value
    double wv[UB];
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const int64_t k = kb + (int64_t)u * RST_NT, kc = k < k1 ? k : k0;
      nn[u] = (uint32_t)cnode[kc];
      wv[u] = cwt[kc];
    }
    double z[UB], rv[UB][3];
    int dv[UB][3];
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      z[u] = zeta[nn[u]];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        dv[u][c] = dm[(size_t)c * N + nn[u]];
        rv[u][c] = (double)r[(size_t)c * N + nn[u]];
      }
    }
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const bool in = kb + (int64_t)u * RST_NT < k1;
      double l[NCZ];
      zprof(z[u], l);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double v = (dv[u][c] || !in) ? 0.0 : rv[u][c];
        for (int m = 0; m < NCZ; ++m) acc[c][m] += wv[u] * l[m] * v;
      }
    }
  }
  for (int c = 0; c < 3; ++c)
    for (int m = 0; m < NCZ; ++m) red[c * NCZ + m][threadIdx.x] = acc[c][m];
  __syncthreads();
  for (int h = RST_NT / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h)
      for (int f = 0; f < 3 * NCZ; ++f) red[f][threadIdx.x] += red[f][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x < 3 * NCZ) {
    const int c = threadIdx.x / NCZ, m = threadIdx.x % NCZ;
    rc[((size_t)c * nc + J) * NCZ + m] = red[threadIdx.x][0];
  }
}

hipError_t launch_prolong(hipStream_t s, int prec, int64_t N, int64_t nc, const int32_t *cpt, const double *cw,
                          const double *zeta, const uint8_t *dm, const double *xc, void *x) {
  if (N <= 0) return hipSuccess;
  if (prec == 0)
    hipLaunchKernelGGL(k_prolong<double>, dim3(nblk(N)), dim3(BLAS_NT), 0, s, N, nc, cpt, cw, zeta, dm, xc, (double *)x);
  else
    hipLaunchKernelGGL(k_prolong<float>, dim3(nblk(N)), dim3(BLAS_NT), 0, s, N, nc, cpt, cw, zeta, dm, xc, (float *)x);
  return hipGetLastError();
}
hipError_t launch_restrict(hipStream_t s, int prec, int64_t N, int64_t nc, const int64_t *cptr, const int32_t *cnode,
                           const double *cwt, const double *zeta, const uint8_t *dm, const void *r, double *rc) {
  if (nc <= 0) return hipSuccess;
  if (prec == 0)
    hipLaunchKernelGGL(k_restrict<double>, dim3((unsigned)nc), dim3(RST_NT), 0, s, N, nc, cptr, cnode, cwt, zeta, dm,
                       (const double *)r, rc);
  else
    hipLaunchKernelGGL(k_restrict<float>, dim3((unsigned)nc), dim3(RST_NT), 0, s, N, nc, cptr, cnode, cwt, zeta, dm,
                       (const float *)r, rc);
  return hipGetLastError();
}

}  // namespace nsmf
