// Tall-skinny dense kernels for the Nystrom build and apply: C = A^T B (reduction
// over the long dimension, split into ordered partial sums), C = A B with a
// fused epilogue, and small reductions.  All reductions run in a fixed order,
// so results are bitwise reproducible run to run.
#include <algorithm>

#include "nys_internal.h"

namespace nys {

constexpr int GT = 64;   // output tile
constexpr int GK = 16;   // k slice

// --------------------------------------------------------------- C = A^T B
template <class TA, class TB, class TO>
__global__ __launch_bounds__(256) void gemm_tn_kernel(const TA *A, int lda, const TB *B, int ldb,
                                                      int64_t n, int p, int q, int64_t rows_per,
                                                      TO *out, int ldo, int64_t zstride) {
  __shared__ TA As[GK][GT + 1];
  __shared__ TB Bs[GK][GT + 1];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int p0 = blockIdx.x * GT, q0 = blockIdx.y * GT;
  const int64_t r0 = (int64_t)blockIdx.z * rows_per;
  const int64_t r1 = std::min<int64_t>(n, r0 + rows_per);
  double acc[4][4] = {};
  for (int64_t k0 = r0; k0 < r1; k0 += GK) {
    for (int e = threadIdx.x; e < GK * GT; e += 256) {
      int kk = e / GT, c = e - kk * GT;
      int64_t row = k0 + kk;
      As[kk][c] = (row < r1 && p0 + c < p) ? A[row * lda + p0 + c] : (TA)0;
      Bs[kk][c] = (row < r1 && q0 + c < q) ? B[row * ldb + q0 + c] : (TB)0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK; ++kk) {
      TA a[4];
      TB b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = As[kk][ty * 4 + u];
        b[u] = Bs[kk][tx * 4 + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] += (double)(a[u] * b[v]);
    }
    __syncthreads();
  }
  TO *o = out + (int64_t)blockIdx.z * zstride;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      int i = p0 + ty * 4 + u, j = q0 + tx * 4 + v;
      if (i < p && j < q) o[(int64_t)i * ldo + j] = (TO)acc[u][v];
    }
}

template <class T>
__global__ void sum_partials_kernel(const T *partial, int splits, int p, int q, T *C, int ldc) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)p * q) return;
  const int i = (int)(idx / q), j = (int)(idx - (int64_t)i * q);
  double s = 0.0;
  for (int z = 0; z < splits; ++z) s += (double)partial[(int64_t)z * p * q + idx];
  C[(int64_t)i * ldc + j] = (T)s;
}

int gemm_tn_splits(int64_t n, int p, int q) {
  int64_t tiles = ceil_div(p, GT) * ceil_div(q, GT);
  int64_t want = ceil_div(1024, tiles);
  int64_t maxs = std::max<int64_t>(1, n / 256);
  return (int)std::max<int64_t>(1, std::min<int64_t>(want, maxs));
}

template <class TA, class TB, class T>
static int32_t gemm_tn_impl(const TA *A, int lda, const TB *B, int ldb, int64_t n, int p, int q, T *C,
                            int ldc, T *partial, int splits, hipStream_t s) {
  const int64_t rows_per = round_up(ceil_div(n, splits), GK);
  const int z = (int)ceil_div(n, rows_per);
  dim3 grid((unsigned)ceil_div(p, GT), (unsigned)ceil_div(q, GT), (unsigned)std::max(z, 1));
  if (z <= 1) {
    hipLaunchKernelGGL((gemm_tn_kernel<TA, TB, T>), grid, dim3(256), 0, s, A, lda, B, ldb, n, p, q, rows_per,
                       C, ldc, (int64_t)0);
    NYS_LAUNCH_CHECK();
    return NYS_OK;
  }
  hipLaunchKernelGGL((gemm_tn_kernel<TA, TB, T>), grid, dim3(256), 0, s, A, lda, B, ldb, n, p, q, rows_per,
                     partial, q, (int64_t)p * q);
  NYS_LAUNCH_CHECK();
  const int64_t tot = (int64_t)p * q;
  hipLaunchKernelGGL(sum_partials_kernel<T>, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, s,
                     partial, z, p, q, C, ldc);
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}

template <class T>
int32_t gemm_tn(const T *A, int lda, const T *B, int ldb, int64_t n, int p, int q, T *C, int ldc,
                T *partial, int splits, hipStream_t s) {
  return gemm_tn_impl<T, T, T>(A, lda, B, ldb, n, p, q, C, ldc, partial, splits, s);
}

int32_t gemm_tn_df(const double *A, int lda, const float *B, int ldb, int64_t n, int p, int q, double *C,
                   int ldc, double *partial, int splits, hipStream_t s) {
  return gemm_tn_impl<double, float, double>(A, lda, B, ldb, n, p, q, C, ldc, partial, splits, s);
}

template <class T>
int32_t gemm_tn_to_double(const T *A, int lda, const T *B, int ldb, int64_t n, int p, int q, double *C, int ldc,
                          double *partial, int splits, hipStream_t s) {
  return gemm_tn_impl<T, T, double>(A, lda, B, ldb, n, p, q, C, ldc, partial, splits, s);
}
template int32_t gemm_tn_to_double<float>(const float *, int, const float *, int, int64_t, int, int, double *, int,
                                          double *, int, hipStream_t);
template int32_t gemm_tn_to_double<double>(const double *, int, const double *, int, int64_t, int, int, double *,
                                           int, double *, int, hipStream_t);

// --------------------------------------------------------------- C = A B (+ R * rscale)
// Arithmetic in T; the output C and the epilogue operand R have type TC.
template <class T, class TC>
__global__ __launch_bounds__(256) void gemm_nn_kernel(const T *A, int lda, const T *B, int ldb,
                                                      int64_t n, int p, int q, TC *C, int ldc,
                                                      int epi, const TC *R, int ldr,
                                                      const double *rscale) {
  __shared__ T As[GK][GT + 1];   // As[k][row]
  __shared__ T Bs[GK][GT + 1];   // Bs[k][col]
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int q0 = blockIdx.x * GT;
  const int64_t i0 = (int64_t)blockIdx.y * GT;
  T acc[4][4] = {};
  for (int k0 = 0; k0 < p; k0 += GK) {
    for (int e = threadIdx.x; e < GK * GT; e += 256) {
      int r = e / GK, kk = e - r * GK;          // A: 64 rows x 16 k (k fastest)
      int64_t row = i0 + r;
      As[kk][r] = (row < n && k0 + kk < p) ? A[row * lda + k0 + kk] : (T)0;
      int kb = e / GT, c = e - kb * GT;         // B: 16 k x 64 cols
      Bs[kb][c] = (k0 + kb < p && q0 + c < q) ? B[(int64_t)(k0 + kb) * ldb + q0 + c] : (T)0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK; ++kk) {
      T a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = As[kk][ty * 4 + u];
        b[u] = Bs[kk][tx * 4 + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      int64_t i = i0 + ty * 4 + u;
      int j = q0 + tx * 4 + v;
      if (i < n && j < q) {
        T val = acc[u][v];
        if (epi == 1) val += (T)R[i * ldr + j] * (T)rscale[j];
        C[i * ldc + j] = (TC)val;
      }
    }
}

template <class T>
int32_t gemm_nn(const T *A, int lda, const T *B, int ldb, int64_t n, int p, int q, T *C, int ldc,
                int epi, const T *R, int ldr, const double *rscale, hipStream_t s) {
  if (n <= 0 || q <= 0) return NYS_OK;
  dim3 grid((unsigned)ceil_div(q, GT), (unsigned)ceil_div(n, GT));
  hipLaunchKernelGGL((gemm_nn_kernel<T, T>), grid, dim3(256), 0, s, A, lda, B, ldb, n, p, q, C, ldc, epi, R,
                     ldr, rscale);
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}

int32_t gemm_nn_dd_f(const double *A, int lda, const double *B, int ldb, int64_t n, int p, int q, float *C,
                     int ldc, const float *R, int ldr, const double *rscale, hipStream_t s) {
  if (n <= 0 || q <= 0) return NYS_OK;
  dim3 grid((unsigned)ceil_div(q, GT), (unsigned)ceil_div(n, GT));
  hipLaunchKernelGGL((gemm_nn_kernel<double, float>), grid, dim3(256), 0, s, A, lda, B, ldb, n, p, q, C, ldc, 1,
                     R, ldr, rscale);
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}

template int32_t gemm_tn<double>(const double *, int, const double *, int, int64_t, int, int, double *,
                                 int, double *, int, hipStream_t);
template int32_t gemm_tn<float>(const float *, int, const float *, int, int64_t, int, int, float *, int,
                                float *, int, hipStream_t);
template int32_t gemm_nn<double>(const double *, int, const double *, int, int64_t, int, int, double *,
                                 int, int, const double *, int, const double *, hipStream_t);
template int32_t gemm_nn<float>(const float *, int, const float *, int, int64_t, int, int, float *, int,
                                int, const float *, int, const double *, hipStream_t);

// --------------------------------------------------------------- reductions / elementwise
size_t sumsq_partial_elems(int64_t count) {
  return (size_t)std::max<int64_t>(1, std::min<int64_t>(ceil_div(count, 4096), 1024));
}

__global__ void sumsq_partial_kernel(const double *A, int64_t count, int64_t per, double *partial) {
  __shared__ double red[256];
  const int64_t b0 = (int64_t)blockIdx.x * per;
  const int64_t b1 = std::min<int64_t>(count, b0 + per);
  double s = 0.0;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += 256) s += A[i] * A[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void sum_vec_kernel(const double *partial, int nb, double *out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += partial[b];
    out[0] = s;
  }
}

int32_t launch_sumsq(const double *A, int64_t count, double *partial, double *out, hipStream_t s) {
  const int64_t nb = (int64_t)sumsq_partial_elems(count);
  const int64_t per = ceil_div(count, nb);
  hipLaunchKernelGGL(sumsq_partial_kernel, dim3((unsigned)nb), dim3(256), 0, s, A, count, per, partial);
  NYS_LAUNCH_CHECK();
  hipLaunchKernelGGL(sum_vec_kernel, dim3(1), dim3(64), 0, s, partial, (int)nb, out);
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}

__global__ void axpy_kernel(double a, const double *x, double *y, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) y[i] += a * x[i];
}
__global__ void d2f_kernel(const double *x, float *y, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) y[i] = (float)x[i];
}
__global__ void f2d_kernel(const float *x, double *y, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) y[i] = (double)x[i];
}
__global__ void fill_kernel(double *y, double v, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) y[i] = v;
}
__global__ void fill_f_kernel(float *y, float v, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) y[i] = v;
}

int32_t launch_axpy(double a, const double *x, double *y, int64_t count, hipStream_t s) {
  if (count <= 0) return NYS_OK;
  hipLaunchKernelGGL(axpy_kernel, dim3((unsigned)ceil_div(count, 256)), dim3(256), 0, s, a, x, y, count);
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}
int32_t launch_copy_d2f(const double *x, float *y, int64_t count, hipStream_t s) {
  if (count <= 0) return NYS_OK;
  hipLaunchKernelGGL(d2f_kernel, dim3((unsigned)ceil_div(count, 256)), dim3(256), 0, s, x, y, count);
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}
int32_t launch_copy_f2d(const float *x, double *y, int64_t count, hipStream_t s) {
  if (count <= 0) return NYS_OK;
  hipLaunchKernelGGL(f2d_kernel, dim3((unsigned)ceil_div(count, 256)), dim3(256), 0, s, x, y, count);
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}
int32_t launch_fill(double *y, double v, int64_t count, hipStream_t s) {
  if (count <= 0) return NYS_OK;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)ceil_div(count, 256)), dim3(256), 0, s, y, v, count);
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}
int32_t launch_fill_f(float *y, float v, int64_t count, hipStream_t s) {
  if (count <= 0) return NYS_OK;
  hipLaunchKernelGGL(fill_f_kernel, dim3((unsigned)ceil_div(count, 256)), dim3(256), 0, s, y, v, count);
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}

}  // namespace nys
