// Matrix-vector products with a dense row-major float64 matrix X (n x p), the two
// halves of the normal operator X^T (X v) used by the ridge and NysADMM paths.
//
//   rowdot:   t = X v          one wave per row, lanes stride the row (coalesced; 16-byte
//                              loads when the rows are 16-byte aligned)
//   coltrans: out = a X^T t    a 2-D grid of (row chunk, 256-column tile) blocks, each
//                              thread one column of its tile summed over the chunk's
//                              rows (a wave reads 512 contiguous bytes of a row), the
//                              chunk partials then summed in chunk order
//   coltrans with m columns:   Out = a X^T T (T n x m) the same way, a block holding 8
//                              of the m columns per thread (a third grid dimension over
//                              groups of 8), so X is read ceil(m / 8) times
//
// Both are HBM-bound (each reads X once).  A library GEMV with p output rows and n long
// rows has only p-way parallelism when p is small (p = 1000 for a random-feature
// matrix of 4e5 rows); splitting the rows keeps every CU busy at any shape.  The sums
// are in a fixed order, so the results are bitwise repeatable.
#include "gemv.h"

#include <algorithm>

namespace nys {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kCols = 256;          // columns of a coltrans tile
constexpr int kTargetBlocks = 2048; // enough blocks for 256 CUs at any shape
constexpr int kGroup = 8;           // columns of T per thread in the multi-column form
constexpr size_t kMaxPartial = (size_t)8 << 20;   // doubles of chunk partials (64 MiB)

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// 16-byte loads: lane L reads doubles 2L, 2L + 1 of every 128-double segment of a row
// (p even, unit-stride v, so every row starts 16-byte aligned)
__global__ __launch_bounds__(kThreads) void rowdot2_kernel(const double *__restrict__ X, int64_t n, int64_t p,
                                                           const double *__restrict__ v, double *__restrict__ t) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * kWaves;
  const int64_t p2 = p / 2;
  const double2 *v2 = reinterpret_cast<const double2 *>(v);
  for (int64_t i = wave; i < n; i += nwaves) {
    const double2 *row = reinterpret_cast<const double2 *>(X + i * p);
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int64_t j = lane;
    for (; j + 64 < p2; j += 128) {
      const double2 x0 = row[j], x1 = row[j + 64];
      const double2 w0 = v2[j], w1 = v2[j + 64];
      a0 += x0.x * w0.x;
      a1 += x0.y * w0.y;
      a2 += x1.x * w1.x;
      a3 += x1.y * w1.y;
    }
    for (; j < p2; j += 64) {
      const double2 x0 = row[j], w0 = v2[j];
      a0 += x0.x * w0.x;
      a1 += x0.y * w0.y;
    }
    const double s = wave_sum((a0 + a1) + (a2 + a3));
    if (lane == 0) t[i] = s;
  }
}

__global__ __launch_bounds__(kThreads) void rowdot_kernel(const double *__restrict__ X, int64_t n, int64_t p,
                                                          const double *__restrict__ v, int64_t incv,
                                                          double *__restrict__ t) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * kWaves;
  for (int64_t i = wave; i < n; i += nwaves) {
    const double *row = X + i * p;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int64_t j = lane;
    for (; j + 192 < p; j += 256) {
      a0 += row[j] * v[j * incv];
      a1 += row[j + 64] * v[(j + 64) * incv];
      a2 += row[j + 128] * v[(j + 128) * incv];
      a3 += row[j + 192] * v[(j + 192) * incv];
    }
    for (; j < p; j += 64) a0 += row[j] * v[j * incv];
    const double s = wave_sum((a0 + a1) + (a2 + a3));
    if (lane == 0) t[i] = s;
  }
}

// partial[c * p + j] = sum over rows i of chunk c of t[i] X[i][j]
__global__ __launch_bounds__(kThreads) void coltrans_kernel(const double *__restrict__ X, int64_t n, int64_t p,
                                                            const double *__restrict__ t, int64_t rows_per,
                                                            double *__restrict__ partial) {
  const int64_t j = (int64_t)blockIdx.y * kCols + threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per;
  const int64_t r1 = std::min<int64_t>(n, r0 + rows_per);
  if (j >= p) return;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int64_t i = r0;
  for (; i + 3 < r1; i += 4) {
    a0 += t[i] * X[i * p + j];
    a1 += t[i + 1] * X[(i + 1) * p + j];
    a2 += t[i + 2] * X[(i + 2) * p + j];
    a3 += t[i + 3] * X[(i + 3) * p + j];
  }
  for (; i < r1; ++i) a0 += t[i] * X[i * p + j];
  partial[(int64_t)blockIdx.x * p + j] = (a0 + a1) + (a2 + a3);
}

// partial[(c * p + j) * m + k] = sum over rows i of chunk c of X[i][j] T[i][k], for the
// kGroup columns k of group blockIdx.z
__global__ __launch_bounds__(kThreads) void coltrans_multi_kernel(const double *__restrict__ X, int64_t n, int64_t p,
                                                                  const double *__restrict__ T, int m, int64_t ldt,
                                                                  int64_t rows_per, double *__restrict__ partial) {
  const int64_t j = (int64_t)blockIdx.y * kCols + threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per;
  const int64_t r1 = std::min<int64_t>(n, r0 + rows_per);
  const int k0 = blockIdx.z * kGroup;
  const int kn = m - k0 < kGroup ? m - k0 : kGroup;
  if (j >= p) return;
  double acc[kGroup];
#pragma unroll
  for (int k = 0; k < kGroup; ++k) acc[k] = 0.0;
  for (int64_t i = r0; i < r1; ++i) {
    const double x = X[i * p + j];
    const double *t = T + i * ldt + k0;
#pragma unroll
    for (int k = 0; k < kGroup; ++k)
      if (k < kn) acc[k] += x * t[k];
  }
  double *dst = partial + ((int64_t)blockIdx.x * p + j) * m + k0;
#pragma unroll
  for (int k = 0; k < kGroup; ++k)
    if (k < kn) dst[k] = acc[k];
}

// out[e / m * ldo + e % m] = a sum over chunks of partial[c * cnt + e], e < cnt = p m.
// Four waves of a block each sum every fourth chunk of the same 64 elements; the four
// sums are added in wave order.
__global__ __launch_bounds__(kThreads) void chunk_sum_kernel(const double *__restrict__ partial, int chunks,
                                                             int64_t cnt, int m, double a, double *__restrict__ out,
                                                             int64_t ldo) {
  __shared__ double red[kThreads / 64][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t e = (int64_t)blockIdx.x * 64 + lane;
  double s = 0.0;
  if (e < cnt)
    for (int c = w; c < chunks; c += kThreads / 64) s += partial[(int64_t)c * cnt + e];
  red[w][lane] = s;
  __syncthreads();
  if (w == 0 && e < cnt) {
    double t = red[0][lane];
    for (int q = 1; q < kThreads / 64; ++q) t += red[q][lane];
    out[(e / m) * ldo + e % m] = a * t;
  }
}

void coltrans_shape(int64_t n, int64_t p, int m, int &chunks, int64_t &rows_per) {
  const int64_t tiles = ceil_div(p, kCols) * ceil_div(m, kGroup);
  int64_t c = std::max<int64_t>(1, kTargetBlocks / tiles);
  c = std::min<int64_t>(c, std::max<int64_t>(1, ceil_div(n, 64)));   // at least 64 rows a chunk
  c = std::min<int64_t>(c, std::max<int64_t>(1, (int64_t)(kMaxPartial / ((size_t)p * m))));
  rows_per = ceil_div(n, c);
  chunks = (int)ceil_div(n, rows_per);
}

}  // namespace

size_t gemv_partial_elems(int64_t n, int64_t p, int m) {
  int chunks = 1;
  int64_t rows_per = 1;
  coltrans_shape(n, p, std::max(m, 1), chunks, rows_per);
  return (size_t)chunks * (size_t)p * (size_t)std::max(m, 1);
}

int32_t launch_rowdot(const double *X, int64_t n, int64_t p, const double *v, int64_t incv, double *t,
                      hipStream_t s) {
  const int64_t nb = std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, kWaves), 8192));
  const bool wide = p % 2 == 0 && incv == 1 && (reinterpret_cast<uintptr_t>(X) & 15) == 0 &&
                    (reinterpret_cast<uintptr_t>(v) & 15) == 0;
  if (wide)
    hipLaunchKernelGGL(rowdot2_kernel, dim3((unsigned)nb), dim3(kThreads), 0, s, X, n, p, v, t);
  else
    hipLaunchKernelGGL(rowdot_kernel, dim3((unsigned)nb), dim3(kThreads), 0, s, X, n, p, v, incv, t);
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}

int32_t launch_coltrans(const double *X, int64_t n, int64_t p, const double *t, double a, double *out, int64_t inc,
                        double *partial, hipStream_t s) {
  int chunks = 1;
  int64_t rows_per = 1;
  coltrans_shape(n, p, 1, chunks, rows_per);
  const int64_t tiles = ceil_div(p, kCols);
  if (tiles > 65535) {
    set_error("launch_coltrans: more than 65535 * 256 columns");
    return NYS_EINVAL;
  }
  hipLaunchKernelGGL(coltrans_kernel, dim3((unsigned)chunks, (unsigned)tiles), dim3(kThreads), 0, s, X, n, p, t,
                     rows_per, partial);
  NYS_LAUNCH_CHECK();
  hipLaunchKernelGGL(chunk_sum_kernel, dim3((unsigned)ceil_div(p, 64)), dim3(kThreads), 0, s, partial, chunks, p, 1,
                     a, out, inc);
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}

int32_t launch_coltrans_multi(const double *X, int64_t n, int64_t p, const double *T, int m, int64_t ldt, double a,
                              double *Out, int64_t ldo, double *partial, hipStream_t s) {
  int chunks = 1;
  int64_t rows_per = 1;
  coltrans_shape(n, p, m, chunks, rows_per);
  const int64_t tiles = ceil_div(p, kCols), groups = ceil_div(m, kGroup);
  if (tiles > 65535 || groups > 65535) {
    set_error("launch_coltrans_multi: too many columns");
    return NYS_EINVAL;
  }
  hipLaunchKernelGGL(coltrans_multi_kernel, dim3((unsigned)chunks, (unsigned)tiles, (unsigned)groups), dim3(kThreads),
                     0, s, X, n, p, T, m, ldt, rows_per, partial);
  NYS_LAUNCH_CHECK();
  const int64_t cnt = p * (int64_t)m;
  hipLaunchKernelGGL(chunk_sum_kernel, dim3((unsigned)ceil_div(cnt, 64)), dim3(kThreads), 0, s, partial, chunks, cnt,
                     m, a, Out, ldo);
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}

}  // namespace nys
