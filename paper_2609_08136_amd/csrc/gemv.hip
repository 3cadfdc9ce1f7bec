// Matrix-vector products with a dense row-major float64 matrix X (n x p), the two
// halves of the normal operator X^T (X v) used by the ridge and NysADMM paths.
//
//   rowdot:   t = X v          one wave per row, lanes stride the row (coalesced)
//   coltrans: out = a X^T t    a 2-D grid of (row chunk, 256-column tile) blocks, each
//                              thread one column of its tile summed over the chunk's
//                              rows (a wave reads 512 contiguous bytes of a row), the
//                              chunk partials then summed in chunk order
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
constexpr int kTargetBlocks = 4096; // enough blocks for 256 CUs at any shape

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
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

__global__ __launch_bounds__(kThreads) void chunk_sum_kernel(const double *__restrict__ partial, int chunks,
                                                             int64_t p, double a, double *__restrict__ out,
                                                             int64_t inc) {
  const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (j >= p) return;
  double s = 0.0;
  for (int c = 0; c < chunks; ++c) s += partial[(int64_t)c * p + j];
  out[j * inc] = a * s;
}

void coltrans_shape(int64_t n, int64_t p, int &chunks, int64_t &rows_per) {
  const int64_t tiles = ceil_div(p, kCols);
  int64_t c = std::max<int64_t>(1, kTargetBlocks / tiles);
  c = std::min<int64_t>(c, std::max<int64_t>(1, ceil_div(n, 64)));   // at least 64 rows a chunk
  rows_per = ceil_div(n, c);
  chunks = (int)ceil_div(n, rows_per);
}

}  // namespace

size_t gemv_partial_elems(int64_t n, int64_t p) {
  int chunks = 1;
  int64_t rows_per = 1;
  coltrans_shape(n, p, chunks, rows_per);
  return (size_t)chunks * (size_t)p;
}

int32_t launch_rowdot(const double *X, int64_t n, int64_t p, const double *v, int64_t incv, double *t,
                      hipStream_t s) {
  const int64_t nb = std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, kWaves), 8192));
  hipLaunchKernelGGL(rowdot_kernel, dim3((unsigned)nb), dim3(kThreads), 0, s, X, n, p, v, incv, t);
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}

int32_t launch_coltrans(const double *X, int64_t n, int64_t p, const double *t, double a, double *out, int64_t inc,
                        double *partial, hipStream_t s) {
  int chunks = 1;
  int64_t rows_per = 1;
  coltrans_shape(n, p, chunks, rows_per);
  const int64_t tiles = ceil_div(p, kCols);
  if (tiles > 65535) {
    set_error("launch_coltrans: more than 65535 * 256 columns");
    return NYS_EINVAL;
  }
  hipLaunchKernelGGL(coltrans_kernel, dim3((unsigned)chunks, (unsigned)tiles), dim3(kThreads), 0, s, X, n, p, t,
                     rows_per, partial);
  NYS_LAUNCH_CHECK();
  hipLaunchKernelGGL(chunk_sum_kernel, dim3((unsigned)ceil_div(p, kThreads)), dim3(kThreads), 0, s, partial,
                     chunks, p, a, out, inc);
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}

}  // namespace nys
