// Kernels of block PCG (O'Leary): the per-group s x s update applied to the n x s
// column blocks of a row-major n x m matrix (m = groups x s columns, group g holding
// columns g s .. g s + s - 1).  Arithmetic in float64 whatever the storage type.
#include "block.h"

namespace nys {

namespace {

constexpr int kRows = 64;       // rows of a block
constexpr int kJ = 16;          // output columns per thread
constexpr int kMaxS = 64;

// MODE 0: Out += A C;  MODE 1: Out -= A C;  MODE 2: Out = Zs + A C
// (A, Out, Zs row-major with leading dimension ld; C the group's s x s block)
template <class TA, class TO, int MODE>
__global__ __launch_bounds__(256) void blk_apply_kernel(const TA *__restrict__ A, const double *__restrict__ C,
                                                        int s, int ld, TO *__restrict__ Out,
                                                        const TO *__restrict__ Zs, int64_t n) {
  __shared__ double Cs[kMaxS * kMaxS];
  const int g = blockIdx.y;
  const double *Cg = C + (int64_t)g * s * s;
  for (int e = threadIdx.x; e < s * s; e += blockDim.x) Cs[e] = Cg[e];
  __syncthreads();
  const int r = threadIdx.x / (256 / kRows);          // row within the block (4 threads a row)
  const int jc = threadIdx.x % (256 / kRows);         // which 16 output columns
  const int64_t i = (int64_t)blockIdx.x * kRows + r;
  const int j0 = jc * kJ;
  if (i >= n || j0 >= s) return;
  const int jn = s - j0 < kJ ? s - j0 : kJ;
  const int64_t base = i * ld + (int64_t)g * s;
  double acc[kJ];
#pragma unroll
  for (int j = 0; j < kJ; ++j) acc[j] = 0.0;
  for (int k = 0; k < s; ++k) {
    const double a = (double)A[base + k];
#pragma unroll
    for (int j = 0; j < kJ; ++j) acc[j] += a * Cs[k * s + j0 + (j < jn ? j : 0)];
  }
#pragma unroll
  for (int j = 0; j < kJ; ++j) {
    if (j >= jn) break;
    const int64_t o = base + j0 + j;
    if constexpr (MODE == 0) Out[o] = (TO)((double)Out[o] + acc[j]);
    else if constexpr (MODE == 1) Out[o] = (TO)((double)Out[o] - acc[j]);
    else Out[o] = (TO)((double)Zs[o] + acc[j]);
  }
}

}  // namespace

int block_max_s() { return kMaxS; }

template <class TA, class TO>
int32_t blk_apply(int mode, const TA *A, const double *C, int s, int groups, int ld, TO *Out, const TO *Zs,
                  int64_t n, hipStream_t st) {
  if (s < 1 || s > kMaxS) {
    set_error("blk_apply: block size must be 1..64");
    return NYS_EINVAL;
  }
  if (groups <= 0 || n <= 0) return NYS_OK;
  dim3 grid((unsigned)ceil_div(n, kRows), (unsigned)groups);
  if (mode == 0)
    hipLaunchKernelGGL((blk_apply_kernel<TA, TO, 0>), grid, dim3(256), 0, st, A, C, s, ld, Out, Zs, n);
  else if (mode == 1)
    hipLaunchKernelGGL((blk_apply_kernel<TA, TO, 1>), grid, dim3(256), 0, st, A, C, s, ld, Out, Zs, n);
  else
    hipLaunchKernelGGL((blk_apply_kernel<TA, TO, 2>), grid, dim3(256), 0, st, A, C, s, ld, Out, Zs, n);
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}

template int32_t blk_apply<float, float>(int, const float *, const double *, int, int, int, float *, const float *,
                                         int64_t, hipStream_t);
template int32_t blk_apply<float, double>(int, const float *, const double *, int, int, int, double *,
                                          const double *, int64_t, hipStream_t);
template int32_t blk_apply<double, double>(int, const double *, const double *, int, int, int, double *,
                                           const double *, int64_t, hipStream_t);

}  // namespace nys
