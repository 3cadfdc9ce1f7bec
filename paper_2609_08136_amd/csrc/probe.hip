// Ceiling probes: synthetic kernels that keep one execution unit of the GPU busy,
// timed with HIP events, so that a kernel's rate can be set against what this chip
// actually sustains and not only against its data sheet (bf16 / fp16 / float64 MFMA,
// the float32 transcendental exp2, and a plain device copy for HBM bandwidth).
#include <algorithm>

#include "kmv_common.h"

namespace nys {
namespace {

constexpr int PROBE_THREADS = 256;    // four waves per workgroup
// MFMA probes: two waves per SIMD on 256 CUs, two independent accumulators per wave,
// each updated in place (more chains let the compiler rotate accumulators through
// different registers, which measured 40% slower); exp2 probe: eight waves per SIMD
constexpr int PROBE_BLOCKS_MFMA = 512;
constexpr int PROBE_BLOCKS_EXP = 2048;
constexpr int PROBE_CHAINS = 2;

template <class V, class S>
__device__ inline V probe_operand(int lane, float scale) {
  V v;
#pragma unroll
  for (int e = 0; e < 8; ++e) v[e] = (S)(scale * (float)((lane + 3 * e) % 7 - 3));
  return v;
}

// WHICH 0: v_mfma_f32_16x16x32_bf16, 1: v_mfma_f32_16x16x32_f16,
// 2: v_mfma_f64_16x16x4f64, 3: v_exp_f32 (eight independent chains x <- 2^-x per
// lane; the negation is a free source modifier, so the loop is exp2 alone).
template <int WHICH>
__global__ __launch_bounds__(PROBE_THREADS) void probe_kernel(int iters, float *sink) {
  const int lane = threadIdx.x & 63;
  float out = 0.0f;
  if constexpr (WHICH == 0 || WHICH == 1) {
    using V = typename std::conditional<WHICH == 0, bf8, h8>::type;
    using S = typename std::conditional<WHICH == 0, __bf16, _Float16>::type;
    const V a = probe_operand<V, S>(lane, 1e-3f), b = probe_operand<V, S>(lane + 1, 2e-3f);
    f4 c[PROBE_CHAINS];
#pragma unroll
    for (int k = 0; k < PROBE_CHAINS; ++k) c[k] = f4{0, 0, 0, 0};
    for (int i = 0; i < iters; ++i)
#pragma unroll
      for (int k = 0; k < PROBE_CHAINS; ++k) c[k] = mfma16(a, b, c[k]);
#pragma unroll
    for (int k = 0; k < PROBE_CHAINS; ++k) out += c[k][0] + c[k][1] + c[k][2] + c[k][3];
  } else if constexpr (WHICH == 2) {
    const double a = 1e-3 * (double)(lane % 7), b = 2e-3 * (double)(lane % 5);
    d4 c[PROBE_CHAINS];
#pragma unroll
    for (int k = 0; k < PROBE_CHAINS; ++k) c[k] = d4{0, 0, 0, 0};
    for (int i = 0; i < iters; ++i)
#pragma unroll
      for (int k = 0; k < PROBE_CHAINS; ++k) c[k] = mfma16(a, b, c[k]);
#pragma unroll
    for (int k = 0; k < PROBE_CHAINS; ++k) out += (float)(c[k][0] + c[k][1] + c[k][2] + c[k][3]);
  } else {
    float x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = 0.01f * (float)(lane + k);
    for (int i = 0; i < iters; ++i)
#pragma unroll
      for (int k = 0; k < 8; ++k) x[k] = __builtin_amdgcn_exp2f(-x[k]);
#pragma unroll
    for (int k = 0; k < 8; ++k) out += x[k];
  }
  sink[(int64_t)blockIdx.x * PROBE_THREADS + threadIdx.x] = out;
}

__global__ void probe_copy_kernel(const uint4 *src, uint4 *dst, int64_t count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) dst[i] = src[i];
}

// Work of one probe launch in its unit (flop, exp or byte).
double probe_work(int which, int iters, int64_t copy_chunks) {
  const double waves = (double)PROBE_BLOCKS_MFMA * (PROBE_THREADS / 64);
  switch (which) {
    case 0:
    case 1: return waves * iters * PROBE_CHAINS * (16.0 * 16 * 32 * 2);
    case 2: return waves * iters * PROBE_CHAINS * (16.0 * 16 * 4 * 2);
    case 3: return (double)PROBE_BLOCKS_EXP * PROBE_THREADS * iters * 8.0;
    default: return 2.0 * 16.0 * (double)copy_chunks;   // read + write
  }
}

int32_t probe_launch(int which, int iters, float *sink, const uint4 *src, uint4 *dst, int64_t chunks,
                     hipStream_t s) {
  const dim3 grid(which == 3 ? PROBE_BLOCKS_EXP : PROBE_BLOCKS_MFMA), block(PROBE_THREADS);
  switch (which) {
    case 0: hipLaunchKernelGGL(probe_kernel<0>, grid, block, 0, s, iters, sink); break;
    case 1: hipLaunchKernelGGL(probe_kernel<1>, grid, block, 0, s, iters, sink); break;
    case 2: hipLaunchKernelGGL(probe_kernel<2>, grid, block, 0, s, iters, sink); break;
    case 3: hipLaunchKernelGGL(probe_kernel<3>, grid, block, 0, s, iters, sink); break;
    default: hipLaunchKernelGGL(probe_copy_kernel, dim3(4096), dim3(256), 0, s, src, dst, chunks); break;
  }
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}

}  // namespace

size_t probe_sink_bytes() { return (size_t)PROBE_BLOCKS_EXP * PROBE_THREADS * sizeof(float); }

int32_t peak_probe(int which, int iters, double *rate, void *ws, size_t ws_bytes, hipStream_t s) {
  if (which < 0 || which > 4) {
    set_error("nys_peak_probe: which must be 0..4");
    return NYS_EINVAL;
  }
  if (!rate || !ws) {
    set_error("nys_peak_probe: null pointer");
    return NYS_EINVAL;
  }
  if (iters < 0) {
    set_error("nys_peak_probe: iters must be >= 0");
    return NYS_EINVAL;
  }
  const size_t need = which == 4 ? ((size_t)2 << 20) : probe_sink_bytes();
  if (ws_bytes < need) {
    set_error("nys_peak_probe: workspace too small");
    return NYS_ENOMEM;
  }
  // default loop lengths: about 50-100 ms per launch on MI355X
  static const int def_iters[4] = {1600000, 1600000, 400000, 200000};
  if (which < 4 && iters == 0) iters = def_iters[which];
  float *sink = reinterpret_cast<float *>(ws);
  const int64_t chunks = which == 4 ? (int64_t)(ws_bytes / 2 / 16) : 0;
  const uint4 *src = reinterpret_cast<const uint4 *>(ws);
  uint4 *dst = reinterpret_cast<uint4 *>(reinterpret_cast<char *>(ws) + chunks * 16);
  const int reps = which == 4 ? std::max(1, iters) : 1;
  NYS_RETURN_IF(probe_launch(which, iters, sink, src, dst, chunks, s));   // untimed
  hipEvent_t e0, e1;
  NYS_CHECK_HIP(hipEventCreate(&e0));
  NYS_CHECK_HIP(hipEventCreate(&e1));
  int32_t rc = NYS_OK;
  float ms = 0.0f;
  if (hipEventRecord(e0, s) != hipSuccess) rc = NYS_EHIP;
  for (int t = 0; t < reps && rc == NYS_OK; ++t) rc = probe_launch(which, iters, sink, src, dst, chunks, s);
  if (rc == NYS_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                       hipEventElapsedTime(&ms, e0, e1) != hipSuccess)) {
    set_error("nys_peak_probe: HIP event failure while timing");
    rc = NYS_EHIP;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  NYS_RETURN_IF(rc);
  *rate = ms > 0.0f ? probe_work(which, iters, chunks) * reps / (ms * 1e-3) : 0.0;
  return NYS_OK;
}

}  // namespace nys
