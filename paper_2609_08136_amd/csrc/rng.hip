// Gaussian test matrix of the Nystrom sketch drawn on the device: a counter-based
// generator, so every element is a pure function of (seed, index) and any row
// range can be produced anywhere without communication.
//
// Uniform bits: Philox4x32 with 10 rounds (Salmon, Moraes, Dror and Shaw, "Parallel
// random numbers: as easy as 1, 2, 3", SC 2011).  One round maps the counter
// (c0, c1, c2, c3) under the key (k0, k1) to
//     (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0))
// with M0 = 0xD2511F53, M1 = 0xCD9E8D57 and hi/lo the halves of the 64-bit
// product; the key is advanced by the Weyl constants (0x9E3779B9, 0xBB67AE85)
// between rounds.
// Normals: element e of the row-major n x r matrix uses block b = e / 2, counter
// (b mod 2^32, b / 2^32, 0, 0), key (seed mod 2^32, seed / 2^32).  The four output
// words give two uniforms in (0, 1) with 53 random bits each,
//     u = ((w0 2^32 + w1) / 2^11 + 1/2) 2^-53,   v likewise from (w2, w3),
// and the Box-Muller pair sqrt(-2 ln u) (cos 2 pi v, sin 2 pi v); even e takes the
// cosine, odd e the sine.
#include "nys_internal.h"

namespace nys {
namespace {

struct Philox {
  uint32_t w[4];
};

__device__ inline Philox philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                       uint32_t k1) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint32_t hi0 = __umulhi(M0, c0), lo0 = M0 * c0;
    const uint32_t hi1 = __umulhi(M1, c2), lo1 = M1 * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  return Philox{{c0, c1, c2, c3}};
}

__device__ inline double unit_open(uint32_t hi, uint32_t lo) {
  const uint64_t x = (((uint64_t)hi << 32) | lo) >> 11;         // 53 bits
  return ((double)x + 0.5) * 0x1.0p-53;
}

__global__ void gaussian_kernel(uint64_t seed, int64_t count, double *out) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // one block = two elements
  if (2 * b >= count) return;
  const Philox p = philox4x32_10((uint32_t)b, (uint32_t)((uint64_t)b >> 32), 0u, 0u, (uint32_t)seed,
                                 (uint32_t)(seed >> 32));
  const double u = unit_open(p.w[0], p.w[1]);
  const double v = unit_open(p.w[2], p.w[3]);
  const double rad = sqrt(-2.0 * log(u));
  const double ang = 2.0 * 3.141592653589793 * v;
  out[2 * b] = rad * cos(ang);
  if (2 * b + 1 < count) out[2 * b + 1] = rad * sin(ang);
}

}  // namespace

int32_t launch_gaussian(uint64_t seed, int64_t count, double *out, hipStream_t s) {
  if (count <= 0) return NYS_OK;
  const int64_t blocks = (count + 1) / 2;
  hipLaunchKernelGGL(gaussian_kernel, dim3((unsigned)ceil_div(blocks, 256)), dim3(256), 0, s, seed, count, out);
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}

}  // namespace nys
