// Device-side building blocks of the matrix-free kernel product K V.
//
// K_ij = k(x_i, x_j) is never stored (section "Positive-Definite Linear
// Systems": CG on a dense kernel system costs O(n^2) per iteration; eq.
// rlaopt-krr defines K).  Every 16 x 16 block of K is rebuilt on the fly:
//
//   1. one MFMA chain over the packed, augmented coordinates gives the
//      exponent t_ij = kappa (2 x_i.x_j - |x_i|^2 - |x_j|^2) of a block,
//      transposed (rows j, columns i) so that each lane ends up owning one row
//      i of K and four of its columns j;
//   2. an elementwise epilogue turns t into k (RBF: exp2(min(t, 0)) with
//      log2(e)/(2 sigma^2) folded into kappa; Laplacian: exp2(-c sqrt(-t)));
//   3. the block is contracted with V, either by per-lane FMAs and a
//      cross-lane reduction (few columns) or by a second MFMA (many columns).
#pragma once

#include "nys_internal.h"

namespace nys {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16;

// ------------------------------------------------------------------ bf16
__host__ __device__ inline u16 bf16_bits_rne(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (u16)(u >> 16);
}
__host__ __device__ inline float bf16_bits_to_f(u16 h) {
  return __builtin_bit_cast(float, (uint32_t)h << 16);
}

// ------------------------------------------------------------------ traits
template <int PREC> struct Tr;
template <> struct Tr<NYS_FP64> {
  using E = double;   // packed element
  using F = double;   // epilogue / accumulation scalar
  using Acc = d4;     // MFMA accumulator (16x16 block, 4 per lane)
  using Op = double;  // MFMA operand per lane
  static constexpr int KSTEP = 4;  // K per MFMA
  static constexpr int KL = 1;     // K elements per lane per MFMA
};
template <> struct Tr<NYS_FP32> {
  using E = float;
  using F = float;
  using Acc = f4;
  using Op = float;
  static constexpr int KSTEP = 4;
  static constexpr int KL = 1;
};
template <> struct Tr<NYS_BF16X3> {
  using E = u16;
  using F = float;
  using Acc = f4;
  using Op = bf8;
  static constexpr int KSTEP = 32;
  static constexpr int KL = 8;
};

__device__ inline f4 mfma16(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f4 mfma16(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ inline f4 mfma16(h8 a, h8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// Row of element v (0..3) of a 16x16 MFMA result held by lane group grp = lane/16
// (the column is lane % 16).  The float32 and bf16 instructions place rows
// 4 grp + v in a lane; the float64 instruction interleaves them as grp + 4 v.
template <int PREC>
__device__ inline int out_row(int grp, int v) {
  if constexpr (PREC == NYS_FP64) return grp + 4 * v;
  else return 4 * grp + v;
}

template <int PREC>
__device__ inline typename Tr<PREC>::Op load_op(const typename Tr<PREC>::E *p) {
  if constexpr (PREC == NYS_BF16X3) {
    return *reinterpret_cast<const bf8 *>(p);
  } else {
    return *p;
  }
}
template <int PREC>
__device__ inline typename Tr<PREC>::Op zero_op() {
  if constexpr (PREC == NYS_BF16X3) {
    bf8 z;
#pragma unroll
    for (int e = 0; e < 8; ++e) z[e] = (__bf16)0.0f;
    return z;
  } else {
    return 0;
  }
}

// LDS row stride (elements) of a staged tile of packed points: padded so that
// the 16 rows one MFMA operand touches fall into different banks.
template <int PREC>
__host__ __device__ inline int lds_stride(int Kp) {
  if constexpr (PREC == NYS_BF16X3) return Kp + 8;   // +16 bytes, keeps 16-byte alignment
  else return Kp + 1;                                // odd stride
}

// ------------------------------------------------------------------ epilogue
// t: exponent from the MFMA chain (kappa folded in).  FP64 uses natural units
// (kappa = 1/(2 sigma^2), cL = 1/sigma); FP32/BF16X3 use base-2 units
// (kappa = log2(e)/(2 sigma^2), cL = log2(e)/sigma) and the hardware exp2.
// deriv: dk/dsigma = k d^2 / sigma^3 (RBF) or k d / sigma^2 (Laplacian);
// dcoef = 1/(kappa sigma^3) resp. 1/sigma^2 converts -t or d into that factor.
template <int PREC, int KIND, int DERIV>
__device__ inline typename Tr<PREC>::F kernel_value(typename Tr<PREC>::F t,
                                                    typename Tr<PREC>::F cL,
                                                    typename Tr<PREC>::F dcoef) {
  using F = typename Tr<PREC>::F;
  if constexpr (PREC == NYS_FP64) {
    if constexpr (KIND == NYS_RBF) {
      F tt = t < 0.0 ? t : 0.0;
      F k = exp(tt);
      if constexpr (DERIV) k *= (-tt) * dcoef;
      return k;
    } else {
      F dist = sqrt(t < 0.0 ? -t : 0.0);
      F k = exp(-cL * dist);
      if constexpr (DERIV) k *= dist * dcoef;
      return k;
    }
  } else {
    // The exponent is -kappa |x - y|^2 up to rounding, so a positive t is a rounding
    // excess near the diagonal: exp2 of it differs from 1 by no more than that
    // rounding and needs no clamp (fminf would also cost a canonicalising max).  The
    // Laplacian's square root needs -t >= 0: one v_med3 clamps it.
    if constexpr (KIND == NYS_RBF) {
      F k = __builtin_amdgcn_exp2f(t);
      if constexpr (DERIV) k *= (-t) * dcoef;
      return k;
    } else {
      F dist = __builtin_sqrtf(__builtin_amdgcn_fmed3f(-t, 0.0f, 3.0e38f));
      F k = __builtin_amdgcn_exp2f(-cL * dist);
      if constexpr (DERIV) k *= dist * dcoef;
      return k;
    }
  }
}

// ------------------------------------------------------------------ float64 exp, t <= 0 (or a rounding excess above 0)
// exp(t) = 2^q 2^(j/64) e^r with k = 64 q + j = rint(64 t / ln 2) and
// r = t - k ln2/64, |r| <= ln2/128.  ln2/64 is split into a 36-bit head (k times it
// is exact for |k| < 2^17, so the first reduction step is exact) and a tail.
// 2^(j/64) is read from a 64-entry table in LDS (exp_tab_init); e^r - 1 is the
// Taylor polynomial to r^5, whose remainder r^6/720 is below 2^-54.  About one ulp
// of error against the rounded result; arguments below -1100 return 0 (exp
// underflows to zero below -745.2).  Twelve float64 operations and one LDS read
// against roughly twenty for a reduction by ln 2 alone.
__device__ inline void exp_tab_init(double *tab, int tid) {
  if (tid < 64) tab[tid] = exp2((double)tid * (1.0 / 64.0));
}
__device__ inline double exp_neg_tab(double t, const double *tab) {
  t = t < -1100.0 ? -1100.0 : t;                               // a NaN argument stays NaN
  const double kd = rint(t * 0x1.71547652b82fep+6);           // 64 / ln 2
  const int k = (int)kd;
  double r = fma(-kd, 0x1.62e42fefa0000p-7, t);                // head of ln2/64
  r = fma(-kd, 0x1.cf79abc9e3b3ap-46, r);                      // tail of ln2/64
  double q = fma(r, 1.0 / 120.0, 1.0 / 24.0);
  q = fma(r, q, 1.0 / 6.0);
  q = fma(r, q, 0.5);
  const double p = fma(r * r, q, r);                           // e^r - 1
  const double T = tab[k & 63];
  return ldexp(fma(T, p, T), k >> 6);
}
// kernel_value<NYS_FP64, ...> with the table exp.  RBF: a positive t is a rounding
// excess (the exponent is -kappa |x - y|^2), which exp_neg_tab evaluates as accurately
// as a negative one, so it is not clamped.
template <int KIND, int DERIV>
__device__ inline double kernel_value_tab(double t, double cL, double dcoef, const double *tab) {
  if constexpr (KIND == NYS_RBF) {
    double k = exp_neg_tab(t, tab);
    if constexpr (DERIV) k *= (-t) * dcoef;
    return k;
  } else {
    const double dist = sqrt(t > 0.0 ? 0.0 : -t);              // NaN stays NaN
    double k = exp_neg_tab(-cL * dist, tab);
    if constexpr (DERIV) k *= dist * dcoef;
    return k;
  }
}

// ------------------------------------------------------------------ launch args
struct KArgs {
  const void *Acols;   // packed column points (A operand rows j), [nc_pad][Kp]
  const void *Brows;   // packed row points (B operand rows i), [nr_pad][Kp]
  const void *V;       // small path / FP32,FP64 flash: V (nc x m, ldv); BF16 flash: V hi
  const void *V2;      // BF16 flash: V lo
  const float *vscale; // fp16 product: per-column factor undoing the power-of-two scaling of V
  void *Out;           // nr x m (ldo) or partial [split][nr][m]
  int64_t nr, nc;
  int64_t m_pad;       // BF16 flash: width of the split V
  int Kp, m, ldv, ldo;
  int jsteps;          // j tiles per split
  int nsplit;
  int chunks;          // column chunks (flash)
  int same;            // row and column points are the same set
  int partial;         // write raw sums to the partial buffer
  double cL, dcoef, alpha, beta;
};

// Block index remap: blocks are dealt to the 8 XCDs round robin; give each
// XCD a contiguous range of logical tiles so that co-resident workgroups of
// one XCD share (column chunk, j split) and hit the same column tiles in L2.
__device__ inline int64_t xcd_logical_block(int64_t nb_padded) {
  int64_t b = blockIdx.x;
  int64_t per = nb_padded / 8;
  return (b % 8) * per + b / 8;
}

}  // namespace nys
