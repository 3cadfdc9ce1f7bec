// Host side of the kernel product: point packing, V splitting, launch planning
// and the ordered reduction of column splits.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "kmv_kernels.h"

namespace nys {

// ------------------------------------------------------------------ packing
// bf16 packings are padded to a whole number of 32-wide K-steps from {2, 4, 6, 8}: the
// tiles are instantiated per step count, so the distance chain has a fixed length
static int bf16_steps(int k) {
  const int ks = (int)ceil_div(k, 32);
  return ks <= 2 ? 2 : (ks <= 4 ? 4 : (ks <= 6 ? 6 : (ks <= 8 ? 8 : ks)));
}
int packed_kp(int d, int prec) {
  prec = packing_prec(prec);
  if (prec == NYS_BF16X3) return 32 * bf16_steps(3 * d + 6);
  if (prec == NYS_BF16X3_D6) return 32 * bf16_steps(6 * d + 6);
  if (prec == NYS_BF16X3_D10) return 32 * bf16_steps(10 * d + 8);
  return (int)round_up(d + 2, 4);
}
size_t packed_elem_bytes(int prec) {
  return prec == NYS_FP64 ? 8 : (prec == NYS_FP32 ? 4 : 2);
}

// Scale folded into the MFMA chain so that it directly produces the exponent.
double kernel_kappa(const nys_kernel &k, int prec) {
  const double log2e = 1.4426950408889634;
  if (k.kind == NYS_RBF) {
    double kap = 1.0 / (2.0 * k.sigma * k.sigma);
    return prec == NYS_FP64 ? kap : kap * log2e;
  }
  return 1.0;  // Laplacian: t = -d^2
}

size_t col_mean_partial_elems(int64_t n, int d) {
  int64_t nb = std::min<int64_t>(ceil_div(n, 1024), 512);
  return (size_t)std::max<int64_t>(nb, 1) * d;
}

__global__ void col_mean_partial_kernel(const double *X, int64_t n, int d, int64_t rows_per,
                                        double *partial) {
  // block b sums rows [b*rows_per, ...) for every column; threads stride rows
  __shared__ double red[256];
  const int64_t r0 = (int64_t)blockIdx.x * rows_per;
  const int64_t r1 = std::min<int64_t>(n, r0 + rows_per);
  for (int c = 0; c < d; ++c) {
    double s = 0.0;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) s += X[i * d + c];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * d + c] = red[0];
    __syncthreads();
  }
}

__global__ void col_mean_final_kernel(const double *partial, int nb, int d, int64_t n, double *mu) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= d) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += partial[(int64_t)b * d + c];
  mu[c] = s / (double)n;
}

int32_t launch_col_mean(const double *X, int64_t n, int d, double *mu, double *partial,
                        hipStream_t s) {
  int64_t nb = std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 1024), 512));
  int64_t rows_per = ceil_div(n, nb);
  hipLaunchKernelGGL(col_mean_partial_kernel, dim3((unsigned)nb), dim3(256), 0, s, X, n, d, rows_per,
                     partial);
  NYS_LAUNCH_CHECK();
  hipLaunchKernelGGL(col_mean_final_kernel, dim3((unsigned)ceil_div(d, 64)), dim3(64), 0, s, partial,
                     (int)nb, d, n, mu);
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}

// Split v (double) into n_parts bf16 terms with round-to-nearest-even each.
__device__ inline void split_bf16(double v, int parts, u16 *out) {
  double rem = v;
  for (int p = 0; p < parts; ++p) {
    u16 h = bf16_bits_rne((float)rem);
    out[p] = h;
    rem -= (double)bf16_bits_to_f(h);
  }
}

// Split products of the low-precision distance chain.  A distance operand a is
// split into NPART round-to-nearest bf16 parts a_0 + a_1 + ..., and the dot
// product keeps the NT products a_p b_q of total order p + q below NPART:
//   NT = 3  (two parts):   00, 10, 01
//   NT = 6  (three parts): 00, 01, 10, 02, 20, 11
//   NT = 10 (four parts):  00, 01, 10, 02, 20, 11, 03, 30, 12, 21
// The column side stores part p of its point in segment t, the row side part q.
template <int NT> struct SplitTerms;
template <> struct SplitTerms<3> {
  static constexpr int NPART = 2, NBIAS = 3;
  static constexpr int col[3] = {0, 1, 0}, row[3] = {0, 0, 1};
};
template <> struct SplitTerms<6> {
  static constexpr int NPART = 3, NBIAS = 3;
  static constexpr int col[6] = {0, 0, 1, 0, 2, 1}, row[6] = {0, 1, 0, 2, 0, 1};
};
template <> struct SplitTerms<10> {
  static constexpr int NPART = 4, NBIAS = 4;
  static constexpr int col[10] = {0, 0, 1, 0, 2, 1, 0, 3, 1, 2}, row[10] = {0, 1, 0, 2, 0, 1, 3, 0, 2, 1};
};

// One packed point per thread.  Column side: [2 kappa x | -kappa |x|^2 | 1],
// row side: [x | 1 | -kappa |x|^2], so that the dot product of a row point and a
// column point is the exponent kappa (2 x.y - |x|^2 - |y|^2) of the kernel.
// Points are centred on the column mean mu first (distances do not change).
// A point with a NaN or infinite coordinate (or a non-finite centre, from such a
// point among the column points) sets *bad.
template <int PREC, int SIDE, int NT = 3>
__global__ void pack_kernel(const double *X, int64_t n, int d, const double *mu, double kappa,
                            void *out, int Kp, int64_t n_pad, int *bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_pad) return;
  double s = 0.0;
  if (i < n) {
    for (int l = 0; l < d; ++l) {
      double v = X[i * d + l] - mu[l];
      s += v * v;
    }
    if (!isfinite(s)) *bad = 1;
  }
  if constexpr (PREC == NYS_FP64 || PREC == NYS_FP32) {
    using E = typename Tr<PREC>::E;
    E *o = reinterpret_cast<E *>(out) + i * Kp;
    for (int k = 0; k < Kp; ++k) o[k] = 0;
    if (i < n) {
      for (int l = 0; l < d; ++l) {
        double v = X[i * d + l] - mu[l];
        o[l] = (E)(SIDE == SIDE_COL ? 2.0 * kappa * v : v);
      }
      if (SIDE == SIDE_COL) {
        o[d] = (E)(-kappa * s);
        o[d + 1] = (E)1.0;
      } else {
        o[d] = (E)1.0;
        o[d + 1] = (E)(-kappa * s);
      }
    }
  } else {
    using S = SplitTerms<NT>;
    u16 *o = reinterpret_cast<u16 *>(out) + i * Kp;
    for (int k = 0; k < Kp; ++k) o[k] = 0;
    if (i < n) {
      const u16 one = bf16_bits_rne(1.0f);
      u16 parts[S::NPART];
      for (int l = 0; l < d; ++l) {
        double v = X[i * d + l] - mu[l];
        split_bf16(SIDE == SIDE_COL ? 2.0 * kappa * v : v, S::NPART, parts);
#pragma unroll
        for (int t = 0; t < NT; ++t) o[t * d + l] = parts[SIDE == SIDE_COL ? S::col[t] : S::row[t]];
      }
      // the squared norms enter with NBIAS parts each, against ones on the other side:
      // column side [1 ... 1 | b_0 ... ], row side [a_0 ... | 1 ... 1]
      u16 b[S::NBIAS];
      split_bf16(-kappa * s, S::NBIAS, b);
      const int o0 = NT * d;
#pragma unroll
      for (int p = 0; p < S::NBIAS; ++p) {
        o[o0 + p] = SIDE == SIDE_COL ? one : b[p];
        o[o0 + S::NBIAS + p] = SIDE == SIDE_COL ? b[p] : one;
      }
    }
  }
}

int32_t launch_pack(const double *X, int64_t n, int d, const double *mu, const nys_kernel &k,
                    int prec, int side, Packed *out, int *bad, hipStream_t s) {
  prec = packing_prec(prec);
  const double kappa = kernel_kappa(k, prec);
  const int64_t n_pad = out->n_pad;
  dim3 grid((unsigned)ceil_div(n_pad, 128)), block(128);
#define NYS_PACK(P, S) hipLaunchKernelGGL((pack_kernel<P, S>), grid, block, 0, s, X, n, d, mu, kappa, out->data, out->Kp, n_pad, bad)
  if (prec == NYS_FP64) { if (side == SIDE_COL) NYS_PACK(NYS_FP64, SIDE_COL); else NYS_PACK(NYS_FP64, SIDE_ROW); }
  else if (prec == NYS_FP32) { if (side == SIDE_COL) NYS_PACK(NYS_FP32, SIDE_COL); else NYS_PACK(NYS_FP32, SIDE_ROW); }
  else if (prec == NYS_BF16X3) { if (side == SIDE_COL) NYS_PACK(NYS_BF16X3, SIDE_COL); else NYS_PACK(NYS_BF16X3, SIDE_ROW); }
  else if (prec == NYS_BF16X3_D6) {
    if (side == SIDE_COL)
      hipLaunchKernelGGL((pack_kernel<NYS_BF16X3, SIDE_COL, 6>), grid, block, 0, s, X, n, d, mu, kappa, out->data, out->Kp, n_pad, bad);
    else
      hipLaunchKernelGGL((pack_kernel<NYS_BF16X3, SIDE_ROW, 6>), grid, block, 0, s, X, n, d, mu, kappa, out->data, out->Kp, n_pad, bad);
  } else {
    if (side == SIDE_COL)
      hipLaunchKernelGGL((pack_kernel<NYS_BF16X3, SIDE_COL, 10>), grid, block, 0, s, X, n, d, mu, kappa, out->data, out->Kp, n_pad, bad);
    else
      hipLaunchKernelGGL((pack_kernel<NYS_BF16X3, SIDE_ROW, 10>), grid, block, 0, s, X, n, d, mu, kappa, out->data, out->Kp, n_pad, bad);
  }
#undef NYS_PACK
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}

// ------------------------------------------------------------------ V split
// V (nc x m float, ldv) -> hi/lo parts for the MFMA product with K.  For each block
// of 32 rows j and 16 columns c the parts are stored as [g][c % 16][e] (g < 4,
// e < 8: 512 elements): lane group g of the tile reads the eight rows that the
// exponent MFMA left in its registers, rows 4 g + e (e < 4) and 16 + 4 g + e - 4
// (e >= 4), and the 16 lanes of a group read 256 contiguous bytes.  One thread
// writes one 8-element run (16 bytes per part).
__device__ inline int vsplit_row(int g, int e) { return e < 4 ? 4 * g + e : 16 + 4 * g + (e - 4); }

template <bool F16>
__global__ void vsplit_kernel(const float *V, int ldv, int64_t nc, int m, int64_t m_pad, int64_t nblk,
                              const float *scale, u16 *hi, u16 *lo) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // over nblk * m_pad * 4 runs
  if (t >= nblk * m_pad * 4) return;
  const int c16 = (int)(t & 15);
  const int g = (int)((t >> 4) & 3);
  const int64_t rest = t >> 6;
  const int64_t cg = rest % (m_pad / 16);
  const int64_t jb = rest / (m_pad / 16);
  const int64_t c = cg * 16 + c16;
  const float sc = (F16 && c < m) ? scale[c] : 1.0f;
  u16 h[8], l[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int64_t j = jb * 32 + vsplit_row(g, e);
    const float v = (j < nc && c < m) ? V[j * ldv + c] * sc : 0.0f;
    if constexpr (F16) {
      const _Float16 hv = (_Float16)v;
      h[e] = __builtin_bit_cast(u16, hv);
      l[e] = __builtin_bit_cast(u16, (_Float16)(v - (float)hv));
    } else {
      h[e] = bf16_bits_rne(v);
      l[e] = bf16_bits_rne(v - bf16_bits_to_f(h[e]));
    }
  }
  const int64_t o = jb * m_pad * 32 + cg * 512 + g * 128 + c16 * 8;
  uint4 hv, lv;
  hv.x = h[0] | ((uint32_t)h[1] << 16); hv.y = h[2] | ((uint32_t)h[3] << 16);
  hv.z = h[4] | ((uint32_t)h[5] << 16); hv.w = h[6] | ((uint32_t)h[7] << 16);
  lv.x = l[0] | ((uint32_t)l[1] << 16); lv.y = l[2] | ((uint32_t)l[3] << 16);
  lv.z = l[4] | ((uint32_t)l[5] << 16); lv.w = l[6] | ((uint32_t)l[7] << 16);
  *reinterpret_cast<uint4 *>(hi + o) = hv;
  *reinterpret_cast<uint4 *>(lo + o) = lv;
}

// V (nc x m double, ldv) -> the float64 tile's layout: per 32-row tile jt and column
// chunk of tm, [h][v][cb][g][c % 16] holds V[32 jt + 16 h + 4 v + g][chunk tm + 16 cb + c % 16]
// (zero outside V).  Threads run in output order; 16 consecutive threads read 16
// consecutive columns.
__global__ void vperm64_kernel(const double *V, int ldv, int64_t nc, int m, int tm, int chunks, int64_t total,
                               double *Vp) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int c16 = (int)(idx & 15), g = (int)((idx >> 4) & 3);
  int64_t rest = idx >> 6;
  const int ncb = tm / 16;
  const int cb = (int)(rest % ncb);
  rest /= ncb;
  const int v = (int)(rest & 3), h = (int)((rest >> 2) & 1);
  rest >>= 3;
  const int chunk = (int)(rest % chunks);
  const int64_t jt = rest / chunks;
  const int64_t j = jt * 32 + 16 * h + 4 * v + g;
  const int64_t c = (int64_t)chunk * tm + cb * 16 + c16;
  Vp[idx] = (j < nc && c < m) ? V[j * ldv + c] : 0.0;
}

// fp16 product: per-column power-of-two scales.  Pass 1: max |V| of each column over
// a range of rows (threads run along the columns, so reads are coalesced).
constexpr int VMAX_BLOCKS = 128;
__global__ void col_absmax_partial_kernel(const float *V, int ldv, int64_t nc, int m, int64_t rows_per,
                                          float *partial) {
  const int c = blockIdx.y * blockDim.x + threadIdx.x;
  if (c >= m) return;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per;
  const int64_t r1 = r0 + rows_per < nc ? r0 + rows_per : nc;
  float mx = 0.0f;
  for (int64_t j = r0; j < r1; ++j) mx = fmaxf(mx, fabsf(V[j * ldv + c]));
  partial[(int64_t)blockIdx.x * m + c] = mx;
}
// Pass 2: scale[c] = 2^-e with max |V[:, c]| = f 2^e, f in [0.5, 1) (1 for a zero
// column), and its inverse for the output.
__global__ void col_scale_kernel(const float *partial, int nb, int m, float *scale, float *iscale) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= m) return;
  float mx = 0.0f;
  for (int b = 0; b < nb; ++b) mx = fmaxf(mx, partial[(int64_t)b * m + c]);
  int e = 0;
  if (mx > 0.0f && mx <= 3.0e38f) (void)frexpf(mx, &e);
  scale[c] = ldexpf(1.0f, -e);
  iscale[c] = ldexpf(1.0f, e);
}

// ------------------------------------------------------------------ split reduce
template <class F>
__global__ void split_reduce_kernel(const F *partial, int splits, int64_t nr, int m, F *Out, int ldo,
                                    double alpha, double beta) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nr * m) return;
  const int64_t i = idx / m;
  const int c = (int)(idx - i * m);
  double s = 0.0;
  for (int z = 0; z < splits; ++z) s += (double)partial[(int64_t)z * nr * m + idx];
  double v = alpha * s;
  if (beta != 0.0) v += beta * (double)Out[i * ldo + c];
  Out[i * ldo + c] = (F)v;
}

// ------------------------------------------------------------------ planning
// Tile widths chosen by the autotuner (nys_autotune / nys_set_tile), per original
// precision and column-count range.  kmv_plan takes the chunk width from here.
namespace {
std::mutex g_tune_mu;
struct Tuned {
  int prec, m_lo, m_hi, tm;
};
std::vector<Tuned> g_tuned;
}  // namespace

bool kmv_tile_valid(int prec, int tm) {
  switch (prec) {
    case NYS_FP64: return tm == 16 || tm == 32 || tm == 48 || tm == 64 || tm == 96 || tm == 128 || tm == 256;
    case NYS_FP32: return tm == 32 || tm == 64 || tm == 128;
    case NYS_F16X3_D10:
    case NYS_F16X3_D6: return tm == 16 || tm == 32 || tm == 64 || tm == 128 || tm == 256;
    default: return tm == 32 || tm == 64 || tm == 128 || tm == 256;
  }
}
void kmv_tune_set(int prec, int m_lo, int m_hi, int tm) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  std::vector<Tuned> keep;
  for (const Tuned &t : g_tuned)
    if (t.prec != prec || t.m_hi < m_lo || t.m_lo > m_hi) keep.push_back(t);
  if (tm > 0) keep.push_back(Tuned{prec, m_lo, m_hi, tm});
  g_tuned.swap(keep);
}
// Per-chunk cost of each float64 width (seconds, relative values are what matter),
// measured at n = 1e6, d = 16 until nys_autotune measures the shape at hand.
constexpr int kF64Widths[7] = {16, 32, 48, 64, 96, 128, 256};
// points per float32 accumulator range and the HBM the partial sums may take (kmv_plan)
constexpr int64_t kAccPoints = 16384;
constexpr size_t kMaxPartialBytes = size_t(32) << 30;
constexpr double kF64CostDefault[7] = {1.57, 2.00, 2.50, 2.98, 3.94, 4.63, 8.55};
double g_f64_cost[7] = {1.57, 2.00, 2.50, 2.98, 3.94, 4.63, 8.55};
void kmv_f64_cost_set(const double *c) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (int t = 0; t < 7; ++t) g_f64_cost[t] = c[t];
}
void kmv_tune_clear() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned.clear();
  for (int t = 0; t < 7; ++t) g_f64_cost[t] = kF64CostDefault[t];
}
std::vector<std::array<int, 4>> kmv_tune_snapshot() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  std::vector<std::array<int, 4>> out;
  for (const Tuned &t : g_tuned) out.push_back({t.prec, t.m_lo, t.m_hi, t.tm});
  return out;
}
void kmv_tune_restore(const std::vector<std::array<int, 4>> &t) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned.clear();
  for (const auto &e : t) g_tuned.push_back(Tuned{e[0], e[1], e[2], e[3]});
}
static int kmv_tune_get(int prec, int m) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const Tuned &t : g_tuned)
    if (t.prec == prec && m >= t.m_lo && m <= t.m_hi) return t.tm;
  return 0;
}

static int small_r_for(int prec, int mm) {
  if (prec == NYS_FP64) return mm <= 2 ? 4 : 2;
  return mm <= 4 ? 4 : 2;
}

KmvPlan kmv_plan(int64_t nr, int64_t nc, int m, int prec, int Kp) {
  (void)Kp;
  const bool f16v = f16_product(prec);
  const int prec0 = prec;
  prec = kernel_prec(prec);
  KmvPlan p;
  // float64: the pipelined tile beats the row-sum tile from 5 columns on (16-column
  // chunks); the fp16-product tile (16-column chunk) beats it at every width
  const int mm_cap = prec == NYS_FP64 ? 4 : (f16v ? 0 : 16);
  if (m <= mm_cap) {
    p.path = 0;
    p.mm = 1;
    while (p.mm < m) p.mm *= 2;
    p.r = small_r_for(prec, p.mm);
  } else {
    p.path = 1;
    if (prec == NYS_BF16X3) {
      p.tm = m <= 32 ? (f16v && m <= 16 ? 16 : 32) : (m <= 64 ? 64 : (m <= 128 ? 128 : 256));
      p.r = 2;
    } else if (prec == NYS_FP32) {
      p.tm = m <= 32 ? 32 : (m <= 64 ? 64 : 128);
      p.r = 2;
    } else {
      // float64: the chunk width with the least cost over its full chunks plus the
      // narrowest chunk that holds the remainder, from the per-chunk cost table (every
      // chunk recomputes the exponents; nys_autotune re-measures the table)
      const int *tms = kF64Widths;
      double cost[7];
      {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (int t = 0; t < 7; ++t) cost[t] = g_f64_cost[t];
      }
      double best = 1e300;
      for (int t = 0; t < 7; ++t) {
        const int64_t full = ceil_div(m, tms[t]) - 1;
        const int64_t rem = m - full * tms[t];
        int u = 0;
        while (tms[u] < rem) ++u;
        const double c = (double)full * cost[t] + cost[u];
        if (c < best) {
          best = c;
          p.tm = tms[t];
        }
      }
      p.r = 2;
    }
    const int tuned = kmv_tune_get(tile_key(prec0), m);
    if (tuned > 0) p.tm = tuned;
    // float64: 48-, 64- and 256-column chunks take one 16-row block per wave (four
    // waves per SIMD up to 64 columns; 256 columns within the register budget).
    // Measured at n = 1e6: 64 columns 2.98 s against 3.23 s with two blocks, 256
    // columns 8.6 s against 9.4 s for two 128-column chunks; 128 columns are faster
    // with two blocks (4.83 s against 5.06 s).
    if (prec == NYS_FP64) p.r = p.tm == 48 || p.tm == 64 || p.tm == 256 ? 1 : 2;
    // BF16X3 chunks of >= 64 columns run on the pipelined eight-wave tile; the fp16
    // product exists only there (every chunk width)
    if (prec == NYS_BF16X3 && p.tm >= 64 && p.r == 2) p.waves = 8;
    if (f16v) {
      p.r = 2;
      p.waves = 8;
      p.f16v = 1;
    }
    // float64 chunks run on the pipelined eight-wave float64 tile
    if (prec == NYS_FP64) p.waves = 8;
  }
  if (p.path == 0 || p.waves != 8) {
    p.waves = 4;
  }
  const int TI = p.waves * p.r * 16;
  const int TJ = p.path == 0 ? 64 : 32;
  const int64_t ntiles = ceil_div(nr, TI);
  const int chunks = p.path == 0 ? 1 : (int)ceil_div(m, p.tm);
  const int64_t njt = ceil_div(nc, TJ);
  // enough workgroups to fill 256 CUs several times over; each split keeps >= 8 tiles
  int64_t want = ceil_div(2048, ntiles * chunks);
  int64_t splits = std::max<int64_t>(1, std::min<int64_t>(want, njt / 8));
  // Accumulation length of the float32 tiles.  One MFMA accumulator adds a tile's
  // contribution per column tile, so its rounding error grows with the number of
  // points it sums (5e-6 relative for the row sums of K at n = 1e6 in one range).  In a
  // solve at small lambda that error, times an iterate of norm up to |b| / lambda,
  // becomes the drift between the recursive and the true residual.  The points are
  // therefore split into ranges of at most kAccPoints, each summed in float32 and the
  // ranges added in float64 (split_reduce_kernel), as far as kMaxPartialBytes of
  // partial sums allow.  float64 tiles accumulate in float64 and keep one range.
  if (prec != NYS_FP64) {
    const int64_t acc = ceil_div(njt, std::max<int64_t>(1, kAccPoints / TJ));
    const int64_t cap = std::max<int64_t>(1, (int64_t)(kMaxPartialBytes / ((size_t)std::max<int64_t>(nr, 1) *
                                                                           (size_t)std::max(m, 1) * 4)));
    splits = std::max(splits, std::min(acc, cap));
  }
  p.jsteps = (int)ceil_div(njt, splits);
  p.splits = (int)ceil_div(njt, p.jsteps);
  p.m_pad = p.path == 1 ? (int64_t)chunks * p.tm : 0;
  // the last chunk takes the narrowest width that holds the remaining columns (a
  // second launch; every chunk recomputes the exponents, so a narrower one is cheaper)
  if (p.path == 1 && chunks > 1) {
    const int rem = m - (chunks - 1) * p.tm;
    const int key = tile_key(prec0);
    for (int t : {16, 32, 48, 64, 96, 128, 256}) {
      if (t >= p.tm) break;
      if (t >= rem && kmv_tile_valid(key, t)) {
        p.tail_tm = t;
        break;
      }
    }
  }
  return p;
}

// The plan of the last chunk of a plan with a narrower tail: same precision path and
// column splits, one chunk of tail_tm columns.
static KmvPlan tail_plan(const KmvPlan &p, int prec) {
  KmvPlan t = p;
  t.tm = p.tail_tm;
  t.tail_tm = 0;
  t.m_pad = t.tm;
  prec = kernel_prec(prec);
  if (prec == NYS_FP64) {
    t.r = t.tm == 48 || t.tm == 64 || t.tm == 256 ? 1 : 2;
    t.waves = 8;
  } else if (prec == NYS_BF16X3 && !p.f16v) {
    t.r = 2;
    t.waves = t.tm >= 64 ? 8 : 4;
  }
  return t;
}

void kmv_scratch_sizes(const KmvPlan &p, int64_t nr, int64_t nc, int m, int prec,
                       size_t *partial_bytes, size_t *vsplit_elems, size_t *vlo_elems) {
  prec = kernel_prec(prec);
  const size_t fb = prec == NYS_FP64 ? 8 : 4;
  *partial_bytes = p.splits > 1 ? (size_t)p.splits * nr * m * fb : 0;
  *vsplit_elems = *vlo_elems = 0;
  if (p.path == 1 && prec == NYS_BF16X3) {
    *vsplit_elems = (size_t)ceil_div(nc, 32) * p.m_pad * 32;
    // fp16 product: column maxima and scales (floats) follow the split V in the lo part
    *vlo_elems = *vsplit_elems + (p.f16v ? 2 * (size_t)(VMAX_BLOCKS + 2) * m : 0);
  } else if (p.path == 1 && prec == NYS_FP64 && p.waves == 8) {
    *vsplit_elems = 4 * (size_t)ceil_div(nc, 32) * p.m_pad * 32;   // permuted V, doubles as 4 u16
  }
}

void kmv_reserve(const KmvPlan &p, int64_t nr, int64_t nc, int m, int prec, Arena &ws,
                 void **partial, void **vhi, void **vlo) {
  size_t pb, ve, vl;
  kmv_scratch_sizes(p, nr, nc, m, prec, &pb, &ve, &vl);
  *partial = nullptr;
  *vhi = *vlo = nullptr;
  if (pb) *partial = ws.take<char>(pb);
  if (ve) *vhi = ws.take<u16>(ve);
  if (vl) *vlo = ws.take<u16>(vl);
}

static int ksmax_for(int prec, int Kp) {
  if (kernel_prec(prec) == NYS_BF16X3) {
    const int ks = Kp / 32;   // packed_kp pads to one of the instantiated step counts
    return (ks == 2 || ks == 4 || ks == 6 || ks == 8) && Kp == 32 * ks ? ks : -1;
  }
  int ks = Kp / 4;
  return ks <= 8 ? 8 : (ks <= 16 ? 16 : -1);
}

int32_t kmv_run(const KmvPlan &plan, const nys_kernel &k, int deriv, int prec, const Packed &rows,
                const Packed &cols, int same_points, const void *V, int m, int ldv, void *Out,
                int ldo, double alpha, double beta, void *partial, void *vhi, void *vlo,
                hipStream_t s) {
  if (m <= 0 || rows.n <= 0) return NYS_OK;
  if (plan.path == 1 && plan.tail_tm > 0 && !deriv) {
    // full chunks, then the narrower last chunk as a launch of its own
    const int m1 = (int)(ceil_div(m, plan.tm) - 1) * plan.tm;
    KmvPlan head = plan;
    head.tail_tm = 0;
    head.m_pad = m1;
    NYS_RETURN_IF(kmv_run(head, k, deriv, prec, rows, cols, same_points, V, m1, ldv, Out, ldo, alpha, beta,
                          partial, vhi, vlo, s));
    const size_t eb = kernel_prec(prec) == NYS_FP64 ? 8 : 4;
    return kmv_run(tail_plan(plan, prec), k, deriv, prec, rows, cols, same_points,
                   reinterpret_cast<const char *>(V) + (size_t)m1 * eb, m - m1, ldv,
                   reinterpret_cast<char *>(Out) + (size_t)m1 * eb, ldo, alpha, beta, partial, vhi, vlo, s);
  }
  prec = kernel_prec(prec);
  const int ksmax = ksmax_for(prec, rows.Kp);
  if (ksmax < 0) {
    set_error("kernel_matvec: dimension too large for the tile kernels");
    return NYS_EINVAL;
  }
  if (deriv && plan.path != 0) {
    set_error("kernel_matvec: derivative product needs the small-m path");
    return NYS_EINVAL;
  }
  KArgs a{};
  a.Acols = cols.data;
  a.Brows = rows.data;
  a.V = V;
  a.Out = plan.splits > 1 ? partial : Out;
  a.nr = rows.n;
  a.nc = cols.n;
  a.Kp = rows.Kp;
  a.m = m;
  a.ldv = ldv;
  a.ldo = plan.splits > 1 ? m : ldo;
  a.jsteps = plan.jsteps;
  a.nsplit = plan.splits;
  a.same = same_points;
  a.partial = plan.splits > 1;
  a.alpha = alpha;
  a.beta = beta;
  const double log2e = 1.4426950408889634;
  if (k.kind == NYS_RBF) {
    double kap = kernel_kappa(k, prec);
    a.cL = 0.0;
    a.dcoef = 1.0 / (kap * k.sigma * k.sigma * k.sigma);
  } else {
    a.cL = prec == NYS_FP64 ? 1.0 / k.sigma : log2e / k.sigma;
    a.dcoef = 1.0 / (k.sigma * k.sigma);
  }
  const int TI = plan.waves * plan.r * 16;
  const int64_t ntiles = ceil_div(rows.n, TI);
  int chunks = 1;
  if (plan.path == 1) {
    chunks = (int)ceil_div(m, plan.tm);
    a.chunks = chunks;
    if (prec == NYS_BF16X3 && plan.f16v) {
      const int64_t nblk = ceil_div(cols.n, 32);
      const int64_t total = nblk * plan.m_pad * 32;
      float *fs = reinterpret_cast<float *>(reinterpret_cast<u16 *>(vlo) + total);
      float *vpart = fs, *scale = fs + (size_t)VMAX_BLOCKS * m, *iscale = scale + m;
      const int nbm = (int)std::max<int64_t>(1, std::min<int64_t>(VMAX_BLOCKS, ceil_div(cols.n, 4096)));
      const int64_t rows_per = ceil_div(cols.n, nbm);
      hipLaunchKernelGGL(col_absmax_partial_kernel, dim3((unsigned)nbm, (unsigned)ceil_div(m, 256)), dim3(256), 0,
                         s, reinterpret_cast<const float *>(V), ldv, cols.n, m, rows_per, vpart);
      NYS_LAUNCH_CHECK();
      hipLaunchKernelGGL(col_scale_kernel, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, s, vpart, nbm, m,
                         scale, iscale);
      NYS_LAUNCH_CHECK();
      hipLaunchKernelGGL(vsplit_kernel<true>, dim3((unsigned)ceil_div(total / 8, 256)), dim3(256), 0, s,
                         reinterpret_cast<const float *>(V), ldv, cols.n, m, plan.m_pad, nblk, scale,
                         reinterpret_cast<u16 *>(vhi), reinterpret_cast<u16 *>(vlo));
      NYS_LAUNCH_CHECK();
      a.V = vhi;
      a.V2 = vlo;
      a.vscale = iscale;
      a.m_pad = plan.m_pad;
    } else if (prec == NYS_FP64 && plan.waves == 8) {
      const int64_t total = ceil_div(cols.n, 32) * 32 * plan.m_pad;
      hipLaunchKernelGGL(vperm64_kernel, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, s,
                         reinterpret_cast<const double *>(V), ldv, cols.n, m, plan.tm, chunks, total,
                         reinterpret_cast<double *>(vhi));
      NYS_LAUNCH_CHECK();
      a.V = vhi;
      a.m_pad = plan.m_pad;
    } else if (prec == NYS_BF16X3) {
      const int64_t nblk = ceil_div(cols.n, 32);
      const int64_t total = nblk * plan.m_pad * 32;
      hipLaunchKernelGGL(vsplit_kernel<false>, dim3((unsigned)ceil_div(total / 8, 256)), dim3(256), 0, s,
                         reinterpret_cast<const float *>(V), ldv, cols.n, m, plan.m_pad, nblk, nullptr,
                         reinterpret_cast<u16 *>(vhi), reinterpret_cast<u16 *>(vlo));
      NYS_LAUNCH_CHECK();
      a.V = vhi;
      a.V2 = vlo;
      a.m_pad = plan.m_pad;
    }
  } else {
    a.chunks = 1;
  }
  const int64_t nb = ntiles * chunks * plan.splits;
  const int64_t nb_pad = round_up(nb, 8);
  if (nb_pad > 0x7fffffffLL) {
    set_error("kernel_matvec: grid too large");
    return NYS_EINVAL;
  }
  dim3 grid((unsigned)nb_pad);
  int32_t rc;
  if (prec == NYS_FP64 && plan.path == 1 && plan.waves == 8) rc = kmv_dispatch_f64p(plan, k.kind, deriv, ksmax, a, grid, s);
  else if (prec == NYS_FP64) rc = kmv_dispatch_f64(plan, k.kind, deriv, ksmax, a, grid, s);
  else if (prec == NYS_FP32) rc = kmv_dispatch_f32(plan, k.kind, deriv, ksmax, a, grid, s);
  else if (plan.path == 1 && plan.f16v) rc = kmv_dispatch_f16(plan, k.kind, deriv, ksmax, a, grid, s);
  else rc = kmv_dispatch_bf16(plan, k.kind, deriv, ksmax, a, grid, s);
  NYS_RETURN_IF(rc);
  NYS_LAUNCH_CHECK();
  if (plan.splits > 1) {
    const int64_t total = rows.n * (int64_t)m;
    if (prec == NYS_FP64)
      hipLaunchKernelGGL(split_reduce_kernel<double>, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, s,
                         reinterpret_cast<const double *>(partial), plan.splits, rows.n, m,
                         reinterpret_cast<double *>(Out), ldo, alpha, beta);
    else
      hipLaunchKernelGGL(split_reduce_kernel<float>, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, s,
                         reinterpret_cast<const float *>(partial), plan.splits, rows.n, m,
                         reinterpret_cast<float *>(Out), ldo, alpha, beta);
    NYS_LAUNCH_CHECK();
  }
  return NYS_OK;
}

}  // namespace nys
