// Kernel-product tile kernels (templates; instantiated per precision).
#pragma once

#include "kmv_common.h"

namespace nys {

constexpr int KMV_THREADS = 256;  // 4 wave64s per workgroup

// Stage `rows` packed rows starting at row j0 into LDS with padded stride.
template <int PREC>
__device__ inline void stage_points(typename Tr<PREC>::E *sA, int strideA,
                                    const typename Tr<PREC>::E *src, int64_t j0, int Kp,
                                    int rows) {
  using E = typename Tr<PREC>::E;
  const int tid = threadIdx.x;
  if constexpr (PREC == NYS_BF16X3) {
    // 16-byte chunks: Kp/8 per row (Kp is a multiple of 32).
    const int cpr = Kp / 8;
    const uint4 *g = reinterpret_cast<const uint4 *>(src + j0 * Kp);
    for (int c = tid; c < rows * cpr; c += KMV_THREADS) {
      int r = c / cpr, o = c - r * cpr;
      *reinterpret_cast<uint4 *>(sA + r * strideA + o * 8) = g[c];
    }
  } else {
    const E *g = src + j0 * Kp;
    for (int e = tid; e < rows * Kp; e += KMV_THREADS) {
      int r = e / Kp, o = e - r * Kp;
      sA[r * strideA + o] = g[e];
    }
  }
}

// ===================================================================== small m
// Out_i,c = sum_j k(x_i, x_j) V_j,c for m <= MM.  Workgroup: 4 waves, each wave
// R row blocks of 16 (TI = 64 R rows).  Per column tile of TJ = 64 points: stage
// the packed points and V rows in LDS, then per 16-column sub-block and row block
// one MFMA chain gives the transposed exponent block; lane (col16, grp) owns row
// i = col16 and columns j = out_row(grp, q), q < 4, and accumulates k_ij V_j,c in
// registers.  A 4-way cross-lane reduction at the end yields the row sums.
template <int PREC, int KIND, int DERIV, int KSMAX, int MM, int R>
__global__ __launch_bounds__(KMV_THREADS, 2) void kmv_small_kernel(KArgs a) {
  using T = Tr<PREC>;
  using E = typename T::E;
  using F = typename T::F;
  using Acc = typename T::Acc;
  using Op = typename T::Op;
  constexpr int TJ = 64;
  constexpr int TI = 4 * R * 16;

  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int strideA = lds_stride<PREC>(a.Kp);
  E *sA = reinterpret_cast<E *>(smem);
  const size_t a_bytes = ((size_t)TJ * strideA * sizeof(E) + 15) & ~size_t(15);
  F *sV = reinterpret_cast<F *>(smem + a_bytes);
  double *const tab = reinterpret_cast<double *>(sV + TJ * MM);   // float64: 2^(j/64), j < 64

  const int64_t ntiles = (a.nr + TI - 1) / TI;
  const int64_t nb = ntiles * a.nsplit;
  const int64_t nb_pad = (nb + 7) / 8 * 8;
  const int64_t lid = xcd_logical_block(nb_pad);
  if (lid >= nb) return;
  const int64_t tile = lid % ntiles;
  const int split = (int)(lid / ntiles);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col16 = lane & 15, grp = lane >> 4;
  // bf16 packings are padded to exactly KSMAX K-steps, so the chain length is a constant
  // there; float64 tiles with KSMAX below 8 are instantiated per exact step count
  const int ks = (PREC == NYS_BF16X3 || (PREC == NYS_FP64 && KSMAX < 8)) ? KSMAX : a.Kp / T::KSTEP;
  if constexpr (PREC == NYS_FP64) exp_tab_init(tab, tid);   // visible after the first barrier
  const int64_t i0 = tile * TI;
  const int64_t iw = i0 + (int64_t)wave * R * 16;
  const E *Ag = reinterpret_cast<const E *>(a.Acols);
  const E *Bg = reinterpret_cast<const E *>(a.Brows);
  const F *Vg = reinterpret_cast<const F *>(a.V);

  Op bop[R][KSMAX];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int s = 0; s < KSMAX; ++s)
      bop[r][s] = (s < ks) ? load_op<PREC>(Bg + (iw + r * 16 + col16) * a.Kp + s * T::KSTEP + grp * T::KL)
                           : zero_op<PREC>();

  F acc[R][MM];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int c = 0; c < MM; ++c) acc[r][c] = 0;

  const F cL = (F)a.cL, dcoef = (F)a.dcoef;
  const int64_t njt = (a.nc + TJ - 1) / TJ;
  const int64_t jt0 = (int64_t)split * a.jsteps;
  const int64_t jt1 = jt0 + a.jsteps < njt ? jt0 + a.jsteps : njt;

  for (int64_t jt = jt0; jt < jt1; ++jt) {
    const int64_t j0 = jt * TJ;
    __syncthreads();
    stage_points<PREC>(sA, strideA, Ag, j0, a.Kp, TJ);
    for (int e = tid; e < TJ * MM; e += KMV_THREADS) {
      int jj = e / MM, c = e - jj * MM;
      int64_t j = j0 + jj;
      sV[e] = (j < a.nc && c < a.m) ? Vg[j * a.ldv + c] : (F)0;
    }
    __syncthreads();
    const bool diag = a.same && (j0 < i0 + TI) && (i0 < j0 + TJ);

    // float64: one sub-block at a time keeps the exponentials' table reads within
    // the register budget
    constexpr int JB_UNROLL = PREC == NYS_FP64 ? 1 : 2;
#pragma unroll JB_UNROLL
    for (int jb = 0; jb < TJ / 16; ++jb) {
      Op aop[KSMAX];
#pragma unroll
      for (int s = 0; s < KSMAX; ++s)
        aop[s] = (s < ks) ? load_op<PREC>(sA + (jb * 16 + col16) * strideA + s * T::KSTEP + grp * T::KL)
                          : zero_op<PREC>();
      F vv[4][MM];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int c = 0; c < MM; ++c) vv[q][c] = sV[(jb * 16 + out_row<PREC>(grp, q)) * MM + c];

#pragma unroll
      for (int r = 0; r < R; ++r) {
        Acc t = {0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < KSMAX; ++s)
          if (s < ks) t = mfma16(aop[s], bop[r][s], t);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          F tq = t[q];
          if (diag && (iw + r * 16 + col16 == j0 + jb * 16 + out_row<PREC>(grp, q))) tq = 0;
          F kv;
          if constexpr (PREC == NYS_FP64) kv = kernel_value_tab<KIND, DERIV>(tq, cL, dcoef, tab);
          else kv = kernel_value<PREC, KIND, DERIV>(tq, cL, dcoef);
#pragma unroll
          for (int c = 0; c < MM; ++c) acc[r][c] += kv * vv[q][c];
        }
      }
    }
  }

  // lanes col16, col16+16, col16+32, col16+48 hold partial sums of the same row
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int c = 0; c < MM; ++c) {
      F v = acc[r][c];
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      acc[r][c] = v;
    }
  if (grp == 0) {
    F *O = reinterpret_cast<F *>(a.Out);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t i = iw + r * 16 + col16;
      if (i < a.nr) {
#pragma unroll
        for (int c = 0; c < MM; ++c) {
          if (c < a.m) {
            if (a.partial) {
              O[((int64_t)split * a.nr + i) * a.m + c] = acc[r][c];
            } else {
              F v = (F)a.alpha * acc[r][c];
              if (a.beta != 0.0) v += (F)a.beta * O[i * a.ldo + c];
              O[i * a.ldo + c] = v;
            }
          }
        }
      }
    }
  }
}

// ===================================================================== flash
// Out_I,C += K_IJ V_J,C for a chunk C of TM columns.  Per column tile of TJ = 32
// points: two transposed exponent blocks per 16-row block i (MFMA chain 1),
// epilogue to k, then the 16 x 32 block of K is fed to a second MFMA against
// V_J,C.  The lane layout of chain 1's output (lane owns row i and columns
// j = 4 grp + q and 16 + 4 grp + q) is used as the A operand of chain 2 with
// the matching permutation of the rows of V, so no data moves between lanes.
//   BF16X3: k and V are split into bf16 hi/lo parts; K V ~ k_hi V_hi + k_hi V_lo
//           + k_lo V_hi (v_mfma_f32_16x16x32_bf16).  V arrives pre-split and
//           pre-permuted as [j/32][m_pad][32].
//   FP32/FP64: four K=4 MFMAs per 16x16 block of K.
template <int PREC, int KIND, int KSMAX, int R, int TM>
__global__ __launch_bounds__(KMV_THREADS, 2) void kmv_flash_kernel(KArgs a) {
  using T = Tr<PREC>;
  using E = typename T::E;
  using F = typename T::F;
  using Acc = typename T::Acc;
  using Op = typename T::Op;
  constexpr int TJ = 32;
  constexpr int TI = 4 * R * 16;
  constexpr int NCB = TM / 16;
  constexpr int VS = (PREC == NYS_FP32) ? TM + 4 : TM + 1;  // LDS row stride of V (FP32/FP64)

  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int strideA = lds_stride<PREC>(a.Kp);
  E *sA = reinterpret_cast<E *>(smem);
  const size_t a_bytes = ((size_t)TJ * strideA * sizeof(E) + 15) & ~size_t(15);
  unsigned char *sVraw = smem + a_bytes;

  const int64_t ntiles = (a.nr + TI - 1) / TI;
  const int64_t nb = ntiles * a.chunks * a.nsplit;
  const int64_t nb_pad = (nb + 7) / 8 * 8;
  const int64_t lid = xcd_logical_block(nb_pad);
  if (lid >= nb) return;
  const int64_t tile = lid % ntiles;
  const int64_t rest = lid / ntiles;
  const int chunk = (int)(rest % a.chunks);
  const int split = (int)(rest / a.chunks);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col16 = lane & 15, grp = lane >> 4;
  const int ks = PREC == NYS_BF16X3 ? KSMAX : a.Kp / T::KSTEP;   // bf16 packings: exactly KSMAX steps
  const int64_t i0 = tile * TI;
  const int64_t iw = i0 + (int64_t)wave * R * 16;
  const int c0 = chunk * TM;
  const E *Ag = reinterpret_cast<const E *>(a.Acols);
  const E *Bg = reinterpret_cast<const E *>(a.Brows);

  Op bop[R][KSMAX];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int s = 0; s < KSMAX; ++s)
      bop[r][s] = (s < ks) ? load_op<PREC>(Bg + (iw + r * 16 + col16) * a.Kp + s * T::KSTEP + grp * T::KL)
                           : zero_op<PREC>();

  Acc acc[R][NCB];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) acc[r][cb] = Acc{0, 0, 0, 0};

  const F cL = (F)a.cL, dcoef = (F)a.dcoef;
  const int64_t njt = (a.nc + TJ - 1) / TJ;
  const int64_t jt0 = (int64_t)split * a.jsteps;
  const int64_t jt1 = jt0 + a.jsteps < njt ? jt0 + a.jsteps : njt;

  for (int64_t jt = jt0; jt < jt1; ++jt) {
    const int64_t j0 = jt * TJ;
    __syncthreads();
    stage_points<PREC>(sA, strideA, Ag, j0, a.Kp, TJ);
    if constexpr (PREC == NYS_BF16X3) {
      // contiguous TM x 32 bf16 per part
      const uint4 *gh = reinterpret_cast<const uint4 *>(reinterpret_cast<const u16 *>(a.V) + (jt * a.m_pad + c0) * 32);
      const uint4 *gl = reinterpret_cast<const uint4 *>(reinterpret_cast<const u16 *>(a.V2) + (jt * a.m_pad + c0) * 32);
      uint4 *sh = reinterpret_cast<uint4 *>(sVraw);
      uint4 *sl = sh + TM * 4;
      for (int c = tid; c < TM * 4; c += KMV_THREADS) {
        sh[c] = gh[c];
        sl[c] = gl[c];
      }
    } else {
      F *sV = reinterpret_cast<F *>(sVraw);
      const F *Vg = reinterpret_cast<const F *>(a.V);
      for (int e = tid; e < TJ * TM; e += KMV_THREADS) {
        int jj = e / TM, c = e - jj * TM;
        int64_t j = j0 + jj;
        int cc = c0 + c;
        sV[jj * VS + c] = (j < a.nc && cc < a.m) ? Vg[j * a.ldv + cc] : (F)0;
      }
    }
    __syncthreads();
    const bool diag = a.same && (j0 < i0 + TI) && (i0 < j0 + TJ);

    Op aopA[KSMAX], aopB[KSMAX];
#pragma unroll
    for (int s = 0; s < KSMAX; ++s) {
      aopA[s] = (s < ks) ? load_op<PREC>(sA + col16 * strideA + s * T::KSTEP + grp * T::KL) : zero_op<PREC>();
      aopB[s] = (s < ks) ? load_op<PREC>(sA + (16 + col16) * strideA + s * T::KSTEP + grp * T::KL) : zero_op<PREC>();
    }

    if constexpr (PREC == NYS_BF16X3) {
      bf8 phi[R], plo[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        f4 ta = {0, 0, 0, 0}, tb = {0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < KSMAX; ++s)
          if (s < ks) {
            ta = mfma16(aopA[s], bop[r][s], ta);
            tb = mfma16(aopB[s], bop[r][s], tb);
          }
        const int64_t gi = iw + r * 16 + col16;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          float t = e < 4 ? ta[e] : tb[e - 4];
          const int64_t gj = j0 + (e < 4 ? 4 * grp + e : 16 + 4 * grp + (e - 4));
          if (diag && gi == gj) t = 0.0f;
          float kv = kernel_value<PREC, KIND, 0>(t, cL, dcoef);
          __bf16 h = (__bf16)kv;
          phi[r][e] = h;
          plo[r][e] = (__bf16)(kv - (float)h);
        }
      }
      const u16 *sh = reinterpret_cast<const u16 *>(sVraw);
      const u16 *sl = sh + TM * 32;
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        bf8 vh = *reinterpret_cast<const bf8 *>(sh + cb * 512 + grp * 128 + col16 * 8);
        bf8 vl = *reinterpret_cast<const bf8 *>(sl + cb * 512 + grp * 128 + col16 * 8);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          acc[r][cb] = mfma16(phi[r], vh, acc[r][cb]);
          acc[r][cb] = mfma16(phi[r], vl, acc[r][cb]);
          acc[r][cb] = mfma16(plo[r], vh, acc[r][cb]);
        }
      }
    } else {
      F pa[R][4], pb[R][4];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        Acc ta = {0, 0, 0, 0}, tb = {0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < KSMAX; ++s)
          if (s < ks) {
            ta = mfma16(aopA[s], bop[r][s], ta);
            tb = mfma16(aopB[s], bop[r][s], tb);
          }
        const int64_t gi = iw + r * 16 + col16;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          F t1 = ta[q], t2 = tb[q];
          if (diag && gi == j0 + out_row<PREC>(grp, q)) t1 = 0;
          if (diag && gi == j0 + 16 + out_row<PREC>(grp, q)) t2 = 0;
          pa[r][q] = kernel_value<PREC, KIND, 0>(t1, cL, dcoef);
          pb[r][q] = kernel_value<PREC, KIND, 0>(t2, cL, dcoef);
        }
      }
      const F *sV = reinterpret_cast<const F *>(sVraw);
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          F va = sV[out_row<PREC>(grp, q) * VS + cb * 16 + col16];
          F vb = sV[(16 + out_row<PREC>(grp, q)) * VS + cb * 16 + col16];
#pragma unroll
          for (int r = 0; r < R; ++r) {
            acc[r][cb] = mfma16(pa[r][q], va, acc[r][cb]);
            acc[r][cb] = mfma16(pb[r][q], vb, acc[r][cb]);
          }
        }
      }
    }
  }

  // chain-2 output layout: lane holds rows out_row(grp, v) of each 16-row block, column col16
  F *O = reinterpret_cast<F *>(a.Out);
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t i = iw + r * 16 + out_row<PREC>(grp, v);
        const int c = c0 + cb * 16 + col16;
        if (i < a.nr && c < a.m) {
          F s = acc[r][cb][v];
          if (a.partial) {
            O[((int64_t)split * a.nr + i) * a.m + c] = s;
          } else {
            F val = (F)a.alpha * s;
            if (a.beta != 0.0) val += (F)a.beta * O[i * a.ldo + c];
            O[i * a.ldo + c] = val;
          }
        }
      }
}

// ===================================================================== flash, pipelined (BF16X3)
// Eight waves (256 rows, 32 per wave) share one TM-column chunk of the split V.
// Column tiles of TJ = 32 points are double buffered in LDS: while the MFMAs
// consume tile t, the split V of tile t+1 streams into the other buffer by direct
// global-to-LDS loads (no registers) and the packed points of tile t+1 wait in
// registers; one barrier per tile.  Per tile and wave: 2 R KS MFMAs for the
// exponents, 3 R TM/16 for K V.
// F16V: the K V product splits K and V into fp16 parts instead of bf16 (V arrives
// scaled per column by a power of two, undone on output): 11 + 11 significand bits
// per operand instead of 8 + 8 at the same MFMA rate.
constexpr int KMV2_THREADS = 512;

template <bool F16V> struct ProdType { using V = bf8; using S = __bf16; };
template <> struct ProdType<true> { using V = h8; using S = _Float16; };

// The 16- and (RBF) 32-column tiles run four waves per SIMD (two workgroups per CU)
// within 128 registers; the 32-column one spills a few registers there and is still
// faster (517 against 570 ms at n = 1e6, 32 columns).  So does the 64-column fp16 tile
// over at most four K-steps (the six-term distance at d = 16): 5 registers spilled,
// 459 against 519 ms at n = 1e6 (one box); over six K-steps it spilled 43 and ran
// slower (780 against 635 ms).
template <int KIND, int KSMAX, int TM, bool F16V>
constexpr int flash2_waves_per_simd() {
  return (KSMAX <= 6 && (TM == 16 || (TM == 32 && KIND == NYS_RBF))) || (F16V && KSMAX <= 4 && TM == 64) ? 4 : 2;
}
template <int KIND, int KSMAX, int TM, bool F16V = false>
__global__ __launch_bounds__(KMV2_THREADS, (flash2_waves_per_simd<KIND, KSMAX, TM, F16V>())) void kmv_flash2_kernel(KArgs a) {
  using T = Tr<NYS_BF16X3>;
  using Op = typename T::Op;
  using PV = typename ProdType<F16V>::V;   // operand vector of the K V product
  using PS = typename ProdType<F16V>::S;
  constexpr int R = 2, WAVES = KMV2_THREADS / 64;
  constexpr int TJ = 32, TI = WAVES * R * 16, NCB = TM / 16;
  constexpr int VCH = TM * 4;                      // 16-byte chunks per V part per tile
  typedef __attribute__((address_space(3))) void lds_void;

  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int strideA = lds_stride<NYS_BF16X3>(a.Kp);
  const size_t a_bytes = ((size_t)TJ * strideA * 2 + 15) & ~size_t(15);
  u16 *const sA0 = reinterpret_cast<u16 *>(smem);
  u16 *const sA1 = reinterpret_cast<u16 *>(smem + a_bytes);
  u16 *const sV0 = reinterpret_cast<u16 *>(smem + 2 * a_bytes);
  u16 *const sV1 = sV0 + 2 * TM * 32;

  const int64_t ntiles = (a.nr + TI - 1) / TI;
  const int64_t nb = ntiles * a.chunks * a.nsplit;
  const int64_t nb_pad = (nb + 7) / 8 * 8;
  const int64_t lid = xcd_logical_block(nb_pad);
  if (lid >= nb) return;
  const int64_t tile = lid % ntiles;
  const int64_t rest = lid / ntiles;
  const int chunk = (int)(rest % a.chunks);
  const int split = (int)(rest / a.chunks);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col16 = lane & 15, grp = lane >> 4;
  constexpr int ks = KSMAX;   // the packing pads Kp to exactly KSMAX K-steps
  const int64_t i0 = tile * TI;
  const int64_t iw = i0 + (int64_t)wave * R * 16;
  const int c0 = chunk * TM;
  const u16 *Ag = reinterpret_cast<const u16 *>(a.Acols);
  const u16 *Bg = reinterpret_cast<const u16 *>(a.Brows);
  const u16 *Vh = reinterpret_cast<const u16 *>(a.V);
  const u16 *Vl = reinterpret_cast<const u16 *>(a.V2);

  Op bop[R][KSMAX];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int s = 0; s < KSMAX; ++s)
      bop[r][s] = (s < ks) ? load_op<NYS_BF16X3>(Bg + (iw + r * 16 + col16) * a.Kp + s * T::KSTEP + grp * T::KL)
                           : zero_op<NYS_BF16X3>();

  f4 acc[R][NCB];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) acc[r][cb] = f4{0, 0, 0, 0};

  const float cL = (float)a.cL, dcoef = (float)a.dcoef;
  // -1 kept opaque to the optimiser, so that kv - h stays an fma with a half operand
  float mone = -1.0f;
  if constexpr (F16V) asm volatile("" : "+v"(mone));
  const int64_t njt = (a.nc + TJ - 1) / TJ;
  const int64_t jt0 = (int64_t)split * a.jsteps;
  const int64_t jt1 = jt0 + a.jsteps < njt ? jt0 + a.jsteps : njt;

  // packed points of one tile: TJ rows x Kp bf16 = TJ * Kp / 8 chunks (<= KSMAX * 128)
  constexpr int APRE = (KSMAX * 128 + KMV2_THREADS - 1) / KMV2_THREADS;
  const int cpr = a.Kp / 8;
  const int achunks = TJ * cpr;
  static_assert(APRE <= 2, "point prefetch holds at most two chunks per thread");
  uint4 apre0 = {0, 0, 0, 0}, apre1 = {0, 0, 0, 0};   // scalars, not an array: kept in VGPRs
  auto load_points = [&](int64_t jt) {
    const uint4 *g = reinterpret_cast<const uint4 *>(Ag + jt * TJ * a.Kp);
    apre0 = g[tid < achunks ? tid : achunks - 1];
    if constexpr (APRE > 1) {
      const int c = tid + KMV2_THREADS;
      apre1 = g[c < achunks ? c : achunks - 1];
    }
  };
  auto store_points = [&](u16 *dst) {
    if (tid < achunks) {
      const int r = tid / cpr, o = tid - r * cpr;
      *reinterpret_cast<uint4 *>(dst + r * strideA + o * 8) = apre0;
    }
    if constexpr (APRE > 1) {
      const int c = tid + KMV2_THREADS;
      if (c < achunks) {
        const int r = c / cpr, o = c - r * cpr;
        *reinterpret_cast<uint4 *>(dst + r * strideA + o * 8) = apre1;
      }
    }
  };
  // split V of one tile: two contiguous runs of TM*32 bf16, copied by the waves in
  // 1 KB blocks (lane L of the wave lands 16 L bytes into the block)
  auto stream_v = [&](int64_t jt, u16 *dst) {
    const u16 *gh = Vh + (jt * a.m_pad + c0) * 32;
    const u16 *gl = Vl + (jt * a.m_pad + c0) * 32;
#pragma unroll
    for (int k = 0; k < (VCH + KMV2_THREADS - 1) / KMV2_THREADS; ++k) {
      const int blk = k * KMV2_THREADS + wave * 64;          // wave-uniform
      if (blk < VCH) {
        const int q = blk + lane;
        __builtin_amdgcn_global_load_lds(gh + q * 8, (lds_void *)(dst + blk * 8), 16, 0, 0);
        __builtin_amdgcn_global_load_lds(gl + q * 8, (lds_void *)(dst + TM * 32 + blk * 8), 16, 0, 0);
      }
    }
  };

  if (jt0 < jt1) {
    load_points(jt0);
    stream_v(jt0, sV0);
    store_points(sA0);
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  for (int64_t jt = jt0; jt < jt1; ++jt) {
    const int cur = (int)((jt - jt0) & 1);
    const u16 *sAc = cur ? sA1 : sA0;
    const u16 *sVh = cur ? sV1 : sV0;
    const bool more = jt + 1 < jt1;
    if (more) {
      stream_v(jt + 1, cur ? sV0 : sV1);
      load_points(jt + 1);
    }
    const int64_t j0 = jt * TJ;
    const bool diag = a.same && (j0 < i0 + TI) && (i0 < j0 + TJ);

    // exponents of the 32 x (R*16) pair block: each column-point operand is read
    // from LDS once and used against the R row blocks
    f4 ta[R], tb[R];
#pragma unroll
    for (int r = 0; r < R; ++r) ta[r] = tb[r] = f4{0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < KSMAX; ++s)
      if (s < ks) {
        const Op a0 = load_op<NYS_BF16X3>(sAc + col16 * strideA + s * T::KSTEP + grp * T::KL);
        const Op a1 = load_op<NYS_BF16X3>(sAc + (16 + col16) * strideA + s * T::KSTEP + grp * T::KL);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          ta[r] = mfma16(a0, bop[r][s], ta[r]);
          tb[r] = mfma16(a1, bop[r][s], tb[r]);
        }
      }
    // diagonal tiles (a wave-uniform test) pin the exponent of i == j to 0.  Hoisting the
    // test out of the epilogue measured 5-6% faster at 64 and 256 columns for the bf16
    // product and 6.7% faster at 128 for the fp16 product over the six-term distance
    // (whose narrow tiles are VALU-bound); the bf16 tiles of 128 columns and below keep
    // the per-element select (2.6% faster at 128 when measured).
    constexpr bool HOIST = F16V || TM == 64 || TM == 256;
    if (HOIST && diag) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int64_t gi = iw + r * 16 + col16;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int64_t gj = j0 + (e < 4 ? 4 * grp + e : 16 + 4 * grp + (e - 4));
          if (gi == gj) {
            if (e < 4) ta[r][e] = 0.0f;
            else tb[r][e - 4] = 0.0f;
          }
        }
      }
    }
    // K split into hi and lo parts (k - hi is exact in float32).  The fp16 product
    // converts the entries in pairs, one v_cvt_pk_f16_f32 per pair for the hi parts, so
    // that each hi part is converted once, and forms the lo part as an fma with a half
    // operand (v_fma_mix); the 128-column tile converts the hi pair back and subtracts
    // instead.  Measured at n = 1e6 (one box per pair of runs, six-term distance): 1
    // column 317 -> 292 ms, 32 columns 389 -> 357 ms, 128 columns 838 -> 767 ms, 512
    // columns (two 256-column chunks) 2545 -> 2479 ms; the 256-column tile with the
    // subtracting form measured 5% slower (2524 -> 2651 ms).
    PV phi[R], plo[R];
    if constexpr (F16V) {
      typedef float f2v __attribute__((ext_vector_type(2)));
      typedef _Float16 h2v __attribute__((ext_vector_type(2)));
#pragma unroll
      for (int r = 0; r < R; ++r) {
#pragma unroll
        for (int e = 0; e < 8; e += 2) {
          const float k0 = kernel_value<NYS_BF16X3, KIND, 0>(e < 4 ? ta[r][e] : tb[r][e - 4], cL, dcoef);
          const float k1 = kernel_value<NYS_BF16X3, KIND, 0>(e < 4 ? ta[r][e + 1] : tb[r][e - 3], cL, dcoef);
          const h2v hp = __builtin_convertvector((f2v){k0, k1}, h2v);
          phi[r][e] = hp[0];
          phi[r][e + 1] = hp[1];
          if constexpr (TM != 128) {
            plo[r][e] = (PS)__builtin_fmaf((float)hp[0], mone, k0);
            plo[r][e + 1] = (PS)__builtin_fmaf((float)hp[1], mone, k1);
          } else {
            const f2v hf = __builtin_convertvector(hp, f2v);
            const h2v lp = __builtin_convertvector((f2v){k0 - hf[0], k1 - hf[1]}, h2v);
            plo[r][e] = lp[0];
            plo[r][e + 1] = lp[1];
          }
        }
      }
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          float t = e < 4 ? ta[r][e] : tb[r][e - 4];
          if constexpr (!HOIST) {
            const int64_t gj = j0 + (e < 4 ? 4 * grp + e : 16 + 4 * grp + (e - 4));
            if (diag && iw + r * 16 + col16 == gj) t = 0.0f;
          }
          const float kv = kernel_value<NYS_BF16X3, KIND, 0>(t, cL, dcoef);
          const PS h = (PS)kv;
          phi[r][e] = h;
          plo[r][e] = (PS)(kv - (float)h);
        }
      }
    }
    // V operands are read one column block ahead of the MFMAs that use them
    // 16 lanes of a lane group read 256 contiguous bytes (no LDS bank conflicts)
    const u16 *vrow = sVh + grp * 128 + col16 * 8;
    PV vh_n = *reinterpret_cast<const PV *>(vrow);
    PV vl_n = *reinterpret_cast<const PV *>(vrow + TM * 32);
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      const PV vh = vh_n, vl = vl_n;
      if (cb + 1 < NCB) {
        vh_n = *reinterpret_cast<const PV *>(vrow + (cb + 1) * 16 * 32);
        vl_n = *reinterpret_cast<const PV *>(vrow + TM * 32 + (cb + 1) * 16 * 32);
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        acc[r][cb] = mfma16(phi[r], vh, acc[r][cb]);
        acc[r][cb] = mfma16(phi[r], vl, acc[r][cb]);
        acc[r][cb] = mfma16(plo[r], vh, acc[r][cb]);
      }
    }
    if (more) store_points(cur ? sA0 : sA1);
    __builtin_amdgcn_s_waitcnt(0);   // the streamed tile has landed
    __syncthreads();
  }

  float *O = reinterpret_cast<float *>(a.Out);
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t i = iw + r * 16 + out_row<NYS_BF16X3>(grp, v);
        const int c = c0 + cb * 16 + col16;
        if (i < a.nr && c < a.m) {
          float sum = acc[r][cb][v];
          if constexpr (F16V) sum *= a.vscale[c];
          if (a.partial) {
            O[((int64_t)split * a.nr + i) * a.m + c] = sum;
          } else {
            float val = (float)a.alpha * sum;
            if (a.beta != 0.0) val += (float)a.beta * O[i * a.ldo + c];
            O[i * a.ldo + c] = val;
          }
        }
      }
}

// ===================================================================== flash, pipelined (FP64)
// The float64 product (the refinement residual) on the same eight-wave schedule as
// the BF16X3 tile: R 16-row blocks per wave (128 R rows per workgroup), 32-point
// column tiles double buffered in
// LDS, V streamed global-to-LDS while the previous tile computes.  V arrives
// permuted (vperm64_kernel) so that the B operand of the 16x16x4 float64 MFMA is 64
// consecutive doubles per lane group read: for tile rows j = 16 h + 4 v + g and a
// 16-column block cb, element (j, c) sits at [h][v][cb][g][c % 16].  The exponent
// MFMA leaves K[i][16 h + g + 4 v] in lane (g, i), which is exactly the A operand of
// MFMA v of half h.  Per tile and wave: 2 R KS MFMAs for the exponents, 8 R TM/16 for
// K V, 8 R float64 exponentials per lane.  KSMAX below 8 is the exact number of
// K-steps (a branch-free chain and fewer registers); 8 and 16 are upper bounds.
// Tiles that fit 128 registers without spilling run four waves per SIMD (two
// workgroups per CU).
template <int KIND, int KSMAX, int TM, int R>
constexpr int flash64_waves_per_simd() {
  if constexpr (R == 1) return KSMAX <= 8 && TM <= 64 ? 4 : 2;
  return (TM == 16 && KSMAX <= 8) || (TM == 32 && KSMAX <= 5 && KIND == NYS_RBF) ? 4 : 2;
}
template <int KIND, int KSMAX, int TM, int R>
__global__ __launch_bounds__(KMV2_THREADS, (flash64_waves_per_simd<KIND, KSMAX, TM, R>())) void kmv_flash64_kernel(KArgs a) {
  constexpr int WAVES = KMV2_THREADS / 64;
  constexpr int TJ = 32, TI = WAVES * R * 16, NCB = TM / 16;
  constexpr int VCH = TJ * TM / 2;                 // 16-byte chunks of V per tile
  typedef __attribute__((address_space(3))) void lds_void;

  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int strideA = a.Kp + 2;                    // doubles; 4 (2 Kp / 4 + 1) dwords: conflict-free rows
  const size_t a_bytes = ((size_t)TJ * strideA * 8 + 15) & ~size_t(15);
  double *const sA0 = reinterpret_cast<double *>(smem);
  double *const sA1 = reinterpret_cast<double *>(smem + a_bytes);
  double *const sV0 = reinterpret_cast<double *>(smem + 2 * a_bytes);
  double *const sV1 = sV0 + TJ * TM;
  double *const tab = sV1 + TJ * TM;               // 2^(j/64), j < 64

  const int64_t ntiles = (a.nr + TI - 1) / TI;
  const int64_t nb = ntiles * a.chunks * a.nsplit;
  const int64_t nb_pad = (nb + 7) / 8 * 8;
  const int64_t lid = xcd_logical_block(nb_pad);
  if (lid >= nb) return;
  const int64_t tile = lid % ntiles;
  const int64_t rest = lid / ntiles;
  const int chunk = (int)(rest % a.chunks);
  const int split = (int)(rest / a.chunks);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col16 = lane & 15, grp = lane >> 4;
  const int ks = KSMAX < 8 ? KSMAX : a.Kp / 4;
  exp_tab_init(tab, tid);                          // visible after the first barrier
  const int64_t i0 = tile * TI;
  const int64_t iw = i0 + (int64_t)wave * R * 16;
  const int c0 = chunk * TM;
  const double *Ag = reinterpret_cast<const double *>(a.Acols);
  const double *Bg = reinterpret_cast<const double *>(a.Brows);
  const double *Vp = reinterpret_cast<const double *>(a.V);

  double bop[R][KSMAX];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int s = 0; s < KSMAX; ++s) bop[r][s] = (s < ks) ? Bg[(iw + r * 16 + col16) * a.Kp + s * 4 + grp] : 0.0;

  d4 acc[R][NCB];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) acc[r][cb] = d4{0, 0, 0, 0};

  const double cL = a.cL;
  const int64_t njt = (a.nc + TJ - 1) / TJ;
  const int64_t jt0 = (int64_t)split * a.jsteps;
  const int64_t jt1 = jt0 + a.jsteps < njt ? jt0 + a.jsteps : njt;

  // packed points of one tile: TJ rows x Kp doubles = 16 Kp chunks of 16 bytes
  const int cpr = a.Kp / 2;
  const int achunks = TJ * cpr;
  constexpr int APRE = (KSMAX * 4 * TJ / 2 + KMV2_THREADS - 1) / KMV2_THREADS;
  static_assert(APRE <= 2, "point prefetch holds at most two chunks per thread");
  uint4 apre0 = {0, 0, 0, 0}, apre1 = {0, 0, 0, 0};
  auto load_points = [&](int64_t jt) {
    const uint4 *g = reinterpret_cast<const uint4 *>(Ag + jt * TJ * a.Kp);
    apre0 = g[tid < achunks ? tid : achunks - 1];
    if constexpr (APRE > 1) {
      const int c = tid + KMV2_THREADS;
      apre1 = g[c < achunks ? c : achunks - 1];
    }
  };
  auto store_points = [&](double *dst) {
    if (tid < achunks) {
      const int r = tid / cpr, o = tid - r * cpr;
      *reinterpret_cast<uint4 *>(dst + r * strideA + o * 2) = apre0;
    }
    if constexpr (APRE > 1) {
      const int c = tid + KMV2_THREADS;
      if (c < achunks) {
        const int r = c / cpr, o = c - r * cpr;
        *reinterpret_cast<uint4 *>(dst + r * strideA + o * 2) = apre1;
      }
    }
  };
  // permuted V of one tile: TJ x TM doubles, contiguous; copied in 1 KB wave blocks
  auto stream_v = [&](int64_t jt, double *dst) {
    const double *g = Vp + (jt * a.chunks + chunk) * (TJ * TM);
#pragma unroll
    for (int k = 0; k < (VCH + KMV2_THREADS - 1) / KMV2_THREADS; ++k) {
      const int blk = k * KMV2_THREADS + wave * 64;          // wave-uniform
      if (blk < VCH) {
        const int q = blk + lane;
        __builtin_amdgcn_global_load_lds(g + q * 2, (lds_void *)(dst + blk * 2), 16, 0, 0);
      }
    }
  };

  if (jt0 < jt1) {
    load_points(jt0);
    stream_v(jt0, sV0);
    store_points(sA0);
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  for (int64_t jt = jt0; jt < jt1; ++jt) {
    const int cur = (int)((jt - jt0) & 1);
    const double *sAc = cur ? sA1 : sA0;
    const double *sVc = cur ? sV1 : sV0;
    const bool more = jt + 1 < jt1;
    if (more) {
      stream_v(jt + 1, cur ? sV0 : sV1);
      load_points(jt + 1);
    }
    const int64_t j0 = jt * TJ;
    const bool diag = a.same && (j0 < i0 + TI) && (i0 < j0 + TJ);

    // exponents: rows j of the tile (two halves of 16) against the R row blocks
    d4 ta[R], tb[R];
#pragma unroll
    for (int r = 0; r < R; ++r) ta[r] = tb[r] = d4{0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < KSMAX; ++s)
      if (s < ks) {
        const double a0 = sAc[col16 * strideA + s * 4 + grp];
        const double a1 = sAc[(16 + col16) * strideA + s * 4 + grp];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          ta[r] = mfma16(a0, bop[r][s], ta[r]);
          tb[r] = mfma16(a1, bop[r][s], tb[r]);
        }
      }
    // kernel values: lane (g, i) holds K[i][g + 4 v] (half 0) and K[i][16 + g + 4 v]
    double ka[R][4], kb[R][4];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t gi = iw + r * 16 + col16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double t1 = ta[r][v], t2 = tb[r][v];
        if (diag && gi == j0 + grp + 4 * v) t1 = 0.0;
        if (diag && gi == j0 + 16 + grp + 4 * v) t2 = 0.0;
        ka[r][v] = kernel_value_tab<KIND, 0>(t1, cL, 0.0, tab);
        kb[r][v] = kernel_value_tab<KIND, 0>(t2, cL, 0.0, tab);
      }
    }
    // K V: MFMA v of half h contracts j = 16 h + 4 v + g
    const double *vl = sVc + lane;
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double b0 = vl[((0 * 4 + v) * NCB + cb) * 64];
        const double b1 = vl[((1 * 4 + v) * NCB + cb) * 64];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          acc[r][cb] = mfma16(ka[r][v], b0, acc[r][cb]);
          acc[r][cb] = mfma16(kb[r][v], b1, acc[r][cb]);
        }
      }
    }
    if (more) store_points(cur ? sA0 : sA1);
    __builtin_amdgcn_s_waitcnt(0);   // the streamed tile has landed
    __syncthreads();
  }

  double *O = reinterpret_cast<double *>(a.Out);
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t i = iw + r * 16 + out_row<NYS_FP64>(grp, v);
        const int c = c0 + cb * 16 + col16;
        if (i < a.nr && c < a.m) {
          const double sum = acc[r][cb][v];
          if (a.partial) {
            O[((int64_t)split * a.nr + i) * a.m + c] = sum;
          } else {
            double val = a.alpha * sum;
            if (a.beta != 0.0) val += a.beta * O[i * a.ldo + c];
            O[i * a.ldo + c] = val;
          }
        }
      }
}

template <int TM>
inline size_t kmv_flash64_lds(int Kp) {
  const size_t a = ((size_t)32 * (Kp + 2) * 8 + 15) & ~size_t(15);
  return 2 * a + (size_t)2 * 32 * TM * 8 + 64 * 8;
}

template <int TM>
inline size_t kmv_flash2_lds(int Kp) {
  const size_t a = ((size_t)32 * lds_stride<NYS_BF16X3>(Kp) * 2 + 15) & ~size_t(15);
  return 2 * a + (size_t)2 * 2 * TM * 32 * 2;
}

// LDS bytes of the kernels above for a given plan.
template <int PREC>
inline size_t kmv_small_lds(int Kp, int MM) {
  using T = Tr<PREC>;
  size_t a = ((size_t)64 * lds_stride<PREC>(Kp) * sizeof(typename T::E) + 15) & ~size_t(15);
  return a + (size_t)64 * MM * sizeof(typename T::F) + (PREC == NYS_FP64 ? 64 * 8 : 0);
}
template <int PREC>
inline size_t kmv_flash_lds(int Kp, int TM) {
  using T = Tr<PREC>;
  size_t a = ((size_t)32 * lds_stride<PREC>(Kp) * sizeof(typename T::E) + 15) & ~size_t(15);
  if (PREC == NYS_BF16X3) return a + (size_t)2 * TM * 32 * 2;
  int VS = (PREC == NYS_FP32) ? TM + 4 : TM + 1;
  return a + (size_t)32 * VS * sizeof(typename T::F);
}

// Per-precision dispatch (defined in kmv_<prec>.hip).
int32_t kmv_dispatch_f64(const KmvPlan &p, int kind, int deriv, int ksmax, KArgs &a, dim3 grid,
                         hipStream_t s);
int32_t kmv_dispatch_f32(const KmvPlan &p, int kind, int deriv, int ksmax, KArgs &a, dim3 grid,
                         hipStream_t s);
int32_t kmv_dispatch_bf16(const KmvPlan &p, int kind, int deriv, int ksmax, KArgs &a, dim3 grid,
                          hipStream_t s);
int32_t kmv_dispatch_f16(const KmvPlan &p, int kind, int deriv, int ksmax, KArgs &a, dim3 grid,
                          hipStream_t s);
int32_t kmv_dispatch_f64p(const KmvPlan &p, int kind, int deriv, int ksmax, KArgs &a, dim3 grid,
                          hipStream_t s);

}  // namespace nys
