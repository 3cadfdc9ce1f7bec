// Internal declarations of libnys (not part of the public ABI).
#pragma once

#include <array>
#include <vector>

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/nys.h"

namespace nys {

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);

struct Status {
  int32_t code = NYS_OK;
  bool ok() const { return code == NYS_OK; }
};

#define NYS_CHECK_HIP(expr)                                                         \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess) {                                                         \
      ::nys::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));          \
      return NYS_EHIP;                                                              \
    }                                                                               \
  } while (0)

#define NYS_RETURN_IF(rc)      \
  do {                         \
    int32_t r_ = (rc);         \
    if (r_ != NYS_OK) return r_; \
  } while (0)

#define NYS_LAUNCH_CHECK()                                                          \
  do {                                                                              \
    hipError_t e_ = hipGetLastError();                                              \
    if (e_ != hipSuccess) {                                                         \
      ::nys::set_error(std::string("kernel launch: ") + hipGetErrorString(e_));     \
      return NYS_EHIP;                                                              \
    }                                                                               \
  } while (0)

// ---------------------------------------------------------------- workspace
// Bump allocator over the caller's workspace.  In measuring mode (base ==
// nullptr) it only counts, so the same planning code yields the size query.
struct Arena {
  char *base = nullptr;
  size_t cap = 0;
  size_t off = 0;
  bool measuring() const { return base == nullptr; }
  template <class T>
  T *take(size_t count) {
    size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
    if (bytes == 0) bytes = 256;
    size_t at = off;
    off += bytes;
    if (measuring() || off > cap) return nullptr;
    return reinterpret_cast<T *>(base + at);
  }
  bool overflowed() const { return !measuring() && off > cap; }
};

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }
inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------- packed points
// Points packed for the MFMA distance tiles.  The exponent of the kernel,
// t_ij = kappa (2 x_i.x_j - |x_i|^2 - |x_j|^2), is produced by one MFMA chain from
// augmented rows: "col" rows (the A operand, points j) hold
// [2 kappa x_j, -kappa |x_j|^2, 1] and "row" rows (the B operand, points i) hold
// [x_i, 1, -kappa |x_i|^2]; BF16X3 stores the split parts side by side.
enum Side { SIDE_COL = 0, SIDE_ROW = 1 };

constexpr int ROW_PAD = 256;  // packed row counts are padded to this multiple

struct Packed {
  void *data = nullptr;   // [n_pad][Kp] elements (double, float or bf16 bits)
  int64_t n = 0;          // valid rows
  int64_t n_pad = 0;      // padded rows (zero-filled)
  int Kp = 0;             // padded K extent
  int prec = 0;
};

// The tile kernels run BF16X3_D6, BF16X3_D10, F16X3_D10 and F16X3_D6 with the BF16X3
// instantiations (the packing differs: six or ten distance terms instead of three;
// the F16X3 precisions also switch the K V product to fp16 parts).
inline int kernel_prec(int prec) {
  return (prec == NYS_BF16X3_D6 || prec == NYS_BF16X3_D10 || prec == NYS_F16X3_D10 || prec == NYS_F16X3_D6)
             ? NYS_BF16X3
             : prec;
}
inline bool f16_product(int prec) { return prec == NYS_F16X3_D10 || prec == NYS_F16X3_D6; }
// the distance packing of a precision (the F16X3 precisions pack as their bf16 twins)
inline int packing_prec(int prec) {
  return prec == NYS_F16X3_D10 ? NYS_BF16X3_D10 : (prec == NYS_F16X3_D6 ? NYS_BF16X3_D6 : prec);
}
// key of the tile tables (valid and tuned widths): the fp16-product precisions have
// their own, the other split precisions share BF16X3's
inline int tile_key(int prec) { return f16_product(prec) ? prec : kernel_prec(prec); }

int packed_kp(int d, int prec);
size_t packed_elem_bytes(int prec);
double kernel_kappa(const nys_kernel &k, int prec);

// Column mean of X (n x d float64) into mu (d), deterministic two-pass.
int32_t launch_col_mean(const double *X, int64_t n, int d, double *mu, double *partial,
                        hipStream_t s);
size_t col_mean_partial_elems(int64_t n, int d);

// Packs the points; a non-finite coordinate (or centre) sets *bad (device int).
int32_t launch_pack(const double *X, int64_t n, int d, const double *mu, const nys_kernel &k,
                    int prec, int side, Packed *out, int *bad, hipStream_t s);

// ---------------------------------------------------------------- kernel product
struct KmvPlan {
  int path = 0;          // 0 small-m row sums, 1 flash (second MFMA against V)
  int mm = 1;            // small path: compile-time column bound
  int tm = 64;           // flash path: column chunk
  int r = 4;             // row subtiles of 16 per wave
  int waves = 4;         // waves per workgroup (8: pipelined BF16X3 flash tile)
  int splits = 1;        // split of the column (j) range
  int jsteps = 0;        // j tiles per split
  int64_t m_pad = 0;     // flash BF16: padded width of the split V
  int f16v = 0;          // flash: fp16 K V product with column-scaled V
  int tail_tm = 0;       // flash: width of the last chunk when narrower than tm (its own launch)
};

// Decide the launch shape for an (nr, nc, m, prec) product.
KmvPlan kmv_plan(int64_t nr, int64_t nc, int m, int prec, int Kp);
// Scratch needed by kmv_run for a plan (partials, split V).
void kmv_reserve(const KmvPlan &p, int64_t nr, int64_t nc, int m, int prec, Arena &ws,
                 void **partial, void **vhi, void **vlo);
// Bytes of partial sums and u16 elements of the two split-V parts (hi, lo) a plan
// needs (the float64 tile keeps its permuted V in the hi part).
void kmv_scratch_sizes(const KmvPlan &p, int64_t nr, int64_t nc, int m, int prec,
                       size_t *partial_bytes, size_t *vsplit_elems, size_t *vlo_elems);

// Out = alpha * K V + beta * Out using packed points.  V/Out are double for
// FP64 else float.  same_points marks A == B point sets (K_ii = 1 exactly).
int32_t kmv_run(const KmvPlan &plan, const nys_kernel &k, int deriv, int prec,
                const Packed &rows, const Packed &cols, int same_points, const void *V,
                int m, int ldv, void *Out, int ldo, double alpha, double beta, void *partial,
                void *vhi, void *vlo, hipStream_t s);

// Autotuned chunk widths: tm for columns m in [m_lo, m_hi] of a precision (tm 0 removes).
bool kmv_tile_valid(int prec, int tm);
void kmv_tune_set(int prec, int m_lo, int m_hi, int tm);
void kmv_tune_clear();   // also restores the default float64 cost table
// Replace the float64 planner's per-chunk costs of the widths 16, 32, 48, 64, 96, 128, 256.
void kmv_f64_cost_set(const double *cost7);
std::vector<std::array<int, 4>> kmv_tune_snapshot();
void kmv_tune_restore(const std::vector<std::array<int, 4>> &t);

// ---------------------------------------------------------------- dense helpers
// C[p x q] (+)= A^T B over rows [0, n): A n x p (lda), B n x q (ldb), row-major.
// Split over n into `splits` chunks written to partial[splits][p][q], then reduced.
template <class T>
int32_t gemm_tn(const T *A, int lda, const T *B, int ldb, int64_t n, int p, int q, T *C,
                int ldc, T *partial, int splits, hipStream_t s);
int gemm_tn_splits(int64_t n, int p, int q);
// Mixed: C (double) = A^T B with A double and B float (products and sums in float64).
int32_t gemm_tn_df(const double *A, int lda, const float *B, int ldb, int64_t n, int p, int q, double *C,
                   int ldc, double *partial, int splits, hipStream_t s);
// C (double) = A^T B with A, B of type T (products in T, sums in float64).
template <class T>
int32_t gemm_tn_to_double(const T *A, int lda, const T *B, int ldb, int64_t n, int p, int q, double *C, int ldc,
                          double *partial, int splits, hipStream_t s);
// Mixed: C (float) = A B + R * rscale[col], arithmetic in float64, R float.
int32_t gemm_nn_dd_f(const double *A, int lda, const double *B, int ldb, int64_t n, int p, int q, float *C,
                     int ldc, const float *R, int ldr, const double *rscale, hipStream_t s);

// C[n x q] = A[n x p] B[p x q] (+ epilogue): epi 0: C = AB; 1: C = AB + R * rscale[col]
template <class T>
int32_t gemm_nn(const T *A, int lda, const T *B, int ldb, int64_t n, int p, int q, T *C,
                int ldc, int epi, const T *R, int ldr, const double *rscale, hipStream_t s);

// Frobenius-norm squared of a n x m matrix (double accumulation) into out (device).
int32_t launch_sumsq(const double *A, int64_t count, double *partial, double *out, hipStream_t s);
size_t sumsq_partial_elems(int64_t count);

// y = a x + y elementwise on count doubles (a host scalar).
int32_t launch_axpy(double a, const double *x, double *y, int64_t count, hipStream_t s);
int32_t launch_copy_d2f(const double *x, float *y, int64_t count, hipStream_t s);
int32_t launch_copy_f2d(const float *x, double *y, int64_t count, hipStream_t s);
int32_t launch_fill(double *y, double v, int64_t count, hipStream_t s);
int32_t launch_fill_f(float *y, float v, int64_t count, hipStream_t s);

// ---------------------------------------------------------------- small dense
// In-place lower Cholesky of a symmetric r x r matrix (lower triangle used,
// upper zeroed); flag[0] = 0 on success, 1 + k if pivot k failed.
int32_t launch_chol(double *A, int r, int *flag, hipStream_t s);
// Linv = L^{-1} for lower-triangular L (r x r).
int32_t launch_trinv_lower(const double *L, double *Linv, int r, hipStream_t s);
// Symmetrise: A = (M + M^T)/2 + shift * G where G is given (may be null).
int32_t launch_symmetrise(const double *M, double *A, int r, hipStream_t s);
// Transpose r x r.
int32_t launch_transpose(const double *A, double *At, int r, hipStream_t s);
// Symmetric eigendecomposition by cyclic parallel Jacobi: A (r x r) is
// destroyed, eigenvalues in w (unsorted), eigenvectors in columns of V.
int32_t jacobi_eig(double *A, double *Abuf, double *V, double *w, int r, double *scratch,
                   hipStream_t s);
size_t jacobi_scratch_elems(int r);
// From unsorted eigenpairs (w, V) of B^T B build T = V_sorted diag(1/sqrt(w)) for
// kept columns, lam_hat = max(0, w - nu) descending; rank_out (device int).
int32_t launch_eig_finish(const double *w, const double *V, int r, double nu, double *T,
                          double *lam_hat, int *rank_out, hipStream_t s);

// ---------------------------------------------------------------- test matrix
// count standard normals (Philox4x32-10 + Box-Muller, a pure function of seed and
// index) into out.
int32_t launch_gaussian(uint64_t seed, int64_t count, double *out, hipStream_t s);

// ---------------------------------------------------------------- ceiling probes
// Time one synthetic kernel keeping one unit busy (0 bf16 MFMA, 1 fp16 MFMA,
// 2 float64 MFMA, 3 v_exp_f32, 4 device copy); *rate in that unit per second.
int32_t peak_probe(int which, int iters, double *rate, void *ws, size_t ws_bytes, hipStream_t s);

// ---------------------------------------------------------------- preconditioner apply
template <class T>
int32_t precond_apply_impl(const nys_precond &P, const double *lambdas, const T *R, int m,
                           T *Z, Arena &ws, hipStream_t s);

// ---------------------------------------------------------------- PCG vector kernels
struct ColState;  // defined in pcg.hip
}  // namespace nys
