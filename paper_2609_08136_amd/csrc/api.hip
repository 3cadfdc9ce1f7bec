// C ABI of libnys: argument checking, workspace planning and the host-side
// orchestration of the device kernels (sketch, preconditioner build/apply,
// the PCG driver with column compaction and float64 refinement, backward).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <mutex>

#include <rocblas/rocblas.h>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "admm.h"
#include "block.h"
#include "gemv.h"
#include "pcg.h"

namespace nys {
static thread_local std::string g_err;
void set_error(const std::string &m) { g_err = m; }
const char *last_error_cstr() { return g_err.c_str(); }
}  // namespace nys

using namespace nys;

namespace {

typedef unsigned short bf16bits;

hipStream_t as_stream(void *p) { return reinterpret_cast<hipStream_t>(p); }

int32_t einval(const std::string &m) {
  set_error(m);
  return NYS_EINVAL;
}
bool valid_prec(int p) { return p >= NYS_FP64 && p <= NYS_F16X3_D6; }
int max_dim(int prec) {
  switch (prec) {
    case NYS_BF16X3: return 82;
    case NYS_BF16X3_D6:
    case NYS_F16X3_D6: return 41;
    case NYS_BF16X3_D10:
    case NYS_F16X3_D10: return 24;
    default: return 62;
  }
}
size_t elem_bytes(int prec) { return prec == NYS_FP64 ? 8 : 4; }

int32_t check_kernel(const nys_kernel &k) {
  if (!(k.kind == NYS_RBF || k.kind == NYS_LAPLACIAN)) return einval("unknown kernel kind");
  if (!(k.sigma > 0.0) || !std::isfinite(k.sigma)) return einval("sigma must be positive and finite");
  return NYS_OK;
}

int32_t check_ws(const Arena &a) {
  if (a.overflowed()) {
    set_error("workspace smaller than nys_workspace_bytes() for these arguments");
    return NYS_ENOMEM;
  }
  return NYS_OK;
}

// ------------------------------------------------------------ kernel product buffers
struct KmvBufs {
  double *mu = nullptr, *mpart = nullptr;
  int *bad = nullptr;   // set by the packing when a point is not finite
  Packed rows, cols;
  void *partial = nullptr, *vhi = nullptr, *vlo = nullptr;
};

void plan_points(Packed &p, int64_t n, int d, int prec, Arena &ws) {
  p.n = n;
  p.n_pad = round_up(std::max<int64_t>(n, 1), ROW_PAD);
  p.Kp = packed_kp(d, prec);
  p.prec = prec;
  p.data = ws.take<char>((size_t)p.n_pad * p.Kp * packed_elem_bytes(prec));
}

// Points packed once; scratch reserved for every column count in [m_lo, m_max]
// (the solver shrinks its column count as columns converge).
void plan_kmv(KmvBufs &b, int64_t nr, int64_t nc, int d, int m_lo, int m_max, int prec, Arena &ws) {
  b.mu = ws.take<double>(d);
  b.mpart = ws.take<double>(col_mean_partial_elems(nc, d));
  b.bad = ws.take<int>(4);
  plan_points(b.rows, nr, d, prec, ws);
  plan_points(b.cols, nc, d, prec, ws);
  size_t pb = 0, ve = 0, vl = 0, a = 0, e = 0, l = 0;
  for (int m = std::max(1, m_lo); m <= m_max; ++m) {
    KmvPlan p = kmv_plan(nr, nc, m, prec, b.rows.Kp);
    kmv_scratch_sizes(p, nr, nc, m, prec, &a, &e, &l);
    pb = std::max(pb, a);
    ve = std::max(ve, e);
    vl = std::max(vl, l);
  }
  // the derivative product runs in chunks of <= 4 columns with the 4-column plan
  // (row-sum tile: planned with the distance packing's precision, no fp16 product)
  const KmvPlan p4 = kmv_plan(nr, nc, 4, packing_prec(prec), b.rows.Kp);
  kmv_scratch_sizes(p4, nr, nc, std::min(4, std::max(1, m_max)), packing_prec(prec), &a, &e, &l);
  pb = std::max(pb, a);
  b.partial = pb ? ws.take<char>(pb) : nullptr;
  b.vhi = ve ? ws.take<bf16bits>(ve) : nullptr;
  b.vlo = vl ? ws.take<bf16bits>(vl) : nullptr;
}

// Centre and pack both point sets.  Synchronises the stream once to read the
// packing's finiteness flag: a NaN or Inf coordinate returns NYS_ENUMERIC (a NaN
// would otherwise turn every packed point, through the column mean, into NaN).
int32_t prep_points(KmvBufs &b, const nys_kernel &k, int prec, const double *Xr, const double *Xc,
                    int d, hipStream_t s) {
  NYS_CHECK_HIP(hipMemsetAsync(b.bad, 0, sizeof(int), s));
  NYS_RETURN_IF(launch_col_mean(Xc, b.cols.n, d, b.mu, b.mpart, s));
  NYS_RETURN_IF(launch_pack(Xr, b.rows.n, d, b.mu, k, prec, SIDE_ROW, &b.rows, b.bad, s));
  NYS_RETURN_IF(launch_pack(Xc, b.cols.n, d, b.mu, k, prec, SIDE_COL, &b.cols, b.bad, s));
  int bad = 0;
  NYS_CHECK_HIP(hipMemcpyAsync(&bad, b.bad, sizeof(int), hipMemcpyDeviceToHost, s));
  NYS_CHECK_HIP(hipStreamSynchronize(s));
  if (bad) {
    set_error("NaN or Inf in the point coordinates X");
    return NYS_ENUMERIC;
  }
  return NYS_OK;
}

// Out = alpha K V + beta Out for m columns (ldv / ldo strides), planned for m.
int32_t run_kmv(KmvBufs &b, const nys_kernel &k, int deriv, int prec, int same, const void *V, int m,
                int ldv, void *Out, int ldo, double alpha, double beta, hipStream_t s) {
  if (m <= 0) return NYS_OK;
  const size_t eb = elem_bytes(prec);
  if (deriv) {
    // the derivative runs on the row-sum tile in chunks of <= 4 columns
    const KmvPlan p = kmv_plan(b.rows.n, b.cols.n, m == 1 ? 1 : 4, packing_prec(prec), b.rows.Kp);
    for (int c0 = 0; c0 < m; c0 += 4) {
      const int mc = std::min(4, m - c0);
      NYS_RETURN_IF(kmv_run(p, k, 1, prec, b.rows, b.cols, same,
                            reinterpret_cast<const char *>(V) + c0 * eb, mc, ldv,
                            reinterpret_cast<char *>(Out) + c0 * eb, ldo, alpha, beta, b.partial,
                            b.vhi, b.vlo, s));
    }
    return NYS_OK;
  }
  const KmvPlan p = kmv_plan(b.rows.n, b.cols.n, m, prec, b.rows.Kp);
  return kmv_run(p, k, deriv, prec, b.rows, b.cols, same, V, m, ldv, Out, ldo, alpha, beta,
                 b.partial, b.vhi, b.vlo, s);
}

// ------------------------------------------------------------ kernel_matvec
struct MatvecPlan {
  KmvBufs kv;
};

// Autotuner buffers: V (n x m), Out (n_rows x m) and the kernel-product scratch of
// the largest candidate chunk width.  The candidates are the instantiated widths
// of the precision with at most 4 chunks and at most twice the next power of two
// of m (none when m runs on the row-sum tile).
struct AutotunePlan {
  KmvBufs kv;
  void *V = nullptr, *Out = nullptr;
  std::vector<int> cands;
};
void plan_matvec(MatvecPlan &p, int64_t nr, int64_t nc, int d, int m, int prec, Arena &ws) {
  // the derivative product runs in chunks of <= 4 columns: reserve for both
  plan_kmv(p.kv, nr, nc, d, std::min(m, 4), m, prec, ws);
}

int32_t plan_autotune(AutotunePlan &p, int64_t n_rows, int64_t n, int d, int m, int prec, Arena &ws) {
  const int key = tile_key(prec);
  p.cands.clear();
  const int base = kmv_plan(n_rows, n, m, prec, packed_kp(d, prec)).path;
  if (base == 1) {
    int pw = 1;
    while (pw < m) pw *= 2;
    for (int tm : {16, 32, 48, 64, 96, 128, 256})
      if (kmv_tile_valid(key, tm) && ceil_div(m, tm) <= 4 && tm <= 2 * std::max(pw, 16)) p.cands.push_back(tm);
  }
  const size_t eb = elem_bytes(prec);
  p.V = ws.take<char>((size_t)n * m * eb);
  p.Out = ws.take<char>((size_t)n_rows * m * eb);
  // points packed once; scratch for the largest candidate (the table is restored after)
  p.kv.mu = ws.take<double>(d);
  p.kv.mpart = ws.take<double>(col_mean_partial_elems(n, d));
  p.kv.bad = ws.take<int>(4);
  plan_points(p.kv.rows, n_rows, d, prec, ws);
  plan_points(p.kv.cols, n, d, prec, ws);
  size_t pb = 0, ve = 0, vl = 0, a = 0, e = 0, l = 0;
  std::vector<int> widths = p.cands;
  if (widths.empty()) widths.push_back(0);
  const auto saved = kmv_tune_snapshot();
  for (int tm : widths) {
    if (tm) kmv_tune_set(key, m, m, tm);
    const KmvPlan kp = kmv_plan(n_rows, n, m, prec, p.kv.rows.Kp);
    kmv_scratch_sizes(kp, n_rows, n, m, prec, &a, &e, &l);
    pb = std::max(pb, a);
    ve = std::max(ve, e);
    vl = std::max(vl, l);
  }
  kmv_tune_restore(saved);
  p.kv.partial = pb ? ws.take<char>(pb) : nullptr;
  p.kv.vhi = ve ? ws.take<bf16bits>(ve) : nullptr;
  p.kv.vlo = vl ? ws.take<bf16bits>(vl) : nullptr;
  return NYS_OK;
}

// ------------------------------------------------------------ sketch
struct SketchPlan {
  double *G = nullptr, *Gpart = nullptr, *Linv = nullptr, *LinvT = nullptr, *Qtmp = nullptr;
  int *flag = nullptr;
  float *Q32 = nullptr, *Y32 = nullptr;
  KmvBufs kv;
};
void plan_sketch(SketchPlan &p, int64_t n, int d, int r, int prec, Arena &ws) {
  const int splits = gemm_tn_splits(n, r, r);
  p.G = ws.take<double>((size_t)r * r);
  p.Gpart = ws.take<double>((size_t)splits * r * r);
  p.Linv = ws.take<double>((size_t)r * r);
  p.LinvT = ws.take<double>((size_t)r * r);
  p.Qtmp = ws.take<double>((size_t)n * r);
  p.flag = ws.take<int>(4);
  if (prec != NYS_FP64) {
    p.Q32 = ws.take<float>((size_t)n * r);
    p.Y32 = ws.take<float>((size_t)n * r);
  }
  plan_kmv(p.kv, n, n, d, r, r, prec, ws);
}

// ------------------------------------------------------------ precond build
struct BuildPlan {
  double *ssq_part = nullptr, *ssq = nullptr, *Ynu = nullptr, *Bm = nullptr;
  double *M = nullptr, *Mpart = nullptr, *L = nullptr, *Linv = nullptr, *LinvT = nullptr;
  double *G = nullptr, *Gs = nullptr, *Gbuf = nullptr, *Vev = nullptr, *w = nullptr, *T = nullptr;
  double *jac = nullptr;
  int *flag = nullptr, *rank = nullptr;
};
void plan_build(BuildPlan &p, int64_t n, int r, Arena &ws) {
  const int64_t cnt = n * (int64_t)r;
  const int splits = gemm_tn_splits(n, r, r);
  p.ssq_part = ws.take<double>(sumsq_partial_elems(cnt));
  p.ssq = ws.take<double>(1);
  p.Ynu = ws.take<double>((size_t)cnt);
  p.Bm = ws.take<double>((size_t)cnt);
  p.M = ws.take<double>((size_t)r * r);
  p.Mpart = ws.take<double>((size_t)splits * r * r);
  p.L = ws.take<double>((size_t)r * r);
  p.Linv = ws.take<double>((size_t)r * r);
  p.LinvT = ws.take<double>((size_t)r * r);
  p.G = ws.take<double>((size_t)r * r);
  p.Gs = ws.take<double>((size_t)r * r);
  p.Gbuf = ws.take<double>((size_t)r * r);
  p.Vev = ws.take<double>((size_t)r * r);
  p.w = ws.take<double>((size_t)r);
  p.T = ws.take<double>((size_t)r * r);
  p.jac = ws.take<double>(jacobi_scratch_elems(r));
  p.flag = ws.take<int>(4);
  p.rank = ws.take<int>(4);
}

// ------------------------------------------------------------ solve
struct SolvePlan {
  int prec = 0;
  bool lowp = false, need64 = false;
  KmvBufs kv;        // packed points in the solve precision
  KmvBufs kv64;      // float64 packed points (refinement / true residual) when prec != FP64
  char *X = nullptr, *R = nullptr, *Z = nullptr, *P = nullptr, *W = nullptr, *Spare = nullptr;
  double *X64 = nullptr, *R64 = nullptr, *Spare64 = nullptr;
  double *lam = nullptr, *rho = nullptr, *ab = nullptr, *rr = nullptr, *tmpc = nullptr;
  double *red = nullptr;
  int *bcol = nullptr, *restart = nullptr, *flag = nullptr, *idx = nullptr, *idx2 = nullptr;
  int *bcol2 = nullptr;
  double *lam2 = nullptr;
  char *pws = nullptr;
  size_t pws_bytes = 0;
};

void plan_solve(SolvePlan &p, int64_t n, int d, int r, int m, int prec, bool refine, bool check_true,
                Arena &ws, bool kernel = true) {
  p.prec = prec;
  p.lowp = prec != NYS_FP64;
  p.need64 = p.lowp && (refine || check_true);
  if (kernel) {
    plan_kmv(p.kv, n, n, d, 1, m, prec, ws);
    if (p.need64) plan_kmv(p.kv64, n, n, d, 1, m, NYS_FP64, ws);
  }
  const size_t vb = (size_t)n * m * elem_bytes(prec);
  p.X = ws.take<char>(vb);
  p.R = ws.take<char>(vb);
  p.Z = ws.take<char>(vb);
  p.P = ws.take<char>(vb);
  p.W = ws.take<char>(vb);
  p.Spare = ws.take<char>(vb);
  if (p.lowp && (refine || check_true)) {
    p.X64 = ws.take<double>((size_t)n * m);
    p.R64 = ws.take<double>((size_t)n * m);
    p.Spare64 = ws.take<double>((size_t)n * m);
  } else if (check_true) {
    p.R64 = ws.take<double>((size_t)n * m);
  }
  p.lam = ws.take<double>(m);
  p.rho = ws.take<double>(m);
  p.ab = ws.take<double>(m);
  p.rr = ws.take<double>(m);
  p.tmpc = ws.take<double>(m);
  const ColRedShape sh = colred_shape(n, m);
  p.red = ws.take<double>((size_t)sh.nb * m);
  p.bcol = ws.take<int>(m);
  p.restart = ws.take<int>(m);
  p.flag = ws.take<int>(m);
  p.idx = ws.take<int>(m);
  p.idx2 = ws.take<int>(m);
  p.bcol2 = ws.take<int>(m);
  p.lam2 = ws.take<double>(m);
  if (r > 0) {
    size_t mx = 0;
    for (int mm = 1; mm <= m; ++mm) mx = std::max(mx, precond_apply_scratch_bytes(n, r, mm, prec));
    p.pws_bytes = mx;
    p.pws = ws.take<char>(mx);
  }
}

// kernel_dot: the product K v into tmp, then one ordered dot product with u
struct DotPlan {
  KmvBufs kv;
  double *tmp = nullptr, *red = nullptr, *out = nullptr;
};
void plan_dot(DotPlan &p, int64_t nr, int64_t nc, int d, Arena &ws) {
  plan_kmv(p.kv, nr, nc, d, 1, 1, NYS_FP64, ws);
  p.tmp = ws.take<double>((size_t)nr);
  p.red = ws.take<double>((size_t)colred_shape(nr, 1).nb);
  p.out = ws.take<double>(2);
}

struct DerivPlan {
  KmvBufs kv;
  double *tmp = nullptr, *red = nullptr, *out = nullptr;
};
void plan_deriv(DerivPlan &p, int64_t n, int d, Arena &ws) {
  plan_kmv(p.kv, n, n, d, 1, 1, NYS_FP64, ws);
  p.tmp = ws.take<double>((size_t)n);
  p.red = ws.take<double>((size_t)colred_shape(n, 1).nb);
  p.out = ws.take<double>(2);
}

template <class T>
int32_t apply_precond_or_copy(const nys_precond *P, SolvePlan &sp, const T *R, int m, T *Z, int64_t n,
                              hipStream_t s) {
  if (!P) {
    NYS_CHECK_HIP(hipMemcpyAsync(Z, R, sizeof(T) * n * m, hipMemcpyDeviceToDevice, s));
    return NYS_OK;
  }
  Arena a;
  a.base = sp.pws;
  a.cap = sp.pws_bytes;
  return precond_apply_impl<T>(*P, sp.lam, R, m, Z, a, s);
}

// The kernel matrix as the solver's operator: products at the solve's precision and,
// for refinement, in float64 (its own packing when the solve runs in low precision).
struct KernelOp {
  const nys_kernel &k;
  const double *X;
  int d;
  SolvePlan &sp;
  int32_t prepare(hipStream_t s) {
    NYS_RETURN_IF(prep_points(sp.kv, k, sp.prec, X, X, d, s));
    if (sp.need64) NYS_RETURN_IF(prep_points(sp.kv64, k, NYS_FP64, X, X, d, s));
    return NYS_OK;
  }
  int32_t apply(const void *V, int m, int ldv, void *Out, int ldo, hipStream_t s) {
    return run_kmv(sp.kv, k, 0, sp.prec, 1, V, m, ldv, Out, ldo, 1.0, 0.0, s);
  }
  int32_t apply64(const double *V, int m, int ldv, double *Out, int ldo, hipStream_t s) {
    return run_kmv(sp.need64 ? sp.kv64 : sp.kv, k, 0, NYS_FP64, 1, V, m, ldv, Out, ldo, 1.0, 0.0, s);
  }
};

// ------------------------------------------------------------ ridge normal operator
// One rocBLAS handle per device, created on first use (plain library GEMMs).
int32_t blas_handle(rocblas_handle *out) {
  static std::mutex mu;
  static std::vector<rocblas_handle> handles;
  int dev = 0;
  NYS_CHECK_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  if ((int)handles.size() <= dev) handles.resize(dev + 1, nullptr);
  if (!handles[dev]) {
    rocblas_handle h = nullptr;
    // atomics off: the same call gives the same bits, as every other product here
    if (rocblas_create_handle(&h) != rocblas_status_success ||
        rocblas_set_atomics_mode(h, rocblas_atomics_not_allowed) != rocblas_status_success) {
      if (h) rocblas_destroy_handle(h);
      set_error("rocBLAS handle creation failed");
      return NYS_EHIP;
    }
    handles[dev] = h;
  }
  *out = handles[dev];
  return NYS_OK;
}

// The normal matrix X^T X of ridge regression (eq. experiment-ridge) on p-vectors,
// applied matrix-free as two products with the dense n x p data matrix X (row-major),
// never forming X^T X: T = X V (n x m), K V = X^T T, both float64 GEMMs.  In rocBLAS's
// column-major terms a row-major a x b matrix is its b x a transpose.
struct RidgeOp {
  const double *X;
  int64_t nrows, p;
  double *T;            // nrows x m scratch
  double *part;         // scratch of the matrix-vector kernels (ridge_part_elems)
  size_t part_cap;      // its size in doubles
  rocblas_handle h = nullptr;
  double scale = 1.0;   // the operator is scale * X^T X
  int32_t prepare(hipStream_t s) {
    NYS_RETURN_IF(blas_handle(&h));
    if (rocblas_set_stream(h, s) != rocblas_status_success) {
      set_error("rocblas_set_stream failed");
      return NYS_EHIP;
    }
    return NYS_OK;
  }
  int32_t apply(const void *V, int m, int ldv, void *Out, int ldo, hipStream_t s) {
    return apply64(reinterpret_cast<const double *>(V), m, ldv, reinterpret_cast<double *>(Out), ldo, s);
  }
  int32_t apply64(const double *V, int m, int ldv, double *Out, int ldo, hipStream_t s) {
    if (m <= 0) return NYS_OK;
    NYS_RETURN_IF(prepare(s));
    const double one = 1.0, zero = 0.0;
    if (m == 1) {
      // one column: two matrix-vector products of our own, each a single pass over X
      NYS_RETURN_IF(launch_rowdot(X, nrows, p, V, ldv, T, s));
      return launch_coltrans(X, nrows, p, T, scale, Out, ldo, part, s);
    }
    if (rocblas_dgemm_64(h, rocblas_operation_none, rocblas_operation_none, m, (int64_t)nrows, (int64_t)p, &one,
                      V, ldv, X, (int64_t)p, &zero, T, m) != rocblas_status_success) {
      set_error("rocblas_dgemm failed in the ridge operator");
      return NYS_EHIP;
    }
    // Out = X^T T has a long inner dimension (the n rows).  With few 128 x 128 output
    // tiles (small p) the library GEMM leaves most CUs idle; the row-split kernel
    // spreads the rows instead.
    if (ceil_div(p, 128) * ceil_div(m, 128) < 512 && gemv_partial_elems(nrows, p, m) <= part_cap)
      return launch_coltrans_multi(X, nrows, p, T, m, m, scale, Out, ldo, part, s);
    if (rocblas_dgemm_64(h, rocblas_operation_none, rocblas_operation_transpose, m, (int64_t)p, (int64_t)nrows,
                         &scale, T, m, X, (int64_t)p, &zero, Out, ldo) != rocblas_status_success) {
      set_error("rocblas_dgemm failed in the ridge operator");
      return NYS_EHIP;
    }
    return NYS_OK;
  }
};

// scratch of RidgeOp's matrix-vector kernels for products of one and of m columns
size_t ridge_part_elems(int64_t n, int64_t p, int m) {
  return std::max(gemv_partial_elems(n, p, 1), gemv_partial_elems(n, p, std::max(m, 1)));
}

// Scratch of the ridge calls: the normal-operator intermediate (n x m) and, for the
// solve, the right-hand sides X^T y (p x nrhs); for the sketch, the Cholesky QR.
struct RidgeSketchPlan {
  double *G = nullptr, *Gpart = nullptr, *Linv = nullptr, *LinvT = nullptr, *Om = nullptr, *T = nullptr;
  double *part = nullptr;
  size_t part_cap = 0;
  int *flag = nullptr;
};
void plan_ridge_sketch(RidgeSketchPlan &p, int64_t n, int64_t pd, int r, Arena &ws) {
  const int splits = gemm_tn_splits(pd, r, r);
  p.G = ws.take<double>((size_t)r * r);
  p.Gpart = ws.take<double>((size_t)splits * r * r);
  p.Linv = ws.take<double>((size_t)r * r);
  p.LinvT = ws.take<double>((size_t)r * r);
  p.Om = ws.take<double>((size_t)pd * r);
  p.T = ws.take<double>((size_t)n * r);
  p.part_cap = ridge_part_elems(n, pd, r);
  p.part = ws.take<double>(p.part_cap);
  p.flag = ws.take<int>(4);
}
struct RidgeSolvePlan {
  SolvePlan sp;
  double *T = nullptr, *B = nullptr, *part = nullptr;
  size_t part_cap = 0;
};
void plan_ridge_solve(RidgeSolvePlan &p, int64_t n, int64_t pd, int r, int nrhs, int m, Arena &ws) {
  plan_solve(p.sp, pd, 1, r, m, NYS_FP64, false, true, ws, false);
  p.T = ws.take<double>((size_t)n * m);
  p.B = ws.take<double>((size_t)pd * nrhs);
  p.part_cap = ridge_part_elems(n, pd, m);
  p.part = ws.take<double>(p.part_cap);
}

// Q = Omega L^-T with L L^T = Omega^T Omega (Cholesky QR, float64): the orthonormalised
// pd x r test matrix; Omega NULL draws it from the seed (nys_test_matrix).  Synchronises.
int32_t orth_test_matrix(const double *Omega, uint64_t seed, int64_t pd, int r, RidgeSketchPlan &pl, double *Q,
                         hipStream_t s) {
  const int64_t cnt = pd * (int64_t)r;
  const double *Om = Omega;
  if (!Om) {
    NYS_RETURN_IF(launch_gaussian(seed, cnt, pl.Om, s));
    Om = pl.Om;
  }
  const int splits = gemm_tn_splits(pd, r, r);
  NYS_RETURN_IF(gemm_tn<double>(Om, r, Om, r, pd, r, r, pl.G, r, pl.Gpart, splits, s));
  NYS_RETURN_IF(launch_chol(pl.G, r, pl.flag, s));
  int flag = 0;
  NYS_CHECK_HIP(hipMemcpyAsync(&flag, pl.flag, sizeof(int), hipMemcpyDeviceToHost, s));
  NYS_CHECK_HIP(hipStreamSynchronize(s));
  if (flag) {
    set_error("the test matrix Omega is rank deficient or not finite");
    return NYS_ENOTPD;
  }
  NYS_RETURN_IF(launch_trinv_lower(pl.G, pl.Linv, r, s));
  NYS_RETURN_IF(launch_transpose(pl.Linv, pl.LinvT, r, s));
  NYS_RETURN_IF(gemm_nn<double>(Om, r, pl.LinvT, r, pd, r, r, Q, r, 0, nullptr, 0, nullptr, s));
  return NYS_OK;
}

// The PCG driver (solve_columns) and its block variant (solve_blocks).
#include "solve_impl.h"
#include "block_impl.h"

// The stabilised approximation from a sketch (Y, Q of r columns): fills P->U (n x r),
// P->lam_hat, P->U32 (when given), P->rank and P->nu.
int32_t build_impl(const double *Y, const double *Q, int64_t n, int r, int sketch_prec, nys_precond *P,
                   BuildPlan &p, hipStream_t s) {
  const int64_t cnt = n * (int64_t)r;
  NYS_RETURN_IF(launch_sumsq(Y, cnt, p.ssq_part, p.ssq, s));
  double ssq = 0.0;
  NYS_CHECK_HIP(hipMemcpyAsync(&ssq, p.ssq, sizeof(double), hipMemcpyDeviceToHost, s));
  NYS_CHECK_HIP(hipStreamSynchronize(s));
  if (!std::isfinite(ssq)) {
    set_error("nys_precond_build: NaN or Inf in the sketch");
    return NYS_ENUMERIC;
  }
  const double yf = std::sqrt(ssq);
  const double cprec = sketch_prec == NYS_FP64 ? 0.0 : (sketch_prec == NYS_FP32 ? std::ldexp(1.0, -21) : std::ldexp(1.0, -14));
  double nu = std::max(std::sqrt((double)n) * std::ldexp(1.0, -52) * yf, cprec * yf / std::sqrt((double)r));
  if (!(nu > 0.0)) nu = std::ldexp(1.0, -52);
  const int splits = gemm_tn_splits(n, r, r);
  bool ok = false;
  for (int attempt = 0; attempt < 6; ++attempt) {
    NYS_CHECK_HIP(hipMemcpyAsync(p.Ynu, Y, sizeof(double) * cnt, hipMemcpyDeviceToDevice, s));
    NYS_RETURN_IF(launch_axpy(nu, Q, p.Ynu, cnt, s));
    NYS_RETURN_IF(gemm_tn<double>(Q, r, p.Ynu, r, n, r, r, p.M, r, p.Mpart, splits, s));
    NYS_RETURN_IF(launch_symmetrise(p.M, p.L, r, s));
    NYS_RETURN_IF(launch_chol(p.L, r, p.flag, s));
    int flag = 0;
    NYS_CHECK_HIP(hipMemcpyAsync(&flag, p.flag, sizeof(int), hipMemcpyDeviceToHost, s));
    NYS_CHECK_HIP(hipStreamSynchronize(s));
    if (flag == 0) {
      ok = true;
      break;
    }
    nu *= 10.0;
  }
  if (!ok) {
    set_error("nys_precond_build: shifted Cholesky of the sketch core failed after 5 retries");
    return NYS_ENOTPD;
  }
  // B = Y_nu L^{-T};  B^T B = V S^2 V^T;  U = B V S^{-1}
  NYS_RETURN_IF(launch_trinv_lower(p.L, p.Linv, r, s));
  NYS_RETURN_IF(launch_transpose(p.Linv, p.LinvT, r, s));
  NYS_RETURN_IF(gemm_nn<double>(p.Ynu, r, p.LinvT, r, n, r, r, p.Bm, r, 0, nullptr, 0, nullptr, s));
  NYS_RETURN_IF(gemm_tn<double>(p.Bm, r, p.Bm, r, n, r, r, p.G, r, p.Mpart, splits, s));
  NYS_RETURN_IF(launch_symmetrise(p.G, p.Gs, r, s));
  NYS_RETURN_IF(jacobi_eig(p.Gs, p.Gbuf, p.Vev, p.w, r, p.jac, s));
  NYS_RETURN_IF(launch_eig_finish(p.w, p.Vev, r, nu, p.T, P->lam_hat, p.rank, s));
  NYS_RETURN_IF(gemm_nn<double>(p.Bm, r, p.T, r, n, r, r, P->U, r, 0, nullptr, 0, nullptr, s));
  if (P->U32) NYS_RETURN_IF(launch_copy_d2f(P->U, P->U32, cnt, s));
  int rank = 0;
  NYS_CHECK_HIP(hipMemcpyAsync(&rank, p.rank, sizeof(int), hipMemcpyDeviceToHost, s));
  NYS_CHECK_HIP(hipStreamSynchronize(s));
  P->rank = rank;
  P->nu = nu;
  return NYS_OK;
}

// ------------------------------------------------------------ rank adaptation
// Scratch of nys_precond_adaptive: the test matrix and K times it (n x rank_max), the
// orthonormalised sketch of the current rank, the Cholesky QR factors, the build, and
// the vectors of the power iteration.
struct AdaptPlan {
  double *Om = nullptr, *Yraw = nullptr, *Q = nullptr, *Y = nullptr;
  float *O32 = nullptr, *Y32 = nullptr, *v32 = nullptr, *w32 = nullptr;
  double *G = nullptr, *Gpart = nullptr, *Linv = nullptr, *LinvT = nullptr;
  double *v = nullptr, *w = nullptr, *t = nullptr, *c = nullptr, *cpart = nullptr, *red = nullptr, *out = nullptr;
  int *flag = nullptr;
  KmvBufs kv;
  BuildPlan bp;
};
void plan_adapt(AdaptPlan &p, int64_t n, int d, int rmax, int prec, Arena &ws) {
  const size_t cnt = (size_t)n * rmax;
  p.Om = ws.take<double>(cnt);
  p.Yraw = ws.take<double>(cnt);
  p.Q = ws.take<double>(cnt);
  p.Y = ws.take<double>(cnt);
  if (prec != NYS_FP64) {
    p.O32 = ws.take<float>(cnt);
    p.Y32 = ws.take<float>(cnt);
    p.v32 = ws.take<float>((size_t)n);
    p.w32 = ws.take<float>((size_t)n);
  }
  const int splits = gemm_tn_splits(n, rmax, rmax);
  p.G = ws.take<double>((size_t)rmax * rmax);
  p.Gpart = ws.take<double>((size_t)splits * rmax * rmax);
  p.Linv = ws.take<double>((size_t)rmax * rmax);
  p.LinvT = ws.take<double>((size_t)rmax * rmax);
  p.flag = ws.take<int>(4);
  p.v = ws.take<double>((size_t)n);
  p.w = ws.take<double>((size_t)n);
  p.t = ws.take<double>((size_t)n);
  p.c = ws.take<double>((size_t)rmax);
  p.cpart = ws.take<double>((size_t)gemm_tn_splits(n, rmax, 1) * rmax);
  p.red = ws.take<double>((size_t)colred_shape(n, 1).nb);
  p.out = ws.take<double>(2);
  plan_kmv(p.kv, n, n, d, 1, rmax, prec, ws);
  plan_build(p.bp, n, rmax, ws);
}

__global__ void scale_vec_kernel(const double *x, const double *coef, double *y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = coef[i] * x[i];
}
__global__ void scale_by_kernel(double *y, double a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] *= a;
}

// host value of a . b (float64 vectors of n)
int32_t dot_host(const double *a, const double *b, int64_t n, double *red, double *out, double *h, hipStream_t s) {
  NYS_RETURN_IF(colred<double>(0, a, const_cast<double *>(b), nullptr, nullptr, n, 1, nullptr, red, s));
  NYS_RETURN_IF(colfinal(red, n, 1, 0, out, nullptr, nullptr, nullptr, nullptr, s));
  NYS_CHECK_HIP(hipMemcpyAsync(h, out, sizeof(double), hipMemcpyDeviceToHost, s));
  NYS_CHECK_HIP(hipStreamSynchronize(s));
  return NYS_OK;
}

// Rank doubling: K is applied only to the test-matrix columns added since the last
// round (Yraw = K Omega), the first l columns are orthonormalised by Cholesky QR
// (Q = Omega_l L^-T, Y = Yraw_l L^-T: the same sketch as K Q), the approximation is
// built, and its error |K - K_hat|_2 is estimated by power iterations.
int32_t adaptive_impl(const nys_kernel &k, int prec, const double *X, int64_t n, int d, const nys_nystrom_config &cfg,
                      int rmax, nys_precond *P, double *err_out, AdaptPlan &p, hipStream_t s) {
  const int64_t cnt = n * (int64_t)rmax;
  NYS_RETURN_IF(launch_gaussian(cfg.seed, cnt, p.Om, s));
  if (prec != NYS_FP64) NYS_RETURN_IF(launch_copy_d2f(p.Om, p.O32, cnt, s));
  NYS_RETURN_IF(prep_points(p.kv, k, prec, X, X, d, s));
  int l = std::min(cfg.rank_init, rmax), done_cols = 0;
  double err = 0.0;
  const unsigned gb = (unsigned)ceil_div(n, 256);
  while (true) {
    // K times the new columns
    if (prec == NYS_FP64) {
      NYS_RETURN_IF(run_kmv(p.kv, k, 0, prec, 1, p.Om + done_cols, l - done_cols, rmax, p.Yraw + done_cols, rmax,
                            1.0, 0.0, s));
    } else {
      NYS_RETURN_IF(run_kmv(p.kv, k, 0, prec, 1, p.O32 + done_cols, l - done_cols, rmax, p.Y32 + done_cols, rmax,
                            1.0, 0.0, s));
      NYS_RETURN_IF(launch_copy_f2d(p.Y32, p.Yraw, cnt, s));
    }
    done_cols = l;
    // Cholesky QR of the first l columns
    const int splits = gemm_tn_splits(n, l, l);
    NYS_RETURN_IF(gemm_tn<double>(p.Om, rmax, p.Om, rmax, n, l, l, p.G, l, p.Gpart, splits, s));
    NYS_RETURN_IF(launch_chol(p.G, l, p.flag, s));
    int flag = 0;
    NYS_CHECK_HIP(hipMemcpyAsync(&flag, p.flag, sizeof(int), hipMemcpyDeviceToHost, s));
    NYS_CHECK_HIP(hipStreamSynchronize(s));
    if (flag) {
      set_error("nys_precond_adaptive: the test matrix is rank deficient");
      return NYS_ENOTPD;
    }
    NYS_RETURN_IF(launch_trinv_lower(p.G, p.Linv, l, s));
    NYS_RETURN_IF(launch_transpose(p.Linv, p.LinvT, l, s));
    NYS_RETURN_IF(gemm_nn<double>(p.Om, rmax, p.LinvT, l, n, l, l, p.Q, l, 0, nullptr, 0, nullptr, s));
    NYS_RETURN_IF(gemm_nn<double>(p.Yraw, rmax, p.LinvT, l, n, l, l, p.Y, l, 0, nullptr, 0, nullptr, s));
    nys_precond Pl = *P;
    Pl.r = l;
    NYS_RETURN_IF(build_impl(p.Y, p.Q, n, l, prec, &Pl, p.bp, s));
    P->rank = Pl.rank;
    P->nu = Pl.nu;
    P->r = l;
    // power iteration on E = K - U diag(lam_hat) U^T from a seeded start vector
    err = 0.0;
    if (cfg.num_power_iters > 0) {
      double h = 0.0;
      NYS_RETURN_IF(launch_gaussian(cfg.seed + 1, n, p.v, s));
      NYS_RETURN_IF(dot_host(p.v, p.v, n, p.red, p.out, &h, s));
      hipLaunchKernelGGL(scale_by_kernel, dim3(gb), dim3(256), 0, s, p.v, 1.0 / std::sqrt(h), n);
      NYS_LAUNCH_CHECK();
      for (int it = 0; it < cfg.num_power_iters; ++it) {
        if (prec == NYS_FP64) {
          NYS_RETURN_IF(run_kmv(p.kv, k, 0, prec, 1, p.v, 1, 1, p.w, 1, 1.0, 0.0, s));
        } else {
          NYS_RETURN_IF(launch_copy_d2f(p.v, p.v32, n, s));
          NYS_RETURN_IF(run_kmv(p.kv, k, 0, prec, 1, p.v32, 1, 1, p.w32, 1, 1.0, 0.0, s));
          NYS_RETURN_IF(launch_copy_f2d(p.w32, p.w, n, s));
        }
        const int cs = gemm_tn_splits(n, l, 1);
        NYS_RETURN_IF(gemm_tn<double>(P->U, l, p.v, 1, n, l, 1, p.c, 1, p.cpart, cs, s));
        hipLaunchKernelGGL(scale_vec_kernel, dim3((unsigned)ceil_div(l, 256)), dim3(256), 0, s, p.c, P->lam_hat,
                           p.c, (int64_t)l);
        NYS_LAUNCH_CHECK();
        NYS_RETURN_IF(gemm_nn<double>(P->U, l, p.c, 1, n, l, 1, p.t, 1, 0, nullptr, 0, nullptr, s));
        NYS_RETURN_IF(launch_axpy(-1.0, p.t, p.w, n, s));           // w = E v
        NYS_RETURN_IF(dot_host(p.v, p.w, n, p.red, p.out, &err, s));   // Rayleigh quotient
        NYS_RETURN_IF(dot_host(p.w, p.w, n, p.red, p.out, &h, s));
        if (!(h > 0.0) || !std::isfinite(h)) break;
        NYS_CHECK_HIP(hipMemcpyAsync(p.v, p.w, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        hipLaunchKernelGGL(scale_by_kernel, dim3(gb), dim3(256), 0, s, p.v, 1.0 / std::sqrt(h), n);
        NYS_LAUNCH_CHECK();
      }
    }
    double lam1 = 0.0;
    NYS_CHECK_HIP(hipMemcpyAsync(&lam1, P->lam_hat, sizeof(double), hipMemcpyDeviceToHost, s));
    NYS_CHECK_HIP(hipStreamSynchronize(s));
    if (err <= cfg.error_tolerance * lam1 || l >= rmax) break;
    l = std::min(2 * l, rmax);
  }
  // the build wrote U as n x l (row stride l) at the start of the n x rank_max buffer;
  // zero the unused tail of lam_hat so that the buffers describe exactly the result
  if (P->r < rmax) NYS_RETURN_IF(launch_fill(P->lam_hat + P->r, 0.0, rmax - P->r, s));
  P->shift = 0.0;
  if (cfg.damping_mode == NYS_DAMPING_ADAPTIVE && P->rank > 0) {
    NYS_CHECK_HIP(hipMemcpyAsync(&P->shift, P->lam_hat + (P->rank - 1), sizeof(double), hipMemcpyDeviceToHost, s));
  }
  NYS_CHECK_HIP(hipStreamSynchronize(s));
  if (err_out) *err_out = err;
  return NYS_OK;
}

int32_t check_precond(const nys_precond *P, int64_t n, int prec) {
  if (!P) return NYS_OK;
  if (P->n != n) return einval("preconditioner built for a different n");
  if (P->r < 1 || !P->U || !P->lam_hat) return einval("preconditioner buffers missing");
  (void)prec;
  return NYS_OK;
}

int32_t check_opts(const nys_pcg_opts *o) {
  if (!o) return einval("opts is NULL");
  if (!(o->tol > 0.0) || !std::isfinite(o->tol)) return einval("tol must be positive");
  if (o->max_iters < 0) return einval("max_iters must be >= 0");
  if (!valid_prec(o->prec)) return einval("unsupported precision");
  if (o->refine_mode < 0 || o->refine_mode > 2) return einval("refine_mode must be 0, 1 or 2");
  if (!(o->refine_join == 0.0 || o->refine_join >= 1.0) || !std::isfinite(o->refine_join))
    return einval("refine_join must be 0 or >= 1");
  if (o->block != 0 && o->block != 1) return einval("block must be 0 or 1");
  return NYS_OK;
}

// ------------------------------------------------------------ NysADMM (bounded elastic net)
struct AdmmPlan {
  double *Xc = nullptr, *ones = nullptr, *mu = nullptr, *c = nullptr;
  double *x = nullptr, *z = nullptr, *u = nullptr, *dx = nullptr, *rhs = nullptr, *r0 = nullptr, *Hx = nullptr;
  double *partial = nullptr, *out = nullptr, *U = nullptr, *lam_hat = nullptr, *Q = nullptr, *Y = nullptr;
  double *redn = nullptr;  // partials of one length-n dot product
  RidgeSketchPlan sk;
  BuildPlan bp;
  SolvePlan sp;
};
void plan_admm(AdmmPlan &p, int64_t n, int64_t pd, int r, Arena &ws) {
  p.Xc = ws.take<double>((size_t)n * pd);
  p.ones = ws.take<double>((size_t)n);
  p.redn = ws.take<double>((size_t)colred_shape(n, 1).nb);
  for (double **v : {&p.mu, &p.c, &p.x, &p.z, &p.u, &p.dx, &p.rhs, &p.r0, &p.Hx}) *v = ws.take<double>((size_t)pd);
  p.partial = ws.take<double>(admm_partial_elems(pd));
  p.out = ws.take<double>(8);
  p.U = ws.take<double>((size_t)pd * r);
  p.lam_hat = ws.take<double>((size_t)r);
  p.Q = ws.take<double>((size_t)pd * r);
  p.Y = ws.take<double>((size_t)pd * r);
  plan_ridge_sketch(p.sk, n, pd, r, ws);
  plan_build(p.bp, pd, r, ws);
  plan_solve(p.sp, pd, 1, r, 1, NYS_FP64, false, false, ws, false);
}

int32_t admm_config(const nys_admm_config *in, int64_t p, nys_admm_config &c) {
  c = *in;
  auto dflt = [](double v, double d) { return v == 0.0 ? d : v; };
  c.rho = dflt(c.rho, 1.0);
  c.rho_update_factor = dflt(c.rho_update_factor, 2.0);
  c.rho_update_threshold = dflt(c.rho_update_threshold, 10.0);
  c.alpha = dflt(c.alpha, 1.6);
  c.sigma = dflt(c.sigma, 1e-6);
  c.gamma = dflt(c.gamma, 1.2);
  c.eps_abs = dflt(c.eps_abs, 1e-4);
  c.eps_rel = dflt(c.eps_rel, 1e-4);
  if (c.rho_update_freq == 0) c.rho_update_freq = 25;
  if (c.precond_update_freq == 0) c.precond_update_freq = 20;
  if (c.rank == 0) c.rank = (int32_t)std::min<int64_t>(50, p);
  if (c.max_iters == 0) c.max_iters = 1000;
  if (c.pcg_max_iters == 0) c.pcg_max_iters = 1000;
  const bool fin = std::isfinite(c.rho) && std::isfinite(c.rho_update_factor) &&
                   std::isfinite(c.rho_update_threshold) && std::isfinite(c.alpha) && std::isfinite(c.sigma) &&
                   std::isfinite(c.gamma) && std::isfinite(c.eps_abs) && std::isfinite(c.eps_rel);
  if (!fin || c.rho <= 0.0 || c.rho_update_factor <= 1.0 || c.rho_update_threshold < 1.0 || c.alpha <= 0.0 ||
      c.alpha >= 2.0 || c.sigma < 0.0 || c.gamma <= 1.0 || c.eps_abs < 0.0 || c.eps_rel < 0.0 ||
      c.eps_abs + c.eps_rel <= 0.0)
    return einval("nys_admm_config: a parameter is out of range (rho > 0, factor > 1, threshold >= 1, "
                  "0 < alpha < 2, sigma >= 0, gamma > 1, tolerances >= 0 and not both 0)");
  if (c.rho_update_freq < 1 || c.precond_update_freq < 1 || c.max_iters < 1 || c.pcg_max_iters < 1)
    return einval("nys_admm_config: iteration counts must be >= 1");
  if (c.rank < 1 || c.rank > p || c.rank > 1024) return einval("nys_admm_config: need 1 <= rank <= min(p, 1024)");
  return NYS_OK;
}

// The iteration of nys_admm_elastic_net (documented with its declaration).
int32_t admm_impl(const double *X, int64_t n, int64_t pd, const double *y, double lam1, double lam2, double lo,
                  double hi, const nys_admm_config &c, double *W, nys_admm_info *info, AdmmPlan &pl,
                  hipStream_t s) {
  const int r = c.rank;
  const double inv_n = 1.0 / (double)n;
  RidgeOp op{pl.Xc, n, pd, pl.sk.T, pl.sk.part, pl.sk.part_cap};
  op.scale = inv_n;
  NYS_RETURN_IF(op.prepare(s));
  // centring: mu = X^T 1 / n, Xc = X - 1 mu^T, c = Xc^T y / n (Xc^T 1 = 0), ybar
  NYS_RETURN_IF(launch_fill(pl.ones, 1.0, n, s));
  NYS_RETURN_IF(launch_coltrans(X, n, pd, pl.ones, inv_n, pl.mu, 1, pl.sk.part, s));
  NYS_RETURN_IF(admm_center(X, pl.mu, n, pd, pl.Xc, s));
  NYS_RETURN_IF(launch_coltrans(pl.Xc, n, pd, y, inv_n, pl.c, 1, pl.sk.part, s));
  double ybar = 0.0;
  NYS_RETURN_IF(dot_host(pl.ones, y, n, pl.redn, pl.out, &ybar, s));
  ybar *= inv_n;
  if (!std::isfinite(ybar)) {
    set_error("nys_admm_elastic_net: NaN or Inf in y");
    return NYS_ENUMERIC;
  }
  for (double *v : {pl.x, pl.z, pl.u, pl.Hx}) NYS_RETURN_IF(launch_fill(v, 0.0, pd, s));

  nys_precond P{};
  P.n = pd;
  P.r = r;
  P.U = pl.U;
  P.U32 = nullptr;
  P.lam_hat = pl.lam_hat;
  nys_pcg_opts po{};
  po.max_iters = c.pcg_max_iters;
  po.prec = NYS_FP64;
  po.refine_every = -1;

  double rho = c.rho, rp = 0.0, rd = 0.0, eps_pri = 0.0, eps_dual = 0.0;
  int64_t pcg_total = 0;
  bool converged = false;
  int k = 0;
  const double sq = std::sqrt((double)pd);
  const bool verbose = std::getenv("NYS_VERBOSE") != nullptr;
  for (k = 1; k <= c.max_iters; ++k) {
    if ((k - 1) % c.precond_update_freq == 0) {
      const uint64_t sd = c.seed + (uint64_t)((k - 1) / c.precond_update_freq);
      NYS_RETURN_IF(orth_test_matrix(nullptr, sd, pd, r, pl.sk, pl.Q, s));
      NYS_RETURN_IF(op.apply64(pl.Q, r, r, pl.Y, r, s));
      NYS_RETURN_IF(build_impl(pl.Y, pl.Q, pd, r, NYS_FP64, &P, pl.bp, s));
    }
    // x-subproblem, warm-started: solve A dx = r0 with r0 = rhs - A x_prev
    NYS_RETURN_IF(admm_rhs(pl.c, pl.z, pl.u, pl.x, pl.Hx, rho, c.sigma, pd, pl.rhs, pl.r0, pl.partial, pl.out, s));
    double nn[2];
    NYS_CHECK_HIP(hipMemcpyAsync(nn, pl.out, sizeof(nn), hipMemcpyDeviceToHost, s));
    NYS_CHECK_HIP(hipStreamSynchronize(s));
    const double bn = std::sqrt(nn[0]), r0n = std::sqrt(nn[1]);
    if (!std::isfinite(bn) || !std::isfinite(r0n)) {
      set_error("nys_admm_elastic_net: NaN or Inf in the x-subproblem");
      return NYS_ENUMERIC;
    }
    const double scale = k == 1 ? 1.0 : std::min(1.0, std::sqrt(rp * rd));
    const double tol_k = std::max(scale * std::pow((double)k, -c.gamma), 1e-15);
    const double *dx = nullptr;
    if (bn > 0.0 && r0n > tol_k * bn) {
      po.tol = tol_k * bn / r0n;
      const double lk = rho + c.sigma;
      nys_col_info ci{};
      const int32_t rc = solve_columns<double>(op, pd, pl.r0, 1, &lk, 1, &P, po, pl.dx, &ci, pl.sp, s);
      if (rc != NYS_OK && rc != NYS_NOT_CONVERGED) return rc;
      pcg_total += ci.iters;
      dx = pl.dx;
    }
    NYS_RETURN_IF(admm_update(pl.x, dx, c.alpha, pl.z, pl.u, rho, lam1, lam2, lo, hi, pd, pl.partial, s));
    NYS_RETURN_IF(op.apply64(pl.x, 1, 1, pl.Hx, 1, s));
    NYS_RETURN_IF(admm_dual(pl.Hx, pl.c, pl.u, rho, pd, pl.partial, pl.out, s));
    double q[5];
    NYS_CHECK_HIP(hipMemcpyAsync(q, pl.out, sizeof(q), hipMemcpyDeviceToHost, s));
    NYS_CHECK_HIP(hipStreamSynchronize(s));
    rp = std::sqrt(q[0]);
    rd = std::sqrt(q[3]);
    eps_pri = sq * c.eps_abs + c.eps_rel * std::max(std::sqrt(q[1]), std::sqrt(q[2]));
    eps_dual = sq * c.eps_abs + c.eps_rel * std::sqrt(q[4]);
    if (!std::isfinite(rp) || !std::isfinite(rd)) {
      set_error("nys_admm_elastic_net: NaN or Inf in the residuals");
      return NYS_ENUMERIC;
    }
    if (verbose) {
      std::fprintf(stderr, "[nys] admm %d rho %.3g r_pri %.3e (%.3e) r_dual %.3e (%.3e) pcg %lld\n", k, rho, rp,
                   eps_pri, rd, eps_dual, (long long)pcg_total);
      std::fflush(stderr);
    }
    if (rp <= eps_pri && rd <= eps_dual) {
      converged = true;
      break;
    }
    if (k % c.rho_update_freq == 0) {
      if (rp > c.rho_update_threshold * rd) {
        rho *= c.rho_update_factor;
        NYS_RETURN_IF(admm_scale(pl.u, 1.0 / c.rho_update_factor, pd, s));
      } else if (rd > c.rho_update_threshold * rp) {
        rho /= c.rho_update_factor;
        NYS_RETURN_IF(admm_scale(pl.u, c.rho_update_factor, pd, s));
      }
    }
  }
  NYS_CHECK_HIP(hipMemcpyAsync(W, pl.z, sizeof(double) * (size_t)pd, hipMemcpyDeviceToDevice, s));
  double muz = 0.0;
  NYS_RETURN_IF(dot_host(pl.mu, pl.z, pd, pl.sp.red, pl.out, &muz, s));
  info->iters = std::min(k, c.max_iters);
  info->converged = converged ? 1 : 0;
  info->pcg_iters = pcg_total;
  info->r_pri = rp;
  info->r_dual = rd;
  info->eps_pri = eps_pri;
  info->eps_dual = eps_dual;
  info->rho = rho;
  info->intercept = ybar - muz;
  return converged ? NYS_OK : NYS_NOT_CONVERGED;
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

const char *nys_last_error(void) { return last_error_cstr(); }

int32_t nys_peak_probe(int32_t which, int32_t iters, double *rate, void *ws, size_t ws_bytes, void *stream) {
  return peak_probe(which, iters, rate, ws, ws_bytes, as_stream(stream));
}
const char *nys_version(void) { return "libnys 0.1.0 (gfx950)"; }

int32_t nys_workspace_bytes(int32_t op, int64_t n, int64_t n2, int32_t d, int32_t r, int32_t m,
                            int32_t prec, size_t *bytes) {
  if (!bytes) return einval("bytes is NULL");
  if (n < 0 || n2 < 0 || d < 0 || r < 0 || m < 0) return einval("negative size");
  if (!valid_prec(prec)) return einval("unsupported precision");
  Arena a;
  switch (op) {
    case NYS_OP_KERNEL_MATVEC: {
      MatvecPlan p;
      plan_matvec(p, std::max<int64_t>(n, 1), std::max<int64_t>(n2, 1), std::max(d, 1), std::max(m, 1), prec, a);
      break;
    }
    case NYS_OP_SKETCH: {
      SketchPlan p;
      plan_sketch(p, std::max<int64_t>(n, 1), std::max(d, 1), std::max(r, 1), prec, a);
      break;
    }
    case NYS_OP_PRECOND_BUILD: {
      BuildPlan p;
      plan_build(p, std::max<int64_t>(n, 1), std::max(r, 1), a);
      break;
    }
    case NYS_OP_PRECOND_APPLY:
      a.off = precond_apply_scratch_bytes(std::max<int64_t>(n, 1), std::max(r, 1), std::max(m, 1), prec);
      break;
    case NYS_OP_SOLVE: {
      SolvePlan p;
      plan_solve(p, std::max<int64_t>(n, 1), std::max(d, 1), r, std::max(m, 1), prec, true, true, a);
      BlockPlan b;
      plan_block(b, std::max<int64_t>(n, 1), std::max(m, 1), a);
      break;
    }
    case NYS_OP_BACKWARD: {
      SolvePlan p;
      plan_solve(p, std::max<int64_t>(n, 1), std::max(d, 1), r, 1, prec, true, true, a);
      DerivPlan q;
      plan_deriv(q, std::max<int64_t>(n, 1), std::max(d, 1), a);
      break;
    }
    case NYS_OP_PRECOND_ADAPTIVE: {
      AdaptPlan p;
      plan_adapt(p, std::max<int64_t>(n, 1), std::max(d, 1), std::max(r, 1), prec, a);
      break;
    }
    case NYS_OP_RIDGE_SKETCH: {
      RidgeSketchPlan p;
      plan_ridge_sketch(p, std::max<int64_t>(n, 1), std::max<int64_t>(n2, 1), std::max(r, 1), a);
      break;
    }
    case NYS_OP_RIDGE_SOLVE: {
      RidgeSolvePlan p;
      plan_ridge_solve(p, std::max<int64_t>(n, 1), std::max<int64_t>(n2, 1), r, std::max(d, 1), std::max(m, 1), a);
      break;
    }
    case NYS_OP_ADMM_ELASTIC_NET: {
      AdmmPlan p;
      plan_admm(p, std::max<int64_t>(n, 1), std::max<int64_t>(n2, 1), std::max(r, 1), a);
      break;
    }
    case NYS_OP_KERNEL_DOT: {
      DotPlan p;
      plan_dot(p, std::max<int64_t>(n, 1), std::max<int64_t>(n2, 1), std::max(d, 1), a);
      break;
    }
    case NYS_OP_AUTOTUNE: {
      AutotunePlan p;
      NYS_RETURN_IF(plan_autotune(p, std::max<int64_t>(n, 1), std::max<int64_t>(n2, 1), std::max(d, 1),
                                  std::max(m, 1), prec, a));
      break;
    }
    default:
      return einval("unknown op");
  }
  *bytes = a.off;
  return NYS_OK;
}

// ------------------------------------------------------------ autotuner
int32_t nys_set_tile(int32_t prec, int32_t m_lo, int32_t m_hi, int32_t tm) {
  if (!valid_prec(prec)) return einval("unsupported precision");
  if (m_lo < 1 || m_hi < m_lo) return einval("need 1 <= m_lo <= m_hi");
  const int key = tile_key(prec);
  if (tm != 0 && !kmv_tile_valid(key, tm)) return einval("no tile of this width for this precision");
  kmv_tune_set(key, m_lo, m_hi, tm);
  return NYS_OK;
}

void nys_clear_tiles(void) { kmv_tune_clear(); }

int32_t nys_plan_chunks(int32_t prec, int64_t n, int32_t d, int32_t m, int32_t *tm, int32_t *tail_tm) {
  if (!valid_prec(prec)) return einval("unsupported precision");
  if (n < 1 || m < 1) return einval("need n >= 1 and m >= 1");
  if (d < 1 || d > max_dim(prec)) return einval("d out of range for this precision");
  if (!tm || !tail_tm) return einval("null pointer");
  const KmvPlan p = kmv_plan(n, n, m, prec, packed_kp(d, prec));
  *tm = p.path == 1 ? p.tm : 0;
  *tail_tm = p.path == 1 ? p.tail_tm : 0;
  return NYS_OK;
}

int32_t nys_plan_ranges(int32_t prec, int64_t n, int32_t d, int32_t m, int32_t *ranges, int64_t *points) {
  if (!valid_prec(prec)) return einval("unsupported precision");
  if (n < 1 || m < 1) return einval("need n >= 1 and m >= 1");
  if (d < 1 || d > max_dim(prec)) return einval("d out of range for this precision");
  if (!ranges || !points) return einval("null pointer");
  const KmvPlan p = kmv_plan(n, n, m, prec, packed_kp(d, prec));
  const int64_t tj = p.path == 0 ? 64 : 32;   // column points per tile of the plan's path
  *ranges = p.splits;
  *points = std::min<int64_t>((int64_t)p.jsteps * tj, n);
  return NYS_OK;
}

int32_t nys_autotune(nys_kernel k, int32_t prec, const double *X, int64_t n, int64_t n_rows, int32_t d,
                     int32_t m, int32_t m_lo, int32_t reps, nys_tile_choice *best, void *ws, size_t ws_bytes,
                     void *stream) {
  NYS_RETURN_IF(check_kernel(k));
  if (!valid_prec(prec)) return einval("unsupported precision");
  if (n < 1 || n_rows < 1 || n_rows > n) return einval("need 1 <= n_rows <= n");
  if (d < 1 || d > max_dim(prec)) return einval("d out of range for this precision");
  if (m < 1 || m_lo < 1 || m_lo > m || reps < 1) return einval("need 1 <= m_lo <= m and reps >= 1");
  if (!X || !best || !ws) return einval("null pointer");
  hipStream_t s = as_stream(stream);
  Arena a;
  a.base = reinterpret_cast<char *>(ws);
  a.cap = ws_bytes;
  AutotunePlan p;
  NYS_RETURN_IF(plan_autotune(p, n_rows, n, d, m, prec, a));
  NYS_RETURN_IF(check_ws(a));
  *best = nys_tile_choice{0, 0, 0.0};
  if (p.cands.empty()) return NYS_OK;   // the row-sum tile: nothing to choose
  const int key = tile_key(prec);
  const size_t eb = elem_bytes(prec);
  if (eb == 8) NYS_RETURN_IF(launch_fill(reinterpret_cast<double *>(p.V), 1.0 / n, n * (int64_t)m, s));
  else NYS_RETURN_IF(launch_fill_f(reinterpret_cast<float *>(p.V), 1.0f / (float)n, n * (int64_t)m, s));
  NYS_RETURN_IF(prep_points(p.kv, k, prec, X, X, d, s));
  hipEvent_t e0, e1;
  NYS_CHECK_HIP(hipEventCreate(&e0));
  NYS_CHECK_HIP(hipEventCreate(&e1));
  double best_ms = 1e300;
  int best_tm = 0;
  int32_t rc = NYS_OK;
  const auto saved = kmv_tune_snapshot();
  if (key == NYS_FP64 && m >= 256) {
    // float64: time one chunk of every width and replace the planner's cost table,
    // which then sizes every float64 product (mixed widths and tails) by least cost
    static const int tms[7] = {16, 32, 48, 64, 96, 128, 256};
    double cost[7];
    for (int t = 0; t < 7 && rc == NYS_OK; ++t) {
      kmv_tune_set(key, tms[t], tms[t], tms[t]);
      rc = run_kmv(p.kv, k, 0, prec, 0, p.V, tms[t], m, p.Out, m, 1.0, 0.0, s);   // untimed first call
      if (rc != NYS_OK) break;
      if (hipEventRecord(e0, s) != hipSuccess) { rc = NYS_EHIP; break; }
      for (int q = 0; q < reps && rc == NYS_OK; ++q)
        rc = run_kmv(p.kv, k, 0, prec, 0, p.V, tms[t], m, p.Out, m, 1.0, 0.0, s);
      if (rc != NYS_OK) break;
      float ms = 0.f;
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        rc = NYS_EHIP;
        break;
      }
      cost[t] = ms / reps;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    kmv_tune_restore(saved);
    if (rc != NYS_OK) {
      if (rc == NYS_EHIP) set_error("nys_autotune: HIP event failure while timing");
      return rc;
    }
    kmv_f64_cost_set(cost);
    const KmvPlan kp = kmv_plan(n_rows, n, m, prec, p.kv.rows.Kp);
    double est = 0.0;
    for (int t = 0; t < 7; ++t)
      if (tms[t] == kp.tm) est = cost[t] * (double)ceil_div(m, kp.tm);
    *best = nys_tile_choice{kp.tm, 0, est};
    return NYS_OK;
  }
  for (int tm : p.cands) {
    kmv_tune_set(key, m, m, tm);
    rc = run_kmv(p.kv, k, 0, prec, 0, p.V, m, m, p.Out, m, 1.0, 0.0, s);   // untimed first call
    if (rc != NYS_OK) break;
    if (hipEventRecord(e0, s) != hipSuccess) { rc = NYS_EHIP; break; }
    for (int t = 0; t < reps && rc == NYS_OK; ++t) rc = run_kmv(p.kv, k, 0, prec, 0, p.V, m, m, p.Out, m, 1.0, 0.0, s);
    if (rc != NYS_OK) break;
    float ms = 0.f;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      rc = NYS_EHIP;
      break;
    }
    if (ms / reps < best_ms) {
      best_ms = ms / reps;
      best_tm = tm;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  kmv_tune_restore(saved);
  if (rc == NYS_OK) kmv_tune_set(key, m_lo, m, best_tm);
  if (rc != NYS_OK) {
    if (rc == NYS_EHIP) set_error("nys_autotune: HIP event failure while timing");
    return rc;
  }
  *best = nys_tile_choice{best_tm, 0, best_ms};
  return NYS_OK;
}

int32_t kernel_matvec(nys_kernel k, int32_t deriv, int32_t prec, const double *Xr, int64_t nr,
                      const double *Xc, int64_t nc, int32_t d, const void *V, int32_t m, void *Out,
                      double alpha, double beta, void *ws, size_t ws_bytes, void *stream) {
  NYS_RETURN_IF(check_kernel(k));
  if (!valid_prec(prec)) return einval("unsupported precision");
  if (deriv != 0 && deriv != 1) return einval("deriv must be 0 or 1");
  if (nr < 0 || nc < 0 || m < 0) return einval("negative size");
  if (d < 1 || d > max_dim(prec)) return einval("d out of range for this precision");
  if (nr == 0 || m == 0) return NYS_OK;
  if (nc == 0) return einval("nc must be >= 1");
  if (!Xr || !Xc || !V || !Out) return einval("null pointer");
  if (!std::isfinite(alpha) || !std::isfinite(beta)) return einval("alpha/beta must be finite");
  if (!ws) return einval("ws is NULL");
  hipStream_t s = as_stream(stream);
  Arena a;
  a.base = reinterpret_cast<char *>(ws);
  a.cap = ws_bytes;
  MatvecPlan p;
  plan_matvec(p, nr, nc, d, m, prec, a);
  NYS_RETURN_IF(check_ws(a));
  const int same = (Xr == Xc && nr == nc) ? 1 : 0;
  NYS_RETURN_IF(prep_points(p.kv, k, prec, Xr, Xc, d, s));
  return run_kmv(p.kv, k, deriv, prec, same, V, m, m, Out, m, alpha, beta, s);
}

int32_t nys_test_matrix(uint64_t seed, int64_t n, int32_t r, double *Omega, void *stream) {
  if (n < 1 || r < 1) return einval("need n >= 1 and r >= 1");
  if (!Omega) return einval("null pointer");
  return launch_gaussian(seed, n * (int64_t)r, Omega, as_stream(stream));
}

int32_t nys_sketch(nys_kernel k, int32_t prec, const double *X, int64_t n, int32_t d, const double *Omega,
                   uint64_t seed, int32_t r, double *Q, double *Y, void *ws, size_t ws_bytes, void *stream) {
  NYS_RETURN_IF(check_kernel(k));
  if (!valid_prec(prec)) return einval("unsupported precision");
  if (n < 1 || d < 1 || d > max_dim(prec)) return einval("n >= 1 and 1 <= d <= max required");
  if (r < 1 || r > n || r > 1024) return einval("need 1 <= r <= min(n, 1024)");
  if (!X || !Q || !Y || !ws) return einval("null pointer");
  const int64_t cnt = n * (int64_t)r;
  if (Omega && Omega + cnt > Q && Q + cnt > Omega) return einval("Q must not overlap Omega");
  hipStream_t s = as_stream(stream);
  Arena a;
  a.base = reinterpret_cast<char *>(ws);
  a.cap = ws_bytes;
  SketchPlan p;
  plan_sketch(p, n, d, r, prec, a);
  NYS_RETURN_IF(check_ws(a));
  // the test matrix: the caller's, or drawn from the seed into Qtmp
  const double *Om = Omega;
  if (!Om) {
    NYS_RETURN_IF(launch_gaussian(seed, cnt, p.Qtmp, s));
    Om = p.Qtmp;
  }
  // Q = Omega L^{-T} with L L^T = Omega^T Omega (Cholesky QR)
  const int splits = gemm_tn_splits(n, r, r);
  NYS_RETURN_IF(gemm_tn<double>(Om, r, Om, r, n, r, r, p.G, r, p.Gpart, splits, s));
  NYS_RETURN_IF(launch_chol(p.G, r, p.flag, s));
  int flag = 0;
  NYS_CHECK_HIP(hipMemcpyAsync(&flag, p.flag, sizeof(int), hipMemcpyDeviceToHost, s));
  NYS_CHECK_HIP(hipStreamSynchronize(s));
  if (flag) {
    set_error("nys_sketch: the test matrix Omega is rank deficient or not finite");
    return NYS_ENOTPD;
  }
  NYS_RETURN_IF(launch_trinv_lower(p.G, p.Linv, r, s));
  NYS_RETURN_IF(launch_transpose(p.Linv, p.LinvT, r, s));
  NYS_RETURN_IF(gemm_nn<double>(Om, r, p.LinvT, r, n, r, r, Q, r, 0, nullptr, 0, nullptr, s));
  // Y = K Q
  NYS_RETURN_IF(prep_points(p.kv, k, prec, X, X, d, s));
  if (prec == NYS_FP64) {
    NYS_RETURN_IF(run_kmv(p.kv, k, 0, prec, 1, Q, r, r, Y, r, 1.0, 0.0, s));
  } else {
    NYS_RETURN_IF(launch_copy_d2f(Q, p.Q32, cnt, s));
    NYS_RETURN_IF(run_kmv(p.kv, k, 0, prec, 1, p.Q32, r, r, p.Y32, r, 1.0, 0.0, s));
    NYS_RETURN_IF(launch_copy_f2d(p.Y32, Y, cnt, s));
  }
  return NYS_OK;
}

int32_t kernel_dot(nys_kernel k, int32_t deriv, const double *Xr, int64_t nr, const double *Xc, int64_t nc,
                   int32_t d, const double *u, const double *v, double *out, void *ws, size_t ws_bytes,
                   void *stream) {
  NYS_RETURN_IF(check_kernel(k));
  if (deriv != 0 && deriv != 1) return einval("deriv must be 0 or 1");
  if (nr < 1 || nc < 1) return einval("need nr >= 1 and nc >= 1");
  if (d < 1 || d > max_dim(NYS_FP64)) return einval("d out of range");
  if (!Xr || !Xc || !u || !v || !out || !ws) return einval("null pointer");
  hipStream_t s = as_stream(stream);
  Arena a;
  a.base = reinterpret_cast<char *>(ws);
  a.cap = ws_bytes;
  DotPlan p;
  plan_dot(p, nr, nc, d, a);
  NYS_RETURN_IF(check_ws(a));
  const int same = (Xr == Xc && nr == nc) ? 1 : 0;
  NYS_RETURN_IF(prep_points(p.kv, k, NYS_FP64, Xr, Xc, d, s));
  NYS_RETURN_IF(run_kmv(p.kv, k, deriv, NYS_FP64, same, v, 1, 1, p.tmp, 1, 1.0, 0.0, s));
  NYS_RETURN_IF(colred<double>(0, u, p.tmp, nullptr, nullptr, nr, 1, nullptr, p.red, s));
  NYS_RETURN_IF(colfinal(p.red, nr, 1, 0, p.out, nullptr, nullptr, nullptr, nullptr, s));
  NYS_CHECK_HIP(hipMemcpyAsync(out, p.out, sizeof(double), hipMemcpyDeviceToHost, s));
  NYS_CHECK_HIP(hipStreamSynchronize(s));
  return NYS_OK;
}

int32_t nys_precond_build(const double *Y, const double *Q, int64_t n, int32_t r, int32_t sketch_prec,
                          nys_precond *P, void *ws, size_t ws_bytes, void *stream) {
  if (!Y || !Q || !P || !ws) return einval("null pointer");
  if (!valid_prec(sketch_prec)) return einval("unsupported precision");
  if (n < 1 || r < 1 || r > n || r > 1024) return einval("need 1 <= r <= min(n, 1024)");
  if (P->n != n || P->r != r || !P->U || !P->lam_hat) return einval("preconditioner buffers do not match n, r");
  hipStream_t s = as_stream(stream);
  Arena a;
  a.base = reinterpret_cast<char *>(ws);
  a.cap = ws_bytes;
  BuildPlan p;
  plan_build(p, n, r, a);
  NYS_RETURN_IF(check_ws(a));
  P->shift = 0.0;
  return build_impl(Y, Q, n, r, sketch_prec, P, p, s);
}

int32_t nys_precond_adaptive(nys_kernel k, int32_t prec, const double *X, int64_t n, int32_t d,
                             const nys_nystrom_config *cfg, nys_precond *P, double *err_out, void *ws,
                             size_t ws_bytes, void *stream) {
  NYS_RETURN_IF(check_kernel(k));
  if (!valid_prec(prec)) return einval("unsupported precision");
  if (n < 1 || d < 1 || d > max_dim(prec)) return einval("n >= 1 and 1 <= d <= max required");
  if (!X || !cfg || !P || !ws) return einval("null pointer");
  const int rmax = cfg->rank_max > 0 ? cfg->rank_max : cfg->rank_init;
  if (cfg->rank_init < 1 || rmax < cfg->rank_init || rmax > n || rmax > 1024)
    return einval("need 1 <= rank_init <= rank_max <= min(n, 1024)");
  if (cfg->num_power_iters < 0) return einval("num_power_iters must be >= 0");
  if (!(cfg->error_tolerance >= 0.0) || !std::isfinite(cfg->error_tolerance))
    return einval("error_tolerance must be finite and >= 0");
  if (cfg->damping_mode != NYS_DAMPING_NON_ADAPTIVE && cfg->damping_mode != NYS_DAMPING_ADAPTIVE)
    return einval("unknown damping mode");
  if (P->n != n || P->r != rmax || !P->U || !P->lam_hat)
    return einval("preconditioner buffers must be sized n x rank_max");
  hipStream_t s = as_stream(stream);
  Arena a;
  a.base = reinterpret_cast<char *>(ws);
  a.cap = ws_bytes;
  AdaptPlan p;
  plan_adapt(p, n, d, rmax, prec, a);
  NYS_RETURN_IF(check_ws(a));
  return adaptive_impl(k, prec, X, n, d, *cfg, rmax, P, err_out, p, s);
}

int32_t nys_precond_apply(const nys_precond *P, const double *lambdas, int32_t prec, const void *R,
                          int32_t m, void *Z, void *ws, size_t ws_bytes, void *stream) {
  if (!P || !lambdas || !R || !Z || !ws) return einval("null pointer");
  if (!valid_prec(prec)) return einval("unsupported precision");
  if (m < 1) return einval("m must be >= 1");
  NYS_RETURN_IF(check_precond(P, P->n, prec));
  if (R == Z) return einval("R and Z must not overlap");
  hipStream_t s = as_stream(stream);
  Arena a;
  a.base = reinterpret_cast<char *>(ws);
  a.cap = ws_bytes;
  if (a.cap < precond_apply_scratch_bytes(P->n, P->r, m, prec)) {
    set_error("workspace smaller than nys_workspace_bytes() for these arguments");
    return NYS_ENOMEM;
  }
  if (prec == NYS_FP64)
    return precond_apply_impl<double>(*P, lambdas, reinterpret_cast<const double *>(R), m,
                                      reinterpret_cast<double *>(Z), a, s);
  return precond_apply_impl<float>(*P, lambdas, reinterpret_cast<const float *>(R), m,
                                   reinterpret_cast<float *>(Z), a, s);
}

int32_t nyspcg_solve(nys_kernel k, const double *X, int64_t n, int32_t d, const double *B, int32_t nrhs,
                     const double *lambdas, int32_t nlam, const nys_precond *P, const nys_pcg_opts *opts,
                     double *Xsol, nys_col_info *info, void *ws, size_t ws_bytes, void *stream) {
  NYS_RETURN_IF(check_kernel(k));
  NYS_RETURN_IF(check_opts(opts));
  const int prec = opts->prec;
  if (n < 1 || d < 1 || d > max_dim(prec)) return einval("n >= 1 and 1 <= d <= max required");
  if (nrhs < 1 || nlam < 1) return einval("nrhs and nlam must be >= 1");
  if ((int64_t)nrhs * nlam > 4096) return einval("at most 4096 columns per solve");
  if (!X || !B || !lambdas || !Xsol || !info || !ws) return einval("null pointer");
  for (int l = 0; l < nlam; ++l)
    if (!(lambdas[l] > 0.0) || !std::isfinite(lambdas[l])) return einval("every lambda must be > 0 and finite");
  NYS_RETURN_IF(check_precond(P, n, prec));
  hipStream_t s = as_stream(stream);
  const int m = nrhs * nlam;
  Arena a;
  a.base = reinterpret_cast<char *>(ws);
  a.cap = ws_bytes;
  SolvePlan sp;
  plan_solve(sp, n, d, P ? P->r : 0, m, prec, opts->refine_every >= 0, opts->check_true != 0, a);
  if (opts->block) {
    if (nrhs > block_max_s()) return einval("block PCG takes at most 64 right-hand sides per lambda");
    if (prec != NYS_FP64 && opts->refine_every != 0)
      return einval("block PCG with a low-precision product refines in cycles (refine_every 0)");
    BlockPlan bp;
    plan_block(bp, n, m, a);
    NYS_RETURN_IF(check_ws(a));
    KernelOp op{k, X, d, sp};
    if (prec == NYS_FP64)
      return solve_blocks<double>(op, n, B, nrhs, lambdas, nlam, P, *opts, Xsol, info, sp, bp, s);
    return solve_blocks<float>(op, n, B, nrhs, lambdas, nlam, P, *opts, Xsol, info, sp, bp, s);
  }
  NYS_RETURN_IF(check_ws(a));
  KernelOp op{k, X, d, sp};
  if (prec == NYS_FP64)
    return solve_columns<double>(op, n, B, nrhs, lambdas, nlam, P, *opts, Xsol, info, sp, s);
  return solve_columns<float>(op, n, B, nrhs, lambdas, nlam, P, *opts, Xsol, info, sp, s);
}

int32_t nys_ridge_sketch(const double *X, int64_t n, int64_t p, const double *Omega, uint64_t seed, int32_t r,
                         double *Q, double *Y, void *ws, size_t ws_bytes, void *stream) {
  if (n < 1 || p < 1 || n > INT32_MAX || p > INT32_MAX) return einval("need 1 <= n, p < 2^31");
  if (r < 1 || r > p || r > 1024) return einval("need 1 <= r <= min(p, 1024)");
  if (!X || !Q || !Y || !ws) return einval("null pointer");
  const int64_t cnt = p * (int64_t)r;
  if (Omega && Omega + cnt > Q && Q + cnt > Omega) return einval("Q must not overlap Omega");
  hipStream_t s = as_stream(stream);
  Arena a;
  a.base = reinterpret_cast<char *>(ws);
  a.cap = ws_bytes;
  RidgeSketchPlan pl;
  plan_ridge_sketch(pl, n, p, r, a);
  NYS_RETURN_IF(check_ws(a));
  NYS_RETURN_IF(orth_test_matrix(Omega, seed, p, r, pl, Q, s));
  RidgeOp op{X, n, p, pl.T, pl.part, pl.part_cap};
  NYS_RETURN_IF(op.apply64(Q, r, r, Y, r, s));
  NYS_CHECK_HIP(hipStreamSynchronize(s));
  return NYS_OK;
}

int32_t nys_ridge_solve(const double *X, int64_t n, int64_t p, const double *Yt, int32_t nrhs,
                        const double *lambdas, int32_t nlam, const nys_precond *P, const nys_pcg_opts *opts,
                        double *W, nys_col_info *info, void *ws, size_t ws_bytes, void *stream) {
  NYS_RETURN_IF(check_opts(opts));
  if (opts->block) return einval("block PCG is offered by nyspcg_solve only");
  if (opts->prec != NYS_FP64) return einval("the ridge solve runs in float64 (prec NYS_FP64)");
  if (n < 1 || p < 1 || n > INT32_MAX || p > INT32_MAX) return einval("need 1 <= n, p < 2^31");
  if (nrhs < 1 || nlam < 1) return einval("nrhs and nlam must be >= 1");
  if ((int64_t)nrhs * nlam > 4096) return einval("at most 4096 columns per solve");
  if (!X || !Yt || !lambdas || !W || !info || !ws) return einval("null pointer");
  for (int l = 0; l < nlam; ++l)
    if (!(lambdas[l] > 0.0) || !std::isfinite(lambdas[l])) return einval("every lambda must be > 0 and finite");
  NYS_RETURN_IF(check_precond(P, p, NYS_FP64));
  hipStream_t s = as_stream(stream);
  const int m = nrhs * nlam;
  Arena a;
  a.base = reinterpret_cast<char *>(ws);
  a.cap = ws_bytes;
  RidgeSolvePlan pl;
  plan_ridge_solve(pl, n, p, P ? P->r : 0, nrhs, m, a);
  NYS_RETURN_IF(check_ws(a));
  RidgeOp op{X, n, p, pl.T, pl.part, pl.part_cap};
  NYS_RETURN_IF(op.prepare(s));
  // right-hand sides X^T y (p x nrhs)
  const double one = 1.0, zero = 0.0;
  if (rocblas_dgemm_64(op.h, rocblas_operation_none, rocblas_operation_transpose, nrhs, (int64_t)p, (int64_t)n,
                    &one, Yt, nrhs, X, (int64_t)p, &zero, pl.B, nrhs) != rocblas_status_success) {
    set_error("rocblas_dgemm failed forming X^T y");
    return NYS_EHIP;
  }
  return solve_columns<double>(op, p, pl.B, nrhs, lambdas, nlam, P, *opts, W, info, pl.sp, s);
}

int32_t nys_admm_elastic_net(const double *X, int64_t n, int64_t p, const double *y, double lam1, double lam2,
                             double lo, double hi, const nys_admm_config *cfg, double *W, nys_admm_info *info,
                             void *ws, size_t ws_bytes, void *stream) {
  if (n < 1 || p < 1 || n > INT32_MAX || p > INT32_MAX) return einval("need 1 <= n, p < 2^31");
  if (!X || !y || !cfg || !W || !info || !ws) return einval("null pointer");
  if (!(lam1 >= 0.0) || !(lam2 >= 0.0) || !std::isfinite(lam1) || !std::isfinite(lam2))
    return einval("lam1 and lam2 must be finite and >= 0");
  if (!(lo <= hi) || std::isnan(lo) || std::isnan(hi)) return einval("need lo <= hi");
  nys_admm_config c;
  NYS_RETURN_IF(admm_config(cfg, p, c));
  hipStream_t s = as_stream(stream);
  Arena a;
  a.base = reinterpret_cast<char *>(ws);
  a.cap = ws_bytes;
  AdmmPlan pl;
  plan_admm(pl, n, p, c.rank, a);
  NYS_RETURN_IF(check_ws(a));
  return admm_impl(X, n, p, y, lam1, lam2, lo, hi, c, W, info, pl, s);
}

int32_t nyspcg_backward(nys_kernel k, const double *X, int64_t n, int32_t d, double lambda,
                        const double *xsol, const double *gx, const nys_precond *P, const nys_pcg_opts *opts,
                        double *adj, double *dL_dlambda, double *dL_dsigma, nys_col_info *info, void *ws,
                        size_t ws_bytes, void *stream) {
  NYS_RETURN_IF(check_kernel(k));
  NYS_RETURN_IF(check_opts(opts));
  if (opts->block) return einval("block PCG is offered by nyspcg_solve only");
  const int prec = opts->prec;
  if (n < 1 || d < 1 || d > max_dim(NYS_FP64)) return einval("n >= 1 and 1 <= d <= 62 required");
  if (!(lambda > 0.0) || !std::isfinite(lambda)) return einval("lambda must be > 0");
  if (!X || !xsol || !gx || !adj || !dL_dlambda || !dL_dsigma || !info || !ws) return einval("null pointer");
  NYS_RETURN_IF(check_precond(P, n, prec));
  hipStream_t s = as_stream(stream);
  Arena a;
  a.base = reinterpret_cast<char *>(ws);
  a.cap = ws_bytes;
  SolvePlan sp;
  plan_solve(sp, n, d, P ? P->r : 0, 1, prec, opts->refine_every >= 0, opts->check_true != 0, a);
  DerivPlan dp;
  plan_deriv(dp, n, d, a);
  NYS_RETURN_IF(check_ws(a));
  // adjoint solve (K + lambda I) a = gx with the same preconditioner
  int32_t rc;
  KernelOp op{k, X, d, sp};
  if (prec == NYS_FP64)
    rc = solve_columns<double>(op, n, gx, 1, &lambda, 1, P, *opts, adj, info, sp, s);
  else
    rc = solve_columns<float>(op, n, gx, 1, &lambda, 1, P, *opts, adj, info, sp, s);
  if (rc < 0) return rc;
  // dL/dlambda = -a^T x ;  dL/dsigma = -a^T (dK/dsigma) x
  NYS_RETURN_IF(prep_points(dp.kv, k, NYS_FP64, X, X, d, s));
  NYS_RETURN_IF(run_kmv(dp.kv, k, 1, NYS_FP64, 1, xsol, 1, 1, dp.tmp, 1, 1.0, 0.0, s));
  NYS_RETURN_IF(colred<double>(0, adj, const_cast<double *>(xsol), nullptr, nullptr, n, 1, nullptr, dp.red, s));
  NYS_RETURN_IF(colfinal(dp.red, n, 1, 0, dp.out, nullptr, nullptr, nullptr, nullptr, s));
  NYS_RETURN_IF(colred<double>(0, adj, dp.tmp, nullptr, nullptr, n, 1, nullptr, dp.red, s));
  NYS_RETURN_IF(colfinal(dp.red, n, 1, 0, dp.out + 1, nullptr, nullptr, nullptr, nullptr, s));
  double h[2] = {0, 0};
  NYS_CHECK_HIP(hipMemcpyAsync(h, dp.out, sizeof(h), hipMemcpyDeviceToHost, s));
  NYS_CHECK_HIP(hipStreamSynchronize(s));
  *dL_dlambda = -h[0];
  *dL_dsigma = -h[1];
  return rc;
}

}  // extern "C"
