// Vector kernels of the preconditioned CG recurrence on an n x m block of
// independent columns (row-major, column c has its own lambda_c, alpha_c,
// beta_c), the Nystrom preconditioner apply, and column compaction.
//
// PCG step for every active column (table tab:rlaopt-pcg-stopping for the stop):
//   w = K p + lambda p;  alpha = rho / p^T w;  x += alpha p;  r -= alpha w;
//   z = P^{-1} r;  rho' = r^T z;  beta = rho' / rho;  p = z + beta p.
// Column reductions are two-pass (per-block partials, then a fixed-order sum
// in float64), so every result is reproducible bit for bit.
#include <algorithm>

#include "pcg.h"

namespace nys {

// ------------------------------------------------------------ reduction shape
ColRedShape colred_shape(int64_t n, int m) {
  ColRedShape s;
  s.cw = 1;
  while (s.cw < m && s.cw < 256) s.cw *= 2;
  s.ry = 256 / s.cw;
  // enough blocks to cover the GPU, at least 64 rows per block
  int64_t nb = std::min<int64_t>(ceil_div(n, 64), 2048);
  s.nb = (int)std::max<int64_t>(1, nb);
  s.rows_per = ceil_div(n, s.nb);
  s.nb = (int)ceil_div(n, s.rows_per);
  return s;
}

// op 0: partial = sum a*b;  op 1: W += lam P, partial = sum P*W (a=P, b=W);
// op 2: X += alpha P, R -= alpha W, partial = sum R*R (a=P, b=W, X, R)
// op 3: as op 2 but the iterate is float64 (X64 += alpha P)
template <class T, int OP>
__global__ __launch_bounds__(256) void colred_kernel(const T *a, T *b, T *X, T *R, int64_t n, int m,
                                                     int64_t rows_per, const double *coef,
                                                     double *partial, double *X64) {
  __shared__ double red[256];
  const int cw = blockDim.x, ry = blockDim.y;
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per;
  const int64_t r1 = std::min<int64_t>(n, r0 + rows_per);
  for (int c0 = 0; c0 < m; c0 += cw) {
    const int c = c0 + tx;
    double s = 0.0;
    if (c < m) {
      const double cf = (OP == 0) ? 0.0 : coef[c];
      for (int64_t i = r0 + ty; i < r1; i += ry) {
        const int64_t e = i * m + c;
        if constexpr (OP == 0) {
          s += (double)a[e] * (double)b[e];
        } else if constexpr (OP == 1) {
          const T p = a[e];
          const T w = b[e] + (T)cf * p;
          b[e] = w;
          s += (double)p * (double)w;
        } else {
          const T p = a[e], w = b[e];
          if constexpr (OP == 3) X64[e] += cf * (double)p;
          else X[e] += (T)cf * p;
          const T rr = R[e] - (T)cf * w;
          R[e] = rr;
          s += (double)rr * (double)rr;
        }
      }
    }
    red[ty * cw + tx] = s;
    __syncthreads();
    for (int w = ry / 2; w > 0; w >>= 1) {
      if (ty < w) red[ty * cw + tx] += red[(ty + w) * cw + tx];
      __syncthreads();
    }
    if (ty == 0 && c < m) partial[(int64_t)blockIdx.x * m + c] = red[tx];
    __syncthreads();
  }
}

// Final ordered sum of partials and the scalar update it feeds.
//   mode 0: out[c] = s
//   mode 1 (alpha): pw[c] = s; alpha[c] = rho[c] / s; flag breakdown if s <= 0 or non-finite
//   mode 2 (beta):  beta[c] = s / rho[c]; rho[c] = s   (restart[c] != 0 -> beta = 0)
__global__ void colfinal_kernel(const double *partial, int nb, int m, int mode, double *out,
                                double *rho, double *alpha_beta, const int *restart, int *flag) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= m) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += partial[(int64_t)b * m + c];
  if (out) out[c] = s;
  if (mode == 1) {
    if (!(s > 0.0) || !isfinite(s)) {
      flag[c] = 1;
      alpha_beta[c] = 0.0;
    } else {
      alpha_beta[c] = rho[c] / s;
    }
  } else if (mode == 2) {
    const double b = (restart && restart[c]) ? 0.0 : (rho[c] != 0.0 ? s / rho[c] : 0.0);
    alpha_beta[c] = b;
    rho[c] = s;
  }
}

template <class T>
int32_t colred(int op, const T *a, T *b, T *X, T *R, int64_t n, int m, const double *coef,
               double *partial, hipStream_t s, double *X64) {
  const ColRedShape sh = colred_shape(n, m);
  dim3 block(sh.cw, sh.ry), grid(sh.nb);
  if (op == 0)
    hipLaunchKernelGGL((colred_kernel<T, 0>), grid, block, 0, s, a, b, X, R, n, m, sh.rows_per, coef, partial, X64);
  else if (op == 1)
    hipLaunchKernelGGL((colred_kernel<T, 1>), grid, block, 0, s, a, b, X, R, n, m, sh.rows_per, coef, partial, X64);
  else if (op == 2)
    hipLaunchKernelGGL((colred_kernel<T, 2>), grid, block, 0, s, a, b, X, R, n, m, sh.rows_per, coef, partial, X64);
  else
    hipLaunchKernelGGL((colred_kernel<T, 3>), grid, block, 0, s, a, b, X, R, n, m, sh.rows_per, coef, partial, X64);
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}

int32_t colfinal(const double *partial, int64_t n, int m, int mode, double *out, double *rho,
                 double *ab, const int *restart, int *flag, hipStream_t s) {
  const ColRedShape sh = colred_shape(n, m);
  hipLaunchKernelGGL(colfinal_kernel, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, s, partial, sh.nb, m,
                     mode, out, rho, ab, restart, flag);
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}

// partial = sum (R64[:, t] - R[:, idx[t]])^2 over the ns refined columns: how far the
// recursive residual R (ma columns) had drifted from the float64 one (idx null: t)
template <class T>
__global__ __launch_bounds__(256) void gap_kernel(const double *R64, int ns, const T *R, int ma, const int *idx,
                                                  int64_t n, int64_t rows_per, double *partial) {
  __shared__ double red[256];
  const int cw = blockDim.x, ry = blockDim.y;
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per;
  const int64_t r1 = std::min<int64_t>(n, r0 + rows_per);
  for (int c0 = 0; c0 < ns; c0 += cw) {
    const int c = c0 + tx;
    double s = 0.0;
    if (c < ns) {
      const int cr = idx ? idx[c] : c;
      for (int64_t i = r0 + ty; i < r1; i += ry) {
        const double d = R64[i * ns + c] - (double)R[i * ma + cr];
        s += d * d;
      }
    }
    red[ty * cw + tx] = s;
    __syncthreads();
    for (int w = ry / 2; w > 0; w >>= 1) {
      if (ty < w) red[ty * cw + tx] += red[(ty + w) * cw + tx];
      __syncthreads();
    }
    if (ty == 0 && c < ns) partial[(int64_t)blockIdx.x * ns + c] = red[tx];
    __syncthreads();
  }
}

template <class T>
int32_t gapnorm(const double *R64, int ns, const T *R, int ma, const int *idx, int64_t n, double *partial,
                hipStream_t s) {
  const ColRedShape sh = colred_shape(n, ns);
  hipLaunchKernelGGL((gap_kernel<T>), dim3(sh.nb), dim3(sh.cw, sh.ry), 0, s, R64, ns, R, ma, idx, n, sh.rows_per,
                     partial);
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}
template int32_t gapnorm<float>(const double *, int, const float *, int, const int *, int64_t, double *,
                                hipStream_t);
template int32_t gapnorm<double>(const double *, int, const double *, int, const int *, int64_t, double *,
                                 hipStream_t);

template int32_t colred<float>(int, const float *, float *, float *, float *, int64_t, int, const double *,
                               double *, hipStream_t, double *);
template int32_t colred<double>(int, const double *, double *, double *, double *, int64_t, int,
                                const double *, double *, hipStream_t, double *);

// ------------------------------------------------------------ elementwise
// P = Z + beta P
template <class T>
__global__ void p_update_kernel(T *P, const T *Z, const double *beta, int64_t n, int m) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * m) return;
  const int c = (int)(idx % m);
  P[idx] = Z[idx] + (T)beta[c] * P[idx];
}
template <class T>
int32_t p_update(T *P, const T *Z, const double *beta, int64_t n, int m, hipStream_t s) {
  const int64_t tot = n * m;
  hipLaunchKernelGGL(p_update_kernel<T>, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, s, P, Z, beta, n, m);
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}
template int32_t p_update<float>(float *, const float *, const double *, int64_t, int, hipStream_t);
template int32_t p_update<double>(double *, const double *, const double *, int64_t, int, hipStream_t);

// R = B[:, bcol[c]] (converted to T), X = 0
template <class T>
__global__ void init_rhs_kernel(const double *B, int nrhs, const int *bcol, T *R, T *X, int64_t n, int m) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * m) return;
  const int64_t i = idx / m;
  const int c = (int)(idx - i * m);
  R[idx] = (T)B[i * nrhs + bcol[c]];
  X[idx] = (T)0;
}
template <class T>
int32_t init_rhs(const double *B, int nrhs, const int *bcol, T *R, T *X, int64_t n, int m, hipStream_t s) {
  const int64_t tot = n * m;
  hipLaunchKernelGGL(init_rhs_kernel<T>, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, s, B, nrhs, bcol, R, X, n, m);
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}
template int32_t init_rhs<float>(const double *, int, const int *, float *, float *, int64_t, int, hipStream_t);
template int32_t init_rhs<double>(const double *, int, const int *, double *, double *, int64_t, int, hipStream_t);

// X64 += X (then X = 0): the float64 accumulation of the low-precision iterate
__global__ void flush_x_kernel(float *X, double *X64, int64_t count) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= count) return;
  X64[idx] += (double)X[idx];
  X[idx] = 0.0f;
}
int32_t flush_x(float *X, double *X64, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(flush_x_kernel, dim3((unsigned)ceil_div(count, 256)), dim3(256), 0, s, X, X64, count);
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}

// R64 = B[:, bcol] - KX - lambda X (KX holds K X on entry, overwritten by R64);
// optional float copy into R32.
__global__ void residual64_kernel(const double *B, int nrhs, const int *bcol, const double *lam,
                                  const double *X64, double *KX, float *R32, int64_t n, int m) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * m) return;
  const int64_t i = idx / m;
  const int c = (int)(idx - i * m);
  const double r = B[i * nrhs + bcol[c]] - KX[idx] - lam[c] * X64[idx];
  KX[idx] = r;
  if (R32) R32[idx] = (float)r;
}
int32_t residual64(const double *B, int nrhs, const int *bcol, const double *lam, const double *X64,
                   double *KX, float *R32, int64_t n, int m, hipStream_t s) {
  const int64_t tot = n * m;
  hipLaunchKernelGGL(residual64_kernel, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, s, B, nrhs, bcol, lam,
                     X64, KX, R32, n, m);
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}

// Xsol[:, orig[c]] = (double) X[:, c] (+ X64[:, c]) for the listed slots
template <class T>
__global__ void scatter_sol_kernel(const T *X, const double *X64, int m, const int *slots,
                                   const int *orig, int count, double *Xsol, int mtot, int64_t n) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * count) return;
  const int64_t i = idx / count;
  const int k = (int)(idx - i * count);
  const int c = slots[k];
  double v = (double)X[i * m + c];
  if (X64) v += X64[i * m + c];
  Xsol[i * mtot + orig[k]] = v;
}
template <class T>
int32_t scatter_sol(const T *X, const double *X64, int m, const int *slots, const int *orig, int count,
                    double *Xsol, int mtot, int64_t n, hipStream_t s) {
  if (count <= 0) return NYS_OK;
  const int64_t tot = n * count;
  hipLaunchKernelGGL(scatter_sol_kernel<T>, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, s, X, X64, m, slots,
                     orig, count, Xsol, mtot, n);
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}
template int32_t scatter_sol<float>(const float *, const double *, int, const int *, const int *, int,
                                    double *, int, int64_t, hipStream_t);
template int32_t scatter_sol<double>(const double *, const double *, int, const int *, const int *, int,
                                     double *, int, int64_t, hipStream_t);

// dst[:, k] = src[:, keep[k]]  (n x m_old -> n x m_new)
template <class T>
__global__ void gather_cols_kernel(const T *src, int m_old, const int *keep, int m_new, T *dst, int64_t n) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * m_new) return;
  const int64_t i = idx / m_new;
  const int k = (int)(idx - i * m_new);
  dst[idx] = src[i * m_old + keep[k]];
}
template <class T>
int32_t gather_cols(const T *src, int m_old, const int *keep, int m_new, T *dst, int64_t n, hipStream_t s) {
  if (m_new <= 0) return NYS_OK;
  const int64_t tot = n * m_new;
  hipLaunchKernelGGL(gather_cols_kernel<T>, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, s, src, m_old, keep,
                     m_new, dst, n);
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}
template int32_t gather_cols<float>(const float *, int, const int *, int, float *, int64_t, hipStream_t);
template int32_t gather_cols<double>(const double *, int, const int *, int, double *, int64_t, hipStream_t);

__global__ void scatter_cols_d2f_kernel(const double *src, int ns, const int *idx, float *dst, int m, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * ns) return;
  const int64_t i = e / ns;
  const int k = (int)(e - i * ns);
  dst[i * m + idx[k]] = (float)src[e];
}
int32_t scatter_cols_d2f(const double *src, int ns, const int *idx, float *dst, int m, int64_t n, hipStream_t s) {
  if (ns <= 0) return NYS_OK;
  const int64_t tot = n * ns;
  hipLaunchKernelGGL(scatter_cols_d2f_kernel, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, s, src, ns, idx, dst,
                     m, n);
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}

// ------------------------------------------------------------ preconditioner apply
// Z = U (gamma .* (U^T R)) + R / lambda_c with gamma_ic = -lh_i / (lambda_c (lh_i + lambda_c)),
// the cancellation-free form of (lh_i + lambda_c)^{-1} - lambda_c^{-1}.
template <class T>
// damping rho_c = lam[c] + shift (shift: the adaptive damping of the preconditioner)
__global__ void gamma_scale_kernel(T *W, int r, int m, const double *lam_hat, const double *lam, double shift,
                                   double *inv_lam) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (int64_t)r * m) {
    const int i = (int)(idx / m), c = (int)(idx - (int64_t)i * m);
    const double lh = lam_hat[i], lc = lam[c] + shift;
    const double g = -lh / (lc * (lh + lc));
    W[idx] = (T)((double)W[idx] * g);
  }
  if (idx < m) inv_lam[idx] = 1.0 / (lam[idx] + shift);
}

size_t precond_apply_scratch_bytes(int64_t n, int r, int m, int prec) {
  (void)prec;
  const int splits = gemm_tn_splits(n, r, m);
  Arena a;
  a.take<double>((size_t)r * m);
  a.take<double>((size_t)splits * r * m);
  a.take<double>((size_t)m);
  return a.off;
}

// The arithmetic is float64 for every vector type: with lambda far below the
// largest retained eigenvalue, the two terms of the closed form cancel in
// span(U), and in float32 that cancellation leaves errors of about
// u * lam_hat_1 / lambda relative to the smallest eigenvalue of P^{-1}, enough to
// make the applied operator indefinite.  Float32 vectors are only rounded once,
// on output (a relative perturbation, which keeps P^{-1} positive definite).
template <class T>
int32_t precond_apply_impl(const nys_precond &P, const double *lambdas, const T *R, int m, T *Z,
                           Arena &ws, hipStream_t s) {
  const int64_t n = P.n;
  const int r = P.r;
  const int splits = gemm_tn_splits(n, r, m);
  double *W = ws.take<double>((size_t)r * m);
  double *part = ws.take<double>((size_t)splits * r * m);
  double *inv_lam = ws.take<double>((size_t)m);
  if (ws.overflowed()) {
    set_error("precond apply: workspace too small");
    return NYS_ENOMEM;
  }
  if (ws.measuring()) return NYS_OK;
  const double *U = P.U;
  if constexpr (sizeof(T) == 8) {
    NYS_RETURN_IF(gemm_tn<double>(U, r, reinterpret_cast<const double *>(R), m, n, r, m, W, m, part, splits, s));
  } else {
    NYS_RETURN_IF(gemm_tn_df(U, r, reinterpret_cast<const float *>(R), m, n, r, m, W, m, part, splits, s));
  }
  const int64_t tot = std::max<int64_t>((int64_t)r * m, m);
  hipLaunchKernelGGL(gamma_scale_kernel<double>, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, s, W, r, m,
                     P.lam_hat, lambdas, P.shift, inv_lam);
  NYS_LAUNCH_CHECK();
  if constexpr (sizeof(T) == 8)
    return gemm_nn<double>(U, r, W, m, n, r, m, reinterpret_cast<double *>(Z), m, 1,
                           reinterpret_cast<const double *>(R), m, inv_lam, s);
  else
    return gemm_nn_dd_f(U, r, W, m, n, r, m, reinterpret_cast<float *>(Z), m,
                        reinterpret_cast<const float *>(R), m, inv_lam, s);
}

template int32_t precond_apply_impl<float>(const nys_precond &, const double *, const float *, int, float *,
                                           Arena &, hipStream_t);
template int32_t precond_apply_impl<double>(const nys_precond &, const double *, const double *, int,
                                            double *, Arena &, hipStream_t);

}  // namespace nys
