// Declarations of the PCG vector kernels (pcg.hip).
#pragma once

#include "nys_internal.h"

namespace nys {

struct ColRedShape {
  int cw = 1, ry = 256, nb = 1;
  int64_t rows_per = 1;
};
ColRedShape colred_shape(int64_t n, int m);

// op 0: partial_c = a_c . b_c
// op 1: b += coef_c a (W += lambda P), partial_c = a_c . b_c
// op 2: X += coef_c a, R -= coef_c b, partial_c = R_c . R_c
// op 3: as op 2 with the iterate accumulated in float64 (X64 += coef_c a)
template <class T>
int32_t colred(int op, const T *a, T *b, T *X, T *R, int64_t n, int m, const double *coef,
               double *partial, hipStream_t s, double *X64 = nullptr);
int32_t colfinal(const double *partial, int64_t n, int m, int mode, double *out, double *rho,
                 double *ab, const int *restart, int *flag, hipStream_t s);

template <class T>
int32_t p_update(T *P, const T *Z, const double *beta, int64_t n, int m, hipStream_t s);
template <class T>
int32_t init_rhs(const double *B, int nrhs, const int *bcol, T *R, T *X, int64_t n, int m, hipStream_t s);
int32_t flush_x(float *X, double *X64, int64_t count, hipStream_t s);
// squared 2-norm of R64[:, t] - R[:, idx[t]] for t < ns into partials (colfinal(n, ns) sums them)
template <class T>
int32_t gapnorm(const double *R64, int ns, const T *R, int ma, const int *idx, int64_t n, double *partial,
                hipStream_t s);
int32_t residual64(const double *B, int nrhs, const int *bcol, const double *lam, const double *X64,
                   double *KX, float *R32, int64_t n, int m, hipStream_t s);
template <class T>
int32_t scatter_sol(const T *X, const double *X64, int m, const int *slots, const int *orig, int count,
                    double *Xsol, int mtot, int64_t n, hipStream_t s);
template <class T>
int32_t gather_cols(const T *src, int m_old, const int *keep, int m_new, T *dst, int64_t n, hipStream_t s);

// dst[:, idx[k]] = (float) src[:, k]   (src n x ns double, dst n x m float)
int32_t scatter_cols_d2f(const double *src, int ns, const int *idx, float *dst, int m, int64_t n, hipStream_t s);

size_t precond_apply_scratch_bytes(int64_t n, int r, int m, int prec);

}  // namespace nys
