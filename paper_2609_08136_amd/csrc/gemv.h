// Declarations of the dense row-major matrix-vector products (gemv.hip).
#pragma once

#include "nys_internal.h"

namespace nys {

// scratch (doubles) that launch_coltrans (m = 1) or launch_coltrans_multi (m columns)
// needs for an n x p matrix
size_t gemv_partial_elems(int64_t n, int64_t p, int m);

// t = X v  (X row-major n x p; v length p with stride incv, t length n)
int32_t launch_rowdot(const double *X, int64_t n, int64_t p, const double *v, int64_t incv, double *t,
                      hipStream_t s);

// out[j * inc] = a sum_i t[i] X[i][j]  (out = a X^T t, length p)
int32_t launch_coltrans(const double *X, int64_t n, int64_t p, const double *t, double a, double *out, int64_t inc,
                        double *partial, hipStream_t s);

// Out[j * ldo + k] = a sum_i X[i][j] T[i * ldt + k]  (Out = a X^T T, p x m)
int32_t launch_coltrans_multi(const double *X, int64_t n, int64_t p, const double *T, int m, int64_t ldt, double a,
                              double *Out, int64_t ldo, double *partial, hipStream_t s);

}  // namespace nys
