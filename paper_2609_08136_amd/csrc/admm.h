// Declarations of the NysADMM vector kernels (admm.hip).
#pragma once

#include "nys_internal.h"

namespace nys {

// partial-sum scratch (doubles) of the three reductions below for length p
size_t admm_partial_elems(int64_t p);

// rhs = c + rho (z - u) + sigma x and the warm-start residual r0 = rhs - Hx - (rho + sigma) x;
// out[0] = |rhs|^2, out[1] = |r0|^2 (device)
int32_t admm_rhs(const double *c, const double *z, const double *u, const double *x, const double *Hx, double rho,
                 double sigma, int64_t p, double *rhs, double *r0, double *partial, double *out, hipStream_t s);

// x += dx (dx may be null), over-relaxation, the elastic-net-and-box proximal step and the
// scaled dual update; leaves the partials of |x - z|^2, |x|^2, |z|^2 for admm_dual
int32_t admm_update(double *x, const double *dx, double alpha, double *z, double *u, double rho, double lam1,
                    double lam2, double lo, double hi, int64_t p, double *partial, hipStream_t s);

// r_dual = Hx - c + rho u; out[0..4] = |x - z|^2, |x|^2, |z|^2, |r_dual|^2, |rho u|^2 (device)
int32_t admm_dual(const double *Hx, const double *c, const double *u, double rho, int64_t p, double *partial,
                  double *out, hipStream_t s);

// Xc = X - 1 mu^T (row-major n x p)
int32_t admm_center(const double *X, const double *mu, int64_t n, int64_t p, double *Xc, hipStream_t s);

// v *= a
int32_t admm_scale(double *v, double a, int64_t p, hipStream_t s);

}  // namespace nys
