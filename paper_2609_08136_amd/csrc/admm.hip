// Vector kernels of NysADMM on the bounded elastic net (section "Splitting for
// ADMM"; the problem of eq. experiment-bounded-en).  Every reduction is two-pass
// and ordered (per-block partials, then one block sums them in block order), so a
// run is bitwise repeatable.
#include "admm.h"

#include <algorithm>

namespace nys {

namespace {

constexpr int kThreads = 256;
constexpr int kMaxBlocks = 1024;

int admm_grid(int64_t p) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(kMaxBlocks, ceil_div(p, 4 * kThreads)));
}

// Block sum of NQ per-thread values into partial[q * gridDim.x + blockIdx.x].
template <int NQ>
__device__ void block_store(const double (&v)[NQ], double *partial) {
  __shared__ double red[NQ][kThreads];
  for (int q = 0; q < NQ; ++q) red[q][threadIdx.x] = v[q];
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int q = 0; q < NQ; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int q = 0; q < NQ; ++q) partial[(int64_t)q * gridDim.x + blockIdx.x] = red[q][0];
}

// rhs = c + rho (z - u) + sigma x;  r0 = rhs - Hx - (rho + sigma) x
// partials: |rhs|^2, |r0|^2
__global__ __launch_bounds__(kThreads) void rhs_kernel(const double *c, const double *z, const double *u,
                                                        const double *x, const double *Hx, double rho,
                                                        double sigma, int64_t p, double *rhs, double *r0,
                                                        double *partial) {
  double acc[2] = {0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < p; i += (int64_t)gridDim.x * kThreads) {
    const double xi = x[i];
    const double b = c[i] + rho * (z[i] - u[i]) + sigma * xi;
    const double r = b - Hx[i] - (rho + sigma) * xi;
    rhs[i] = b;
    r0[i] = r;
    acc[0] += b * b;
    acc[1] += r * r;
  }
  block_store<2>(acc, partial);
}

// x += dx (dx may be null); xh = alpha x + (1 - alpha) z; v = xh + u;
// z = clip(soft(v, lam1/rho) rho/(rho + lam2), lo, hi); u += xh - z
// partials: |x - z|^2, |x|^2, |z|^2
__global__ __launch_bounds__(kThreads) void update_kernel(double *x, const double *dx, double alpha, double *z,
                                                           double *u, double rho, double lam1, double lam2,
                                                           double lo, double hi, int64_t p, double *partial) {
  double acc[3] = {0.0, 0.0, 0.0};
  const double thr = lam1 / rho, shrink = rho / (rho + lam2);
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < p; i += (int64_t)gridDim.x * kThreads) {
    double xi = x[i];
    if (dx) {
      xi += dx[i];
      x[i] = xi;
    }
    const double zo = z[i];
    const double xh = alpha * xi + (1.0 - alpha) * zo;
    const double v = xh + u[i];
    const double a = fabs(v) - thr;
    double zn = a > 0.0 ? copysign(a, v) * shrink : 0.0;
    zn = fmin(fmax(zn, lo), hi);
    z[i] = zn;
    u[i] = u[i] + xh - zn;
    const double e = xi - zn;
    acc[0] += e * e;
    acc[1] += xi * xi;
    acc[2] += zn * zn;
  }
  block_store<3>(acc, partial);
}

// r_dual = Hx - c + rho u; partials: |r_dual|^2, |rho u|^2
__global__ __launch_bounds__(kThreads) void dual_kernel(const double *Hx, const double *c, const double *u,
                                                         double rho, int64_t p, double *partial) {
  double acc[2] = {0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < p; i += (int64_t)gridDim.x * kThreads) {
    const double ru = rho * u[i];
    const double rd = Hx[i] - c[i] + ru;
    acc[0] += rd * rd;
    acc[1] += ru * ru;
  }
  block_store<2>(acc, partial);
}

// out[q] = sum over blocks of partial[q * nb + b], in block order
__global__ void final_kernel(const double *partial, int nb, int nq, double *out) {
  __shared__ double red[kThreads];
  for (int q = 0; q < nq; ++q) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += kThreads) s += partial[(int64_t)q * nb + b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[q] = red[0];
    __syncthreads();
  }
}

// Xc[i][j] = X[i][j] - mu[j]  (row-major n x p)
__global__ __launch_bounds__(kThreads) void center_kernel(const double *X, const double *mu, int64_t n, int64_t p,
                                                           double *Xc) {
  const int64_t total = n * p;
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < total; e += (int64_t)gridDim.x * kThreads)
    Xc[e] = X[e] - mu[e % p];
}

__global__ __launch_bounds__(kThreads) void scale_kernel(double *v, double a, int64_t p) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < p; i += (int64_t)gridDim.x * kThreads)
    v[i] *= a;
}

}  // namespace

size_t admm_partial_elems(int64_t p) { return (size_t)3 * admm_grid(p) + 2 * admm_grid(p); }

int32_t admm_rhs(const double *c, const double *z, const double *u, const double *x, const double *Hx, double rho,
                 double sigma, int64_t p, double *rhs, double *r0, double *partial, double *out, hipStream_t s) {
  const int nb = admm_grid(p);
  hipLaunchKernelGGL(rhs_kernel, dim3(nb), dim3(kThreads), 0, s, c, z, u, x, Hx, rho, sigma, p, rhs, r0, partial);
  NYS_LAUNCH_CHECK();
  hipLaunchKernelGGL(final_kernel, dim3(1), dim3(kThreads), 0, s, partial, nb, 2, out);
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}

int32_t admm_update(double *x, const double *dx, double alpha, double *z, double *u, double rho, double lam1,
                    double lam2, double lo, double hi, int64_t p, double *partial, hipStream_t s) {
  const int nb = admm_grid(p);
  hipLaunchKernelGGL(update_kernel, dim3(nb), dim3(kThreads), 0, s, x, dx, alpha, z, u, rho, lam1, lam2, lo, hi, p,
                     partial);
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}

int32_t admm_dual(const double *Hx, const double *c, const double *u, double rho, int64_t p, double *partial,
                  double *out, hipStream_t s) {
  const int nb = admm_grid(p);
  // the update's three partial rows come first, the dual's two follow
  double *dpart = partial + (size_t)3 * nb;
  hipLaunchKernelGGL(dual_kernel, dim3(nb), dim3(kThreads), 0, s, Hx, c, u, rho, p, dpart);
  NYS_LAUNCH_CHECK();
  hipLaunchKernelGGL(final_kernel, dim3(1), dim3(kThreads), 0, s, partial, nb, 5, out);
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}

int32_t admm_center(const double *X, const double *mu, int64_t n, int64_t p, double *Xc, hipStream_t s) {
  const int64_t nb = std::max<int64_t>(1, std::min<int64_t>(ceil_div(n * p, 4 * kThreads), 8192));
  hipLaunchKernelGGL(center_kernel, dim3((unsigned)nb), dim3(kThreads), 0, s, X, mu, n, p, Xc);
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}

int32_t admm_scale(double *v, double a, int64_t p, hipStream_t s) {
  hipLaunchKernelGGL(scale_kernel, dim3(admm_grid(p)), dim3(kThreads), 0, s, v, a, p);
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}

}  // namespace nys
