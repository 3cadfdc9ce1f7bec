// Small dense float64 linear algebra for the r x r core of the Nystrom build
// (r <= 1024): Cholesky with failure flag, triangular inverse, and a cyclic
// parallel Jacobi eigensolver.  All of it runs on the device; the host only
// reads a failure flag and the off-diagonal norm once per Jacobi sweep.
#include <algorithm>
#include <cmath>
#include <vector>

#include "nys_internal.h"

namespace nys {

// ------------------------------------------------------------ Cholesky
// Right-looking, one workgroup.  Lower triangle of A (row-major r x r) is
// overwritten by L with A = L L^T; the strict upper triangle is zeroed.
__global__ __launch_bounds__(1024) void chol_kernel(double *A, int r, int *flag) {
  __shared__ int fail;
  if (threadIdx.x == 0) fail = 0;
  for (int k = 0; k < r; ++k) {
    __syncthreads();
    if (threadIdx.x == 0) {
      double akk = A[(int64_t)k * r + k];
      if (!(akk > 0.0) || !isfinite(akk)) fail = k + 1;
      else A[(int64_t)k * r + k] = sqrt(akk);
    }
    __syncthreads();
    if (fail) break;
    const double lkk = A[(int64_t)k * r + k];
    for (int i = k + 1 + threadIdx.x; i < r; i += blockDim.x) A[(int64_t)i * r + k] /= lkk;
    __syncthreads();
    const int w = r - k - 1;
    for (int64_t idx = threadIdx.x; idx < (int64_t)w * w; idx += blockDim.x) {
      const int i = k + 1 + (int)(idx / w), j = k + 1 + (int)(idx % w);
      if (j <= i) A[(int64_t)i * r + j] -= A[(int64_t)i * r + k] * A[(int64_t)j * r + k];
    }
  }
  __syncthreads();
  for (int64_t idx = threadIdx.x; idx < (int64_t)r * r; idx += blockDim.x) {
    const int i = (int)(idx / r), j = (int)(idx % r);
    if (j > i) A[idx] = 0.0;
  }
  if (threadIdx.x == 0) flag[0] = fail;
}

int32_t launch_chol(double *A, int r, int *flag, hipStream_t s) {
  hipLaunchKernelGGL(chol_kernel, dim3(1), dim3(1024), 0, s, A, r, flag);
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}

// ------------------------------------------------------------ L^{-1}
// Row-by-row forward substitution for all columns at once: row i of L^{-1} is
// (e_i - sum_{k<i} L_ik Linv_k) / L_ii; thread j owns column j.
__global__ __launch_bounds__(1024) void trinv_kernel(const double *L, double *Linv, int r) {
  for (int64_t idx = threadIdx.x; idx < (int64_t)r * r; idx += blockDim.x) Linv[idx] = 0.0;
  __syncthreads();
  for (int i = 0; i < r; ++i) {
    const double lii = L[(int64_t)i * r + i];
    for (int j = threadIdx.x; j <= i; j += blockDim.x) {
      double s = (i == j) ? 1.0 : 0.0;
      for (int k = j; k < i; ++k) s -= L[(int64_t)i * r + k] * Linv[(int64_t)k * r + j];
      Linv[(int64_t)i * r + j] = s / lii;
    }
    __syncthreads();
  }
}

int32_t launch_trinv_lower(const double *L, double *Linv, int r, hipStream_t s) {
  hipLaunchKernelGGL(trinv_kernel, dim3(1), dim3(1024), 0, s, L, Linv, r);
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}

__global__ void symmetrise_kernel(const double *M, double *A, int r) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)r * r) return;
  const int i = (int)(idx / r), j = (int)(idx % r);
  A[idx] = 0.5 * (M[(int64_t)i * r + j] + M[(int64_t)j * r + i]);
}
int32_t launch_symmetrise(const double *M, double *A, int r, hipStream_t s) {
  const int64_t tot = (int64_t)r * r;
  hipLaunchKernelGGL(symmetrise_kernel, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, s, M, A, r);
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}

__global__ void transpose_kernel(const double *A, double *At, int r) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)r * r) return;
  const int i = (int)(idx / r), j = (int)(idx % r);
  At[(int64_t)j * r + i] = A[idx];
}
int32_t launch_transpose(const double *A, double *At, int r, hipStream_t s) {
  const int64_t tot = (int64_t)r * r;
  hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, s, A, At, r);
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}

// ------------------------------------------------------------ Jacobi
// One round of the cyclic parallel Jacobi method: the round-robin schedule pairs
// the (even) index set {0..rr-1} into rr/2 disjoint pairs; each pair (p, q) gets
// the rotation that zeroes A_pq (Golub & Van Loan, symmetric Schur 2x2), and the
// disjoint rotations J are applied at once: A <- J^T A J, V <- V J.
// For index i with partner pi(i): column i of J is c_i e_i + s_i e_pi(i), with
// s_p = -sin, s_q = +sin for the pair (p < q).
__global__ void jacobi_params_kernel(const double *A, int r, int rr, int round, double *cs,
                                     double *sg, int *partner) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rr / 2) return;
  int a, b;
  const int M = rr - 1;
  if (t == 0) {
    a = M;
    b = round;
  } else {
    a = (round + t) % M;
    b = (round - t + M) % M;
  }
  const int p = a < b ? a : b, q = a < b ? b : a;
  if (q >= r) {  // pair with the padding index: identity on the real one
    if (p < r) {
      cs[p] = 1.0;
      sg[p] = 0.0;
      partner[p] = p;
    }
    return;
  }
  const double app = A[(int64_t)p * r + p], aqq = A[(int64_t)q * r + q], apq = A[(int64_t)p * r + q];
  double c = 1.0, sn = 0.0;
  if (apq != 0.0 && fabs(apq) > 1e-300) {
    const double tau = (aqq - app) / (2.0 * apq);
    const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
    c = 1.0 / sqrt(1.0 + tt * tt);
    sn = tt * c;
  }
  cs[p] = c;
  cs[q] = c;
  sg[p] = -sn;
  sg[q] = sn;
  partner[p] = q;
  partner[q] = p;
}

__global__ void jacobi_apply_kernel(const double *A, double *An, const double *V, double *Vn, int r,
                                    const double *cs, const double *sg, const int *partner) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)r * r) return;
  const int i = (int)(idx / r), j = (int)(idx % r);
  const int pi = partner[i], pj = partner[j];
  const double ci = cs[i], si = sg[i], cj = cs[j], sj = sg[j];
  const double aij = A[(int64_t)i * r + j];
  const double aipj = A[(int64_t)i * r + pj];
  const double apij = A[(int64_t)pi * r + j];
  const double apipj = A[(int64_t)pi * r + pj];
  double v = ci * (cj * aij + sj * aipj) + si * (cj * apij + sj * apipj);
  if (i != j && pi == j) v = 0.0;  // the pair's own off-diagonal entry is zero by construction
  An[idx] = v;
  // V <- V J : row i of V, column j
  Vn[idx] = cj * V[(int64_t)i * r + j] + sj * V[(int64_t)i * r + pj];
}

__global__ void offdiag_kernel(const double *A, int r, double *out2) {
  // one workgroup: out2[0] = sum of squares off the diagonal, out2[1] = total
  __shared__ double so[256], st[256];
  double o = 0.0, t = 0.0;
  for (int64_t idx = threadIdx.x; idx < (int64_t)r * r; idx += 256) {
    const double v = A[idx];
    t += v * v;
    if (idx / r != idx % r) o += v * v;
  }
  so[threadIdx.x] = o;
  st[threadIdx.x] = t;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      so[threadIdx.x] += so[threadIdx.x + w];
      st[threadIdx.x] += st[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out2[0] = so[0];
    out2[1] = st[0];
  }
}

__global__ void eye_kernel(double *V, int r) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)r * r) return;
  V[idx] = (idx / r == idx % r) ? 1.0 : 0.0;
}

__global__ void diag_kernel(const double *A, double *w, int r) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < r) w[i] = A[(int64_t)i * r + i];
}

size_t jacobi_scratch_elems(int r) {
  // cs, sg (r each), partner (r ints as doubles), V buffer (r*r), off-norm (2)
  return (size_t)3 * r + (size_t)r * r + 2;
}

int32_t jacobi_eig(double *A, double *Abuf, double *V, double *w, int r, double *scratch,
                   hipStream_t s) {
  double *cs = scratch;
  double *sg = scratch + r;
  int *partner = reinterpret_cast<int *>(scratch + 2 * r);
  double *Vbuf = scratch + 3 * r;
  double *off = Vbuf + (size_t)r * r;
  const int64_t tot = (int64_t)r * r;
  const unsigned gb = (unsigned)ceil_div(tot, 256);
  hipLaunchKernelGGL(eye_kernel, dim3(gb), dim3(256), 0, s, V, r);
  NYS_LAUNCH_CHECK();
  if (r == 1) {
    hipLaunchKernelGGL(diag_kernel, dim3(1), dim3(64), 0, s, A, w, r);
    NYS_LAUNCH_CHECK();
    return NYS_OK;
  }
  const int rr = r + (r & 1);
  double *Ac = A, *An = Abuf, *Vc = V, *Vn = Vbuf;
  double host_off[2] = {0, 0};
  const int max_sweeps = 40;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    for (int round = 0; round < rr - 1; ++round) {
      hipLaunchKernelGGL(jacobi_params_kernel, dim3((unsigned)ceil_div(rr / 2, 256)), dim3(256), 0, s, Ac, r,
                         rr, round, cs, sg, partner);
      hipLaunchKernelGGL(jacobi_apply_kernel, dim3(gb), dim3(256), 0, s, Ac, An, Vc, Vn, r, cs, sg,
                         partner);
      std::swap(Ac, An);
      std::swap(Vc, Vn);
    }
    NYS_LAUNCH_CHECK();
    hipLaunchKernelGGL(offdiag_kernel, dim3(1), dim3(256), 0, s, Ac, r, off);
    NYS_LAUNCH_CHECK();
    NYS_CHECK_HIP(hipMemcpyAsync(host_off, off, sizeof(host_off), hipMemcpyDeviceToHost, s));
    NYS_CHECK_HIP(hipStreamSynchronize(s));
    if (!(host_off[0] <= 1e-30 * host_off[1])) continue;
    break;
  }
  if (!std::isfinite(host_off[0]) || !std::isfinite(host_off[1])) {
    set_error("nys_precond_build: non-finite values in the Jacobi eigensolver");
    return NYS_ENUMERIC;
  }
  // Past the sweep cap the off-diagonal mass bounds the eigenvalue error (Weyl):
  // up to 1e-12 of the matrix norm is harmless for a preconditioner, more is reported.
  if (!(host_off[0] <= 1e-24 * host_off[1])) {
    set_error("nys_precond_build: the Jacobi eigensolver did not converge in " + std::to_string(max_sweeps) +
              " sweeps (relative off-diagonal norm " + std::to_string(std::sqrt(host_off[0] / host_off[1])) + ")");
    return NYS_ENUMERIC;
  }
  hipLaunchKernelGGL(diag_kernel, dim3((unsigned)ceil_div(r, 256)), dim3(256), 0, s, Ac, w, r);
  NYS_LAUNCH_CHECK();
  if (Vc != V) NYS_CHECK_HIP(hipMemcpyAsync(V, Vc, sizeof(double) * tot, hipMemcpyDeviceToDevice, s));
  return NYS_OK;
}

// ------------------------------------------------------------ eigenpairs -> T, lam_hat
// Thread i ranks eigenvalue w_i (descending, ties by index); kept pairs
// (w_i > 1e-14 max w) give column rank(i) of T = V diag(w^{-1/2}) and
// lam_hat = max(0, w_i - nu); dropped pairs give zero columns and lam_hat = 0.
__global__ __launch_bounds__(1024) void eig_finish_kernel(const double *w, const double *V, int r,
                                                          double nu, double *T, double *lam_hat,
                                                          int *rank_out) {
  __shared__ double wmax;
  __shared__ int kept;
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int i = 0; i < r; ++i) m = w[i] > m ? w[i] : m;
    wmax = m;
    kept = 0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < r; i += blockDim.x) {
    const double wi = w[i];
    int rk = 0;
    for (int j = 0; j < r; ++j) {
      const double wj = w[j];
      if (wj > wi || (wj == wi && j < i)) ++rk;
    }
    const bool keep = wi > 1e-14 * wmax && wi > 0.0;
    if (keep) atomicAdd(&kept, 1);
    const double inv = keep ? 1.0 / sqrt(wi) : 0.0;
    for (int k = 0; k < r; ++k) T[(int64_t)k * r + rk] = V[(int64_t)k * r + i] * inv;
    lam_hat[rk] = keep ? (wi - nu > 0.0 ? wi - nu : 0.0) : 0.0;
  }
  __syncthreads();
  if (threadIdx.x == 0) rank_out[0] = kept;
}

int32_t launch_eig_finish(const double *w, const double *V, int r, double nu, double *T,
                          double *lam_hat, int *rank_out, hipStream_t s) {
  hipLaunchKernelGGL(eig_finish_kernel, dim3(1), dim3(1024), 0, s, w, V, r, nu, T, lam_hat, rank_out);
  NYS_LAUNCH_CHECK();
  return NYS_OK;
}

}  // namespace nys
