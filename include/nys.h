/*
 * nys.h -- C ABI of libnys: Nystrom-preconditioned conjugate gradient (NysPCG)
 * for kernel systems (K + lambda I) x = b on one AMD Instinct MI355X (gfx950).
 *
 * The operation is the regularised positive-definite system of the paper's
 * section "Positive-Definite Linear Systems" (eq. rlaopt-regularized-linear-system)
 * with K the kernel matrix of kernel ridge regression (eq. rlaopt-krr),
 * K_ij = k(x_i, x_j), evaluated on the fly and never stored.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Array arguments are DEVICE pointers unless marked "host".  Matrices are
 *    row-major and dense (a row of an n x m matrix is m contiguous elements).
 *  - All arrays are owned by the caller.  The library never allocates device
 *    memory for them, never frees them and keeps no pointer after returning.
 *  - Scratch memory is passed in as (ws, ws_bytes): a device buffer of at
 *    least the size nys_workspace_bytes() reports for the same arguments,
 *    aligned to 256 bytes.  Its contents on entry are irrelevant.
 *  - `stream` is a hipStream_t (NULL: the null stream).  Work is enqueued on
 *    it; entry points that return host values or host-side decisions
 *    (status of a factorisation, convergence) synchronise that stream.
 *  - Return value: NYS_OK (0), NYS_NOT_CONVERGED (1, not an error: outputs
 *    are valid) or a negative error code.  Nothing aborts and no C++
 *    exception crosses this boundary.  nys_last_error() describes the last
 *    non-zero status of the calling thread.
 *  - Calls on different streams with disjoint buffers may run concurrently.
 *
 * Kernels (the paper names the kernel function k but not its form):
 *    NYS_RBF        k(x, y) = exp(-|x - y|_2^2 / (2 sigma^2))
 *    NYS_LAPLACIAN  k(x, y) = exp(-|x - y|_2 / sigma)        (Euclidean norm)
 *
 * Precisions of the kernel product K V:
 *    NYS_FP64    distances, exponentials and accumulation in float64.
 *    NYS_FP32    float32 MFMA distance products, float32 exp2, float32 accumulation.
 *    NYS_BF16X3  bfloat16 split-precision distance products: each operand
 *                a = a_hi + a_lo (round-to-nearest-even bfloat16 parts) and
 *                a.b ~ a_hi.b_hi + a_hi.b_lo + a_lo.b_hi on MFMA with float32
 *                accumulation; for m >= 16 columns the product with V uses the
 *                same three-term split.  About 16 significant bits per product.
 *    NYS_BF16X3_D6  as NYS_BF16X3, but the distance operands are split into
 *                three bf16 parts and the six leading products are kept
 *                (hh + hm + mh + hl + lh + mm), about 24 bits.  The three-term
 *                distance leaves a structured error K o (X_lo X_lo^T) of norm
 *                about 2^-17 (d / sigma^2) |K|; when lambda is below that the
 *                perturbed operator can be indefinite and CG diverges, so small
 *                regularisations (lambda < ~1e-5 |K|) need this variant.
 *    NYS_BF16X3_D10 four bf16 parts per distance operand and the ten products
 *                of total order <= 3 (hh; hm, mh; hl, lh, mm; h4, 4h, ml, lm),
 *                about 32 bits.  The six-term split still leaves a structured
 *                distance error of about 2^-27 (d / sigma^2) |K|, which bounds
 *                how much one float64 refinement cycle can gain when lambda is
 *                within a few decades of 1e-7 |K|; the ten-term split removes it
 *                for about 1.5x the distance work (d <= 24).
 *    NYS_F16X3_D10  distances as NYS_BF16X3_D10; the K V product splits K and V
 *                into fp16 parts instead (11 + 11 significand bits each, same
 *                MFMA rate), with every column of V scaled by a power of two
 *                so that its largest entry lies in [0.5, 1) and the scale undone
 *                on output.  Entries far below their column's largest lose
 *                relative (not absolute) accuracy.  About 2^-22 per product
 *                entry against 2^-17 for the bf16 split, which is what limits
 *                a refinement cycle once the distance error is gone (d <= 24).
 *    NYS_F16X3_D6   the fp16 K V product of NYS_F16X3_D10 over the six-term
 *                distance of NYS_BF16X3_D6 (d <= 41): two thirds of the exponent
 *                chain's MFMA work at d = 16 (four 32-wide K-steps against six).
 *                Where the exponent's float32 accumulation and exp2 set the
 *                entry error, as for standardised points at sigma^2 >= d / 2,
 *                its entries are as accurate as NYS_F16X3_D10's (measured at
 *                n = 1e6, d = 16, sigma = 4: relative entry error spread 4.7e-8
 *                for both distance splits).
 */
#ifndef NYS_H
#define NYS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define NYS_OK             0
#define NYS_NOT_CONVERGED  1   /* iteration cap reached; outputs valid, info filled */
#define NYS_EINVAL        (-1) /* invalid argument (null pointer, size, sigma <= 0,
                                  lambda <= 0, tol <= 0, unsupported kind/precision) */
#define NYS_ENOTPD        (-2) /* shifted Cholesky of the sketch core failed after
                                  all shift retries, or PCG breakdown (p^T A p <= 0) */
#define NYS_ENUMERIC      (-3) /* NaN or Inf in inputs or in PCG scalars */
#define NYS_EHIP          (-4) /* HIP runtime error */
#define NYS_ENOMEM        (-5) /* workspace smaller than nys_workspace_bytes() */

typedef enum { NYS_RBF = 0, NYS_LAPLACIAN = 1 } nys_kind;
typedef enum {
  NYS_FP64 = 0, NYS_FP32 = 1, NYS_BF16X3 = 2, NYS_BF16X3_D6 = 3, NYS_BF16X3_D10 = 4, NYS_F16X3_D10 = 5,
  NYS_F16X3_D6 = 6
} nys_prec;

/* Operations whose workspace can be queried. */
typedef enum {
  NYS_OP_KERNEL_MATVEC = 0,
  NYS_OP_SKETCH = 1,
  NYS_OP_PRECOND_BUILD = 2,
  NYS_OP_PRECOND_APPLY = 3,
  NYS_OP_SOLVE = 4,
  NYS_OP_BACKWARD = 5,
  NYS_OP_AUTOTUNE = 6,
  NYS_OP_KERNEL_DOT = 7,
  NYS_OP_PRECOND_ADAPTIVE = 8,
  NYS_OP_RIDGE_SKETCH = 9,
  NYS_OP_RIDGE_SOLVE = 10,
  NYS_OP_ADMM_ELASTIC_NET = 11
} nys_op;

/* Kernel function: kind (nys_kind) and bandwidth sigma > 0. */
typedef struct {
  int32_t kind;
  int32_t reserved;
  double sigma;
} nys_kernel;

/* Nystrom preconditioner P = U diag(lam_hat) U^T + (lambda + shift) I, with lambda the
 * regularisation of the column being solved (the base damping) and shift 0 for the
 * damping mode "non_adaptive" or the smallest retained lam_hat for "adaptive" (table
 * tab:rlaopt-nystrom-config).  The caller allocates the buffers; nys_precond_build
 * (shift 0) or nys_precond_adaptive fills them.
 *    n        number of points (rows of U)
 *    r        sketch size = columns of U (rank_init of the paper's NystromConfig)
 *    rank     out: columns of U kept (those with sigma_i^2 > 1e-14 sigma_1^2);
 *             dropped columns of U are zero and their lam_hat is 0
 *    U        device, n x r float64, orthonormal columns
 *    U32      device, n x r float32 copy of U, or NULL (filled when given; the
 *             apply itself always works from U in float64)
 *    lam_hat  device, r float64, descending, >= 0
 *    nu       out: the shift used by the stabilised approximation
 *    shift    extra damping added to every column's lambda in the apply (out of
 *             nys_precond_build: 0; of nys_precond_adaptive: per damping mode)
 */
typedef struct {
  int64_t n;
  int32_t r;
  int32_t rank;
  double *U;
  float *U32;
  double *lam_hat;
  double nu;
  double shift;
} nys_precond;

/* Damping modes of table tab:rlaopt-nystrom-config. */
#define NYS_DAMPING_NON_ADAPTIVE 0   /* damping = base damping (lambda) */
#define NYS_DAMPING_ADAPTIVE     1   /* damping = lambda + smallest retained lam_hat */

/* Nystrom configuration with rank adaptation (NystromConfig of table
 * tab:rlaopt-nystrom-config).
 *    rank_init        initial sketch size l (>= 1)
 *    rank_max         largest l (0: rank_init, i.e. no adaptation)
 *    num_power_iters  power iterations of the error estimate (paper default 10)
 *    damping_mode     NYS_DAMPING_ADAPTIVE (paper default) or NYS_DAMPING_NON_ADAPTIVE
 *    error_tolerance  stop when the estimate of |K - K_hat|_2 is at most
 *                     error_tolerance * lam_hat_1 (paper default 1e-2)
 *    seed             the test matrix is nys_test_matrix(seed, n, rank_max); the power
 *                     iteration starts from nys_test_matrix(seed + 1, n, 1) */
typedef struct {
  int32_t rank_init;
  int32_t rank_max;
  int32_t num_power_iters;
  int32_t damping_mode;
  double error_tolerance;
  uint64_t seed;
} nys_nystrom_config;

/* PCG options (PCGStoppingCriteria, table tab:rlaopt-pcg-stopping, plus the
 * precision controls of this library).
 *    tol           relative residual target: column c stops when
 *                  |r_c|_2 <= tol |b_c|_2 (default of the paper: 1e-6)
 *    max_iters     cap on products with A per column (paper default 1000)
 *    prec          nys_prec of the kernel product and of the CG vectors
 *                  (FP64: float64 vectors; FP32/BF16X3: float32 vectors)
 *    refine_every  FP32/BF16X3 only (float64 refinement; -1 disables it and the
 *                  columns stop on their recursive residual).  A refinement
 *                  accumulates the column's iterate in float64, recomputes
 *                  r = b - (K + lambda I) x with the float64 kernel product and
 *                  accepts the column only if that true residual meets tol.
 *                  refine_every > 0: every refine_every iterations all active
 *                  columns are refined.  0: a column is refined when its
 *                  recursive residual has fallen by its cycle factor since its
 *                  last refinement, or meets tol; columns close to that point
 *                  join the same float64 product.
 *    refine_mode   0: after a refinement keep the search direction when the true
 *                  residual is within 0.8x..1.25x of the recursive one, else
 *                  restart the recurrence (p = z); 1: always restart;
 *                  2: drift-controlled residual replacement (refine_every == 0):
 *                  the refinement also measures the drift q = |r_true - r_rec| /
 *                  |r_rec|; the search direction is kept unless q > 0.5, and the
 *                  next cycle factor is rescaled so that the drift at its end is
 *                  about 0.1 |r_rec| (the drift grows with the reduction a cycle
 *                  makes, so a small replaced perturbation keeps the Krylov
 *                  recurrence useful instead of restarting it)
 *    check_true    1: after the solve compute the float64 true relative residual
 *                  of every column into info (eq. experiment-relative-residual)
 *    max_refinements  cap on refinements per column (0: 50)
 *    refine_reduction  first cycle factor of refine_every == 0 (0: tol); later
 *                  cycles use max(refine_reduction, min(0.5, g)) with g the
 *                  true-residual reduction the previous cycle achieved (modes
 *                  0, 1) or the drift rescaling above (mode 2)
 *    refine_join   refine_every == 0: when one column is due, every column whose
 *                  recursive residual is within refine_join times its own cycle
 *                  target joins the same float64 product (0: 3; else >= 1).
 *                  Larger values trade restarts a little early for fewer float64
 *                  products, each of which costs a full sweep over the n^2 pairs.
 *    block         0: every column its own PCG (the default).  1: block PCG
 *                  (O'Leary): the nrhs right-hand sides of each lambda share one
 *                  block Krylov space (nrhs <= 64, every right-hand side of a lambda
 *                  non-zero); the lambdas share each kernel product.  Low-precision
 *                  products refine whole blocks in cycles (refine_every must be 0;
 *                  refine_mode and refine_join do not apply; every refinement
 *                  restarts the block).  A block's first cycle factor is raised to
 *                  the drift (true - recursive relative residual) that the blocks
 *                  already refined left at the end of their first cycle, scaled by
 *                  their lambda over its lambda.  NYS_ENOTPD when a block loses rank
 *                  twice in a row.
 */
typedef struct {
  double tol;
  int32_t max_iters;
  int32_t prec;
  int32_t refine_every;
  int32_t refine_mode;
  int32_t check_true;
  int32_t max_refinements;
  double refine_reduction;
  double refine_join;
  int32_t block;
  int32_t reserved;
} nys_pcg_opts;

/* Per-column result. */
typedef struct {
  int32_t iters;            /* products with A after set-up */
  int32_t refinements;      /* float64 residual recomputations */
  int32_t status;           /* NYS_OK or NYS_NOT_CONVERGED */
  int32_t reserved;
  double relres_recursive;  /* |r_k| / |b| of the recurrence when it stopped */
  double relres_true;       /* float64 |b - (K + lambda I) x| / |b| (check_true or refinement), else -1 */
} nys_col_info;

/* Workspace size for an operation.  Unused size arguments may be 0.
 *   KERNEL_MATVEC: n = nr, n2 = nc, d, m, prec
 *   SKETCH:        n, d, r, prec
 *   PRECOND_BUILD: n, r
 *   PRECOND_APPLY: n, r, m, prec
 *   SOLVE:         n, d, r (0 if no preconditioner), m = nlam * nrhs, prec
 *   BACKWARD:      n, d, r, prec
 *   AUTOTUNE:      n = n_rows, n2 = n, d, m, prec
 *   KERNEL_DOT:    n = nr, n2 = nc, d
 *   PRECOND_ADAPTIVE: n, d, r = rank_max, prec
 *   RIDGE_SKETCH:  n = rows of X, n2 = p, r
 *   RIDGE_SOLVE:   n = rows of X, n2 = p, d = nrhs, r (0 if no preconditioner),
 *                  m = nlam * nrhs
 *   ADMM_ELASTIC_NET: n = rows of X, n2 = p, r = preconditioner rank
 * Returns NYS_OK and *bytes, or NYS_EINVAL. */
int32_t nys_workspace_bytes(int32_t op, int64_t n, int64_t n2, int32_t d, int32_t r, int32_t m,
                            int32_t prec, size_t *bytes);

/* kernel_matvec: Out = alpha * K(Xr, Xc) V + beta * Out, or with deriv = 1 the
 * entrywise derivative dK/dsigma in place of K (RBF: k d^2 / sigma^3;
 * Laplacian: k d / sigma^2).  This is the matrix-free operator product the
 * paper applies inside CG (section "Positive-Definite Linear Systems": O(n^2)
 * work per CG iteration) and its sketch product (the preconditioner build).
 *    Xr   device float64 nr x d (row points, rows of K)
 *    Xc   device float64 nc x d (column points); Xr == Xc with nr == nc marks a
 *         symmetric product and K_ii is taken as exactly 1
 *    V    device nc x m, float64 if prec == NYS_FP64 else float32
 *    Out  device nr x m, same type as V; not read when beta == 0
 * Coordinates are centred on the column mean of Xc (distances are unchanged).
 * d must be <= 62 (FP32/FP64), <= 82 (BF16X3), <= 41 (BF16X3_D6, F16X3_D6) or <= 24
 * (the ten-term splits).  The low-precision products sum the columns' contributions
 * in float32 over ranges of column points and add the ranges in float64: ranges of
 * at most 16384 points where the range sums fit in 32 GiB of workspace, fewer and
 * longer ranges where they would not (n = 1e6: 62 ranges up to 128 columns, 16 at
 * 512), so the float32 rounding of an output grows with the range, not with nc.  The stream is synchronised once, after the points
 * are packed and before the product is enqueued, to read the packing's finiteness
 * check: a NaN or Inf coordinate in Xr or Xc returns NYS_ENUMERIC. */
int32_t kernel_matvec(nys_kernel k, int32_t deriv, int32_t prec,
                      const double *Xr, int64_t nr, const double *Xc, int64_t nc, int32_t d,
                      const void *V, int32_t m, void *Out, double alpha, double beta,
                      void *ws, size_t ws_bytes, void *stream);

/* kernel_dot: *out = u^T K(Xr, Xc) v, or with deriv = 1 u^T (dK/dsigma) v, in
 * float64: the scalar contractions of the kernel with two vectors that the
 * gradient of a validation loss through the solution needs (eq. rlaopt-bilevel:
 * the explicit sigma-derivative e^T (dK_vt/dsigma) x of the prediction K_vt x).
 *    Xr  device float64 nr x d;  Xc  device float64 nc x d (Xr == Xc with nr == nc
 *        marks a symmetric product, K_ii = 1 exactly)
 *    u   device float64 nr;  v  device float64 nc
 *    out HOST, one double
 * Synchronises the stream.  NaN or Inf in Xr or Xc: NYS_ENUMERIC. */
int32_t kernel_dot(nys_kernel k, int32_t deriv, const double *Xr, int64_t nr, const double *Xc, int64_t nc,
                   int32_t d, const double *u, const double *v, double *out, void *ws, size_t ws_bytes,
                   void *stream);

/* nys_test_matrix: Omega (n x r, device float64, row-major) filled with standard
 * normals as a pure function of (seed, element index): Philox4x32 with 10 rounds
 * (Salmon et al., SC 2011) on the counter (b mod 2^32, b / 2^32, 0, 0) with key
 * (seed mod 2^32, seed / 2^32) for the element pair b = e / 2, two 53-bit uniforms
 * u, v from the output words (w0, w1) and (w2, w3), and the Box-Muller pair
 * sqrt(-2 ln u) (cos 2 pi v, sin 2 pi v) (cosine for even e, sine for odd e).
 * Any row range of Omega can therefore be drawn independently.  This is the
 * Gaussian test matrix of the randomized Nystrom sketch (the method the paper
 * cites for its preconditioner).  Enqueued on stream; no synchronisation. */
int32_t nys_test_matrix(uint64_t seed, int64_t n, int32_t r, double *Omega, void *stream);

/* nys_sketch: the sketch Y = K Q of the randomized Nystrom approximation (the
 * preconditioner the paper cites in "Related Work", configured by table
 * tab:rlaopt-nystrom-config).
 *    X      device float64 n x d
 *    Omega  device float64 n x r, the standard Gaussian test matrix (read only), or
 *           NULL: drawn on the device from `seed` as nys_test_matrix does
 *    seed   used only when Omega is NULL
 *    Q      device float64 n x r, out: the orthonormalised test matrix
 *           Q = Omega L^{-T}, L L^T = Omega^T Omega (Cholesky QR); must not
 *           overlap Omega.  nys_precond_build takes it together with Y.
 *    Y      device float64 n x r, out: K Q computed with the precision prec
 * Requires 1 <= r <= n and r <= 1024.  NYS_ENOTPD if Omega^T Omega is not
 * positive definite (rank-deficient or non-finite Omega); NYS_ENUMERIC for NaN or
 * Inf in X.  Synchronises the stream. */
int32_t nys_sketch(nys_kernel k, int32_t prec, const double *X, int64_t n, int32_t d,
                   const double *Omega, uint64_t seed, int32_t r, double *Q, double *Y, void *ws,
                   size_t ws_bytes, void *stream);

/* nys_precond_build: stabilised fixed-rank Nystrom approximation from the
 * sketch, all in float64 on the device:
 *    nu = max(sqrt(n) 2^-52 |Y|_F, c_prec |Y|_F / sqrt(r)), Y_nu = Y + nu Q,
 *    L L^T = (Q^T Y_nu + Y_nu^T Q) / 2 (retried with nu *= 10 up to 5 times),
 *    B = Y_nu L^{-T}, B^T B = V S^2 V^T (Jacobi), U = B V S^{-1},
 *    lam_hat = max(0, S^2 - nu), descending.
 *    sketch_prec  the precision Y was computed in (sets c_prec: 0 for FP64,
 *                 2^-21 FP32, 2^-14 BF16X3: the sketch error the shift must cover)
 *    P      in: n, r, U, U32 (nullable), lam_hat buffers; out: filled, rank, nu.
 * Returns NYS_ENOTPD if the shifted core never factors. */
int32_t nys_precond_build(const double *Y, const double *Q, int64_t n, int32_t r, int32_t sketch_prec,
                          nys_precond *P, void *ws, size_t ws_bytes, void *stream);

/* nys_precond_adaptive: the Nystrom preconditioner with rank adaptation and the damping
 * mode of cfg (table tab:rlaopt-nystrom-config).  The paper lists the parameters but
 * not the loop; this one starts at l = rank_init and, while the power-iteration
 * estimate of |K - K_hat|_2 exceeds error_tolerance * lam_hat_1 and l < rank_max,
 * doubles l (capped at rank_max).  Growing l applies K only to the test-matrix columns
 * added: the sketch K Omega of the first l columns is orthonormalised by Cholesky QR
 * (Q = Omega_l L^-T, Y = (K Omega_l) L^-T) and built as nys_precond_build does.  The
 * kernel products (sketch and power iteration) run at precision prec.
 *    P       in: n, r = rank_max, buffers U (n x rank_max), U32 (nullable), lam_hat
 *            (rank_max); out: r = the final l, U as n x l (row stride l) at the start
 *            of the buffer, lam_hat (zero past l), rank, nu, shift
 *    err_out HOST, nullable: the last error estimate
 * NYS_ENOTPD / NYS_ENUMERIC as nys_sketch and nys_precond_build. */
int32_t nys_precond_adaptive(nys_kernel k, int32_t prec, const double *X, int64_t n, int32_t d,
                             const nys_nystrom_config *cfg, nys_precond *P, double *err_out, void *ws,
                             size_t ws_bytes, void *stream);

/* nys_precond_apply: Z = P_c^{-1} R for every column c, with
 * P_c = U diag(lam_hat) U^T + rho_c I, rho_c = lambdas[c] + P->shift, through the closed form
 * P_c^{-1} = U diag(1/(lam_hat + rho_c)) U^T + (I - U U^T) / rho_c.
 *    lambdas  device float64, m values (lambda_c > 0)
 *    R, Z     device n x m; float64 if prec == NYS_FP64, else float32
 * The arithmetic is float64 in every case (float32 vectors are rounded once on
 * output): for lambda far below lam_hat_1 the two terms cancel inside span(U),
 * and a float32 evaluation would leave P^{-1} indefinite.
 * R and Z must not overlap. */
int32_t nys_precond_apply(const nys_precond *P, const double *lambdas, int32_t prec,
                          const void *R, int32_t m, void *Z, void *ws, size_t ws_bytes, void *stream);

/* nyspcg_solve: NysPCG (or plain CG when P == NULL) on nlam * nrhs independent
 * columns sharing one kernel matrix and one preconditioner: column
 * c = l * nrhs + j solves (K + lambdas[l] I) x = B[:, j].  Each column stops on
 * its own when |r_c| <= tol |b_c| (table tab:rlaopt-pcg-stopping: the criterion
 * must hold for every right-hand side) or at max_iters.  x0 = 0.  A column with
 * b = 0 returns x = 0 after 0 iterations.
 *    X        device float64 n x d
 *    B        device float64 n x nrhs
 *    lambdas  HOST float64, nlam values > 0
 *    P        NULL (plain CG) or a built preconditioner for the same X
 *    Xsol     device float64 n x (nlam * nrhs), out
 *    info     HOST, nlam * nrhs entries, out
 * Returns NYS_OK if every column converged, NYS_NOT_CONVERGED otherwise. */
int32_t nyspcg_solve(nys_kernel k, const double *X, int64_t n, int32_t d,
                     const double *B, int32_t nrhs, const double *lambdas, int32_t nlam,
                     const nys_precond *P, const nys_pcg_opts *opts,
                     double *Xsol, nys_col_info *info, void *ws, size_t ws_bytes, void *stream);

/* nyspcg_backward: adjoint of x* = (K + lambda I)^{-1} b for the bilevel problem
 * of eq. rlaopt-bilevel.  Given gx = dL/dx*, solves (K + lambda I) a = gx with the
 * same preconditioner (a = dL/db) and returns
 *    dL/dlambda = -a^T x*,   dL/dsigma = -a^T (dK/dsigma) x*.
 *    xsol, gx  device float64 n (one column)
 *    adj       device float64 n, out
 *    dL_dlambda, dL_dsigma  HOST, out
 *    info      HOST, one entry, out (the adjoint solve) */
int32_t nyspcg_backward(nys_kernel k, const double *X, int64_t n, int32_t d, double lambda,
                        const double *xsol, const double *gx, const nys_precond *P,
                        const nys_pcg_opts *opts, double *adj, double *dL_dlambda,
                        double *dL_dsigma, nys_col_info *info, void *ws, size_t ws_bytes,
                        void *stream);

/* ---- tile autotuner -------------------------------------------------------
 * The batched solve runs the kernel product at many column counts (columns
 * leave as they converge).  nys_autotune times kernel_matvec(X[0:n_rows], X)
 * on the calling stream for every candidate column-chunk width of the tile the
 * precision uses at m columns (the instantiated widths 16..256 with at most 4
 * chunks and at most twice the next power of two of m), reps timed calls each
 * after one untimed call, and records the fastest for column counts in
 * [m_lo, m] of this precision; later plans (kernel_matvec, nys_sketch,
 * nyspcg_solve, nyspcg_backward, nys_workspace_bytes) use it.  best gets the
 * width and its average milliseconds ({0, 0, 0} when m runs on the row-sum
 * tile, which has no width to choose).  Synchronizes the stream.  The
 * choice is process-wide; query workspace sizes after tuning.  X is n x d
 * float64 (device), ws at least nys_workspace_bytes(NYS_OP_AUTOTUNE, n_rows, n,
 * d, 0, m, prec).  nys_set_tile installs a width (e.g. from a cache of earlier
 * runs; tm = 0 removes the range) and nys_clear_tiles drops every choice.
 * Valid widths: FP64 16, 32, 48, 64, 96, 128, 256 (without a tuned width its
 * planner takes the least cost over full chunks plus a tail chunk from a per-chunk
 * cost table); FP32 32, 64, 128; F16X3_D10 and F16X3_D6 16..256 (each its own table)
 * and the bf16 splits 32..256 (one table shared by BF16X3, D6 and D10), in powers of
 * two.  For FP64 with m >= 256, nys_autotune instead times one chunk of
 * every float64 width (m_lo is ignored) and replaces that cost table for this shape,
 * so every later float64 product is sized by measured cost; best gets the width the
 * planner then takes at m columns and its estimated milliseconds.  nys_clear_tiles
 * restores the default table (measured at n = 1e6, d = 16).  Whatever the width, the last
 * chunk of a product runs at the narrowest width that holds the remaining
 * columns. */
typedef struct {
  int32_t tm;        /* column-chunk width */
  int32_t reserved;
  double ms;         /* average duration of one product at that width */
} nys_tile_choice;

int32_t nys_autotune(nys_kernel k, int32_t prec, const double *X, int64_t n, int64_t n_rows, int32_t d,
                     int32_t m, int32_t m_lo, int32_t reps, nys_tile_choice *best, void *ws, size_t ws_bytes,
                     void *stream);
int32_t nys_set_tile(int32_t prec, int32_t m_lo, int32_t m_hi, int32_t tm);
void nys_clear_tiles(void);

/* Host-only query of the plan kernel_matvec would use for an n x n product with m
 * columns at precision prec and dimension d (tuned widths included): *tm gets the
 * column-chunk width and *tail_tm the width of the last chunk when it is narrower
 * (0 otherwise); both are 0 when m runs on the row-sum tile.  No device work, no
 * allocation.  Returns NYS_EINVAL for an unsupported precision, n < 1, m < 1, d out
 * of range or a null output. */
int32_t nys_plan_chunks(int32_t prec, int64_t n, int32_t d, int32_t m, int32_t *tm, int32_t *tail_tm);

/* Host-only query of how the same product splits its column points into ranges,
 * each summed in its own accumulator and the ranges added in float64: *ranges gets
 * their number and *points the column points of each (the last one may hold fewer).
 * The low-precision products take ranges of at most 16384 points, fewer and longer
 * ones where the range sums of an n x m product would exceed 32 GiB; the float64
 * products split only to fill the GPU.  No device work, no allocation.  Returns
 * NYS_EINVAL as nys_plan_chunks does. */
int32_t nys_plan_ranges(int32_t prec, int64_t n, int32_t d, int32_t m, int32_t *ranges, int64_t *points);

/* ---- ceiling probes --------------------------------------------------------
 * nys_peak_probe times one synthetic kernel that keeps a single unit of the GPU
 * busy, so that the rates of the kernel product can be set against what the chip
 * sustains as well as against its data sheet.  It is measurement support, not
 * part of the method.
 *    which  0: bf16 MFMA (v_mfma_f32_16x16x32_bf16), flop/s
 *           1: fp16 MFMA (v_mfma_f32_16x16x32_f16), flop/s
 *           2: float64 MFMA (v_mfma_f64_16x16x4f64), flop/s
 *           3: float32 exp2 (v_exp_f32), exponentials/s
 *           4: device copy over the workspace (first half to second half),
 *              bytes read + written per second
 *    iters  loop length per lane (0: about 50-100 ms per launch); for which = 4
 *           the number of timed copies (0: one)
 *    rate   HOST, out
 * ws: device scratch, at least 2 MiB (which = 4 copies ws_bytes / 2 bytes, so a
 * large workspace measures HBM rather than cache).  One untimed launch precedes the
 * timed one(s) on `stream`; synchronises the stream.  NYS_EINVAL for which outside
 * 0..4 or a null pointer, NYS_ENOMEM for a smaller workspace. */
int32_t nys_peak_probe(int32_t which, int32_t iters, double *rate, void *ws, size_t ws_bytes, void *stream);

/* ---- ridge regression (the paper's own NysPCG workload) --------------------
 * The regularised normal equations (X^T X + lambda I) w = X^T y of ridge regression
 * (section "Large-Scale Ridge Regression with NysPCG", eq. experiment-ridge), with the
 * normal matrix applied matrix-free through two float64 products with the dense data
 * matrix X (n x p, row-major, device) and never formed; the products are rocBLAS
 * GEMMs.  The Nystrom preconditioner of X^T X is built from nys_ridge_sketch's (Y, Q)
 * by nys_precond_build (or used with nys_precond_apply) exactly as for a kernel.
 *
 * nys_ridge_sketch: Q = the orthonormalised p x r test matrix (Omega, read only, or
 * drawn from `seed` when NULL, as nys_sketch), Y = X^T (X Q) (p x r).  Requires
 * 1 <= r <= min(p, 1024).  Synchronises the stream.
 *
 * nys_ridge_solve: NysPCG (or CG when P == NULL) for every column c = l nrhs + j:
 * (X^T X + lambdas[l] I) w = X^T y_j, y the n x nrhs targets (device).  Float64
 * only (opts->prec must be NYS_FP64; no refinement is involved).  W is p x (nlam
 * nrhs) (device), info and lambdas HOST, as nyspcg_solve; check_true reports the
 * float64 residual |(X^T X + lambda I) w - X^T y| / |X^T y| (eq.
 * experiment-relative-residual).  Returns NYS_OK or NYS_NOT_CONVERGED. */
int32_t nys_ridge_sketch(const double *X, int64_t n, int64_t p, const double *Omega, uint64_t seed, int32_t r,
                         double *Q, double *Y, void *ws, size_t ws_bytes, void *stream);
int32_t nys_ridge_solve(const double *X, int64_t n, int64_t p, const double *Yt, int32_t nrhs,
                        const double *lambdas, int32_t nlam, const nys_precond *P, const nys_pcg_opts *opts,
                        double *W, nys_col_info *info, void *ws, size_t ws_bytes, void *stream);

/* ---- NysADMM on the bounded elastic net -----------------------------------
 * min over w, b of (1/2n)|X w + b 1 - y|^2 + lam1 |w|_1 + lam2/2 |w|^2 subject to
 * lo <= w <= hi (eq. experiment-bounded-en; the paper's instances use [0, 1]), by
 * ADMM on the splitting x = z (section "Splitting for ADMM") with NysPCG solving
 * every x-subproblem.  X is dense (n x p, row-major, device); the intercept is
 * unregularised and eliminated by centring (the library forms X - 1 mu^T in the
 * workspace), and the Hessian H = X_c^T X_c / n is applied matrix-free through two
 * float64 rocBLAS products, never formed.  Iteration k = 1, 2, ...:
 *   - every precond_update_freq iterations a fresh Nystrom approximation of H,
 *     test matrix nys_test_matrix(seed + refresh count, p, rank);
 *   - (H + (rho + sigma) I) x = X_c^T y / n + rho (z - u) + sigma x_prev by NysPCG
 *     warm-started at x_prev, to relative residual
 *     min(1, sqrt(|r_pri| |r_dual|)) k^-gamma (previous residuals; 1 at k = 1);
 *   - over-relaxation xh = alpha x + (1 - alpha) z, the proximal step
 *     z = clip(soft(xh + u, lam1/rho) rho/(rho + lam2), lo, hi), u += xh - z;
 *   - r_pri = x - z, r_dual = grad f(x) + rho u; stop when
 *     |r_pri| <= sqrt(p) eps_abs + eps_rel max(|x|, |z|) and
 *     |r_dual| <= sqrt(p) eps_abs + eps_rel |rho u| (table tab:rlaopt-admm-stopping);
 *   - every rho_update_freq iterations: rho times rho_update_factor (u divided by
 *     it) when |r_pri| > rho_update_threshold |r_dual|, the reverse when
 *     |r_dual| > rho_update_threshold |r_pri|.
 * Configuration fields and defaults follow table tab:rlaopt-admm-config (rank 50,
 * the NysADMM default preconditioner); a zero field takes its default. */
typedef struct {
  double rho;                   /* initial penalty (1.0) */
  double rho_update_factor;     /* (2.0) */
  double rho_update_threshold;  /* (10.0) */
  int32_t rho_update_freq;      /* iterations between penalty updates (25) */
  int32_t precond_update_freq;  /* iterations between preconditioner refreshes (20) */
  double alpha;                 /* over-relaxation, 0 < alpha < 2 (1.6) */
  double sigma;                 /* proximal regularisation of the x-subproblem (1e-6) */
  double gamma;                 /* decay exponent of the subproblem tolerance, > 1 (1.2) */
  int32_t rank;                 /* Nystrom rank, 1 <= rank <= min(p, 1024) (50) */
  int32_t max_iters;            /* ADMM iterations (1000) */
  double eps_abs;               /* (1e-4) */
  double eps_rel;               /* (1e-4) */
  uint64_t seed;                /* test-matrix seed (0 is a valid seed) */
  int32_t pcg_max_iters;        /* per subproblem (1000) */
  int32_t reserved;
} nys_admm_config;

typedef struct {
  int32_t iters;           /* ADMM iterations run */
  int32_t converged;       /* 1 when both residual tests passed */
  int64_t pcg_iters;       /* PCG iterations over all subproblems */
  double r_pri, r_dual;    /* final residual norms */
  double eps_pri, eps_dual;/* and their tolerances */
  double rho;              /* final penalty */
  double intercept;        /* b = mean(y) - mu^T w */
} nys_admm_info;

/* W (device, p): the solution z (within the box).  y device (n).  info HOST.
 * Returns NYS_OK (converged), NYS_NOT_CONVERGED (max_iters reached; W and info hold
 * the last iterate), NYS_EINVAL (sizes, lo > hi, negative penalties, a config field
 * out of range), NYS_ENOMEM (workspace too small), NYS_ENOTPD / NYS_ENUMERIC (a
 * preconditioner build failed), NYS_EHIP. */
int32_t nys_admm_elastic_net(const double *X, int64_t n, int64_t p, const double *y, double lam1, double lam2,
                             double lo, double hi, const nys_admm_config *cfg, double *W, nys_admm_info *info,
                             void *ws, size_t ws_bytes, void *stream);

/* Thread-local description of the last non-zero status ("" if none). */
const char *nys_last_error(void);

/* Library version string. */
const char *nys_version(void);

#ifdef __cplusplus
}
#endif

#endif /* NYS_H */
