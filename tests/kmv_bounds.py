"""Error bounds of the GPU kernel product against the oracle, shared by the GPU tests.

The bound of one output element is the sum over its terms of a per-pair bound on the
computed kernel entry, times |V|, plus an accumulation term:

* The exponent t_ij = kappa (2 x_i.x_j - |x_i|^2 - |x_j|^2) comes out of one MFMA
  chain over augmented, centred coordinates.  The magnitudes it sums are at most
  kappa (r_i + r_j)^2 (r the distance to the column mean), so its absolute error is
  at most c u_d kappa (r_i + r_j)^2, with u_d the unit roundoff of the split distance
  products accumulated in float32 (2^-16 for the two-part bf16 split, float32 level
  for the six- and ten-term splits, 2^-53 in float64) and c = 16.  For the RBF
  kernel this is the relative error of k; for the Laplacian, k = exp(-d / sigma)
  with d = sqrt(d^2), an error e in d^2 moves d by e / (2 d), or by sqrt(e) when
  d^2 < e.
* exp2 (v_exp_f32) adds a few ulps of float32 (4 x 2^-22 here), the float64 table
  exp a few ulps of float64.
* Where the K V product splits K and V into parts (bf16: 2^-16 per operand; fp16:
  2^-22, the K parts carrying an absolute 2^-25 in the fp16 subnormal range and the V
  parts 2^-23 of their column's power-of-two scale), three split errors per term.
* Accumulation of n_c terms in float32 (float64): (8 sqrt(n_c) + 16) u |K| |V| for
  V >= 0, the probabilistic growth of sequential and blocked sums (the worst case
  n_c u would exceed |K V| itself at n_c = 1e6).
* With random-sign V the entry errors of one output are summed with random signs:
  the bound is Hoeffding's (see bound_from) instead of the worst-case sum.
The derivative dK/dsigma = k d^2 / sigma^3 (RBF) or k d / sigma^2 (Laplacian) adds the
error of its d^2 resp. d factor, and the whole entry bound is taken four times.

`guard` is what keeps such a bound able to fail: the largest tolerance of a case
must stay below a tenth of its largest |reference|, so an all-zero result, or one
that drops a split part, fails.
"""
import math
import numpy as np
import oracle as o

# unit roundoff of the exponent chain (split distance products, float32 accumulation)
UDIST = {0: 2.0 ** -53, 1: 2.0 ** -24, 2: 2.0 ** -16, 3: 2.0 ** -23, 4: 2.0 ** -24, 5: 2.0 ** -24, 6: 2.0 ** -23}
# relative error of one split operand of the K V product
USPLIT = {2: 2.0 ** -16, 3: 2.0 ** -16, 4: 2.0 ** -16, 5: 2.0 ** -22, 6: 2.0 ** -22}


def uacc(prec):
    return 2.0 ** -53 if prec == 0 else 2.0 ** -24


def uexp(prec):
    return 2.0 ** -52 if prec == 0 else 2.0 ** -22


def split_product(prec, m, deriv):
    if deriv:
        return False
    return prec in (5, 6) or (prec in (2, 3, 4) and m > 16)


def entry_abs_bound(Xr, Xc, kind, sigma, prec, m, deriv=0, same=None, mu=None):
    """Per-pair bound on |K~_ij - K_ij| (or of dK/dsigma) and the exact matrix.  mu is
    the centre the GPU packs the points around (the column mean of the full column
    point set; default: the mean of Xc)."""
    mu = Xc.mean(0) if mu is None else mu
    ri = np.linalg.norm(Xr - mu, axis=1)[:, None]
    rj = np.linalg.norm(Xc - mu, axis=1)[None, :]
    D = o.squared_distances(Xr, Xc)
    K = o.kernel_matrix(Xr, Xc, kind, sigma)
    kap = 1.0 / (2 * sigma * sigma) if kind == o.RBF else 1.0
    dt = 16 * UDIST[prec] * kap * (ri + rj) ** 2        # exponent argument (natural units)
    dd2 = dt / kap                                        # squared distance
    if kind == o.RBF:
        relk = dt
    else:
        dist = np.sqrt(D)
        relk = np.where(D > dd2, dd2 / (2 * np.maximum(dist, 1e-300)), np.sqrt(dd2)) / sigma
        ddist = relk * sigma
    relk = relk + 4 * uexp(prec)
    if split_product(prec, m, deriv):
        relk = relk + 3 * USPLIT[prec]
    if same is not None and same:
        np.fill_diagonal(relk, 0.0)                        # K_ii = 1 exactly
    if not deriv:
        A = relk * K
        if prec == 5 and split_product(prec, m, deriv):
            A = A + 2.0 ** -25                             # fp16 subnormal range of the K parts
        return A, K
    Kd = o.kernel_dsigma_matrix(Xr, Xc, kind, sigma)
    if kind == o.RBF:
        A = np.abs(Kd) * relk + K * dd2 / sigma ** 3
    else:
        A = np.abs(Kd) * relk + K * ddist / sigma ** 2
    return 4 * A, Kd


def bound_from(A, K, V, prec, m, deriv=0):
    """Elementwise bound on |GPU K V - oracle K V| from the per-pair entry bound A and
    the exact matrix K.

    V >= 0: the worst case, sum_j A_ij V_j, plus the accumulation term.
    V with random signs: the entry errors e_ij V_j of one output have symmetric signs
    and magnitudes at most A_ij |V_j|, so by Hoeffding's inequality their sum exceeds
    8 sqrt(sum_j (A_ij V_j)^2) with probability below 2 exp(-32) (the smaller of this
    and the worst case is taken); the partial sums of a
    random-sign series stay near sqrt(j) times a term, so their rounding adds O(u)
    |K| |V| rather than sqrt(n_c) u |K| |V|: 16 u |K| |V|."""
    absV = np.abs(V)
    nc = V.shape[0]
    if np.any(V < 0):
        # the worst case stays valid too and is the smaller one for a few terms
        ent = np.minimum(A @ absV, 8.0 * np.sqrt((A * A) @ (absV * absV)))
        tol = ent + 16 * uacc(prec) * (np.abs(K) @ absV)
    else:
        tol = A @ absV + (8 * math.sqrt(nc) + 16) * uacc(prec) * (np.abs(K) @ absV)
    if prec == 5 and split_product(prec, m, deriv):
        # V split into fp16 parts after scaling its column to [0.5, 1): error 2^-23 of
        # the column's power-of-two scale
        tol = tol + 2.0 ** -22 * absV.max(0)[None, :] * np.abs(K).sum(1)[:, None]
    return tol + 1e-300


def product_bound(Xr, Xc, V, kind, sigma, prec, deriv=0, same=None):
    """Elementwise bound on |GPU K V - oracle K V| (see bound_from)."""
    m = V.shape[1]
    A, K = entry_abs_bound(Xr, Xc, kind, sigma, prec, m, deriv, same)
    return bound_from(A, K, V, prec, m, deriv)


def guard(tol, ref):
    """Largest tolerance over largest |reference| of one case."""
    return float(np.max(tol) / max(float(np.max(np.abs(ref))), 1e-300))
