// Block PCG (O'Leary) for the batched solve: the nrhs right-hand sides of one
// lambda form one block of s = nrhs columns that shares a block Krylov space, and all
// active blocks share each kernel product.  Included by api.hip inside its anonymous
// namespace after solve_impl.h (uses SolvePlan, Slot-free host state and
// apply_precond_or_copy defined there).
//
// Per iteration and active group g (P, W, R, Z its n x s column blocks):
//   W = (K + lambda_g I) P;  alpha = (P^T W)^{-1} (R^T Z);  x64 += P alpha;  R -= W alpha
//   Z = M^{-1} R;  beta = (R^T Z)_old^{-1} (R^T Z);  P = Z + P beta
// The s x s systems are solved on the host by Cholesky.  A group stops when every
// column meets the tolerance (table tab:rlaopt-pcg-stopping, per right-hand side).
//
// Low precision (float32 vectors, FP32 / split products): the iterate is accumulated in
// float64, and groups are refined in cycles as the column solver's mode 1: when a
// group's worst recursive residual has fallen by its cycle factor, r = b - (K +
// lambda I) x64 is recomputed in float64 for the whole group, which is accepted when
// every column's true residual meets tol, and otherwise restarts (P = Z).  A Cholesky
// failure (the block lost rank) restarts the group the same way; two in a row end it
// with NYS_ENOTPD.  A later cycle's factor is the true-residual reduction the previous
// one achieved (at least refine_reduction, at most 0.5).  The first cycle's factor is
// at least kap1 / lambda, kap1 the largest first-cycle drift times lambda seen so far
// (the drift of a cycle that starts from x = 0 scales as 1 / lambda), so a group whose
// first cycle would stall on drift ends it where the drift is reached.
#pragma once

struct BlockPlan {
  double *G = nullptr;       // groups x s x s (device): P^T W, then R^T Z
  double *C = nullptr;       // groups x s x s (device): alpha or beta
  double *part = nullptr;    // gemm_tn partial sums
  int splits = 1;
};
void plan_block(BlockPlan &b, int64_t n, int m, Arena &ws) {
  const int s = std::min(std::max(m, 1), block_max_s());
  const int groups = std::max(1, m / s + 1);
  b.splits = gemm_tn_splits(n, s, s);
  b.G = ws.take<double>((size_t)groups * s * s);
  b.C = ws.take<double>((size_t)groups * s * s);
  b.part = ws.take<double>((size_t)b.splits * s * s);
}

// Solve A X = Bm in place for a symmetric positive definite s x s A (row-major,
// symmetrised first) by Cholesky of the unit-diagonal D A D, D = diag(A)^-1/2: the
// columns of a block converge at different rates, so the diagonal of A can span many
// orders of magnitude, and the pivot test must not depend on that scaling.  Returns
// false when a scaled pivot falls below 1e-14 (the block has lost rank).
inline bool chol_solve_host(std::vector<double> &A, double *Bm, int s) {
  std::vector<double> dsc(s);
  for (int i = 0; i < s; ++i) {
    const double a = A[i * s + i];
    if (!(a > 0.0) || !std::isfinite(a)) return false;
    dsc[i] = 1.0 / std::sqrt(a);
  }
  for (int i = 0; i < s; ++i)
    for (int j = 0; j <= i; ++j) {
      const double v = 0.5 * (A[i * s + j] + A[j * s + i]) * dsc[i] * dsc[j];
      A[i * s + j] = A[j * s + i] = v;
    }
  for (int j = 0; j < s; ++j) {
    double d = A[j * s + j];
    for (int k = 0; k < j; ++k) d -= A[j * s + k] * A[j * s + k];
    if (!(d > 1e-14) || !std::isfinite(d)) return false;
    const double ljj = std::sqrt(d);
    A[j * s + j] = ljj;
    for (int i = j + 1; i < s; ++i) {
      double v = A[i * s + j];
      for (int k = 0; k < j; ++k) v -= A[i * s + k] * A[j * s + k];
      A[i * s + j] = v / ljj;
    }
  }
  // (D A D) Y = D Bm, X = D Y
  for (int c = 0; c < s; ++c) {
    for (int i = 0; i < s; ++i) {          // L y = D b
      double v = Bm[i * s + c] * dsc[i];
      for (int k = 0; k < i; ++k) v -= A[i * s + k] * Bm[k * s + c];
      Bm[i * s + c] = v / A[i * s + i];
    }
    for (int i = s - 1; i >= 0; --i) {     // L^T y' = y
      double v = Bm[i * s + c];
      for (int k = i + 1; k < s; ++k) v -= A[k * s + i] * Bm[k * s + c];
      Bm[i * s + c] = v / A[i * s + i];
    }
    for (int i = 0; i < s; ++i) Bm[i * s + c] *= dsc[i];
  }
  return true;
}

template <class T, class Op>
int32_t solve_blocks(Op &op, int64_t n, const double *B, int nrhs, const double *lambdas, int nlam,
                     const nys_precond *P, const nys_pcg_opts &o, double *Xsol, nys_col_info *info, SolvePlan &sp,
                     BlockPlan &bp, hipStream_t s) {
  const int S = nrhs, mtot = nlam * nrhs;
  const bool lowp = sp.lowp;
  const double tol = o.tol;
  const int max_refs = o.max_refinements > 0 ? o.max_refinements : 50;
  const double delta0 = o.refine_reduction > 0.0 ? std::min(o.refine_reduction, 0.5) : 0.0;
  const bool verbose = std::getenv("NYS_VERBOSE") != nullptr;
  T *R = reinterpret_cast<T *>(sp.R), *Z = reinterpret_cast<T *>(sp.Z), *Pd = reinterpret_cast<T *>(sp.P);
  T *W = reinterpret_cast<T *>(sp.W), *Sp = reinterpret_cast<T *>(sp.Spare);
  // the iterate, always float64: the float64 vector buffer or the refinement copy
  double *X64 = lowp ? sp.X64 : reinterpret_cast<double *>(sp.X);
  double *Sp64 = lowp ? sp.Spare64 : nullptr;   // float64 spare of the refinement (low precision)
  double *R64 = sp.R64;
  if (!X64 || !Sp || (lowp && (!R64 || !Sp64))) {
    set_error("nyspcg_solve: block PCG workspace planned without its float64 buffers");
    return NYS_EINVAL;
  }

  NYS_RETURN_IF(op.prepare(s));

  struct Group {
    int g = 0;                  // lambda index
    double lam = 0.0;
    double rstart = 1.0, delta = 0.0;
    int iters = 0, refs = 0, fails = 0;
    bool restart = true;
    std::vector<double> RZ;     // s x s
  };
  std::vector<Group> gr(nlam);
  for (int g = 0; g < nlam; ++g) {
    gr[g].g = g;
    gr[g].lam = lambdas[g];
    gr[g].delta = delta0;
    gr[g].RZ.assign((size_t)S * S, 0.0);
  }
  for (int c = 0; c < mtot; ++c) info[c] = nys_col_info{0, 0, NYS_NOT_CONVERGED, 0, 1.0, -1.0};
  int ga = nlam;                // active groups, slot q holds gr[q]
  std::vector<int> ih(mtot);
  std::vector<double> dh(mtot), bb(mtot), rel(mtot), rt(mtot);
  auto ma = [&]() { return ga * S; };
  auto upload_slots = [&]() -> int32_t {
    for (int q = 0; q < ga; ++q)
      for (int j = 0; j < S; ++j) {
        ih[q * S + j] = j;
        dh[q * S + j] = gr[q].lam;
      }
    if (ga == 0) return NYS_OK;
    NYS_CHECK_HIP(hipMemcpyAsync(sp.bcol, ih.data(), sizeof(int) * ma(), hipMemcpyHostToDevice, s));
    NYS_CHECK_HIP(hipMemcpyAsync(sp.lam, dh.data(), sizeof(double) * ma(), hipMemcpyHostToDevice, s));
    NYS_CHECK_HIP(hipStreamSynchronize(s));
    return NYS_OK;
  };
  NYS_RETURN_IF(upload_slots());
  NYS_RETURN_IF(init_rhs<T>(B, nrhs, sp.bcol, R, Z, n, mtot, s));          // Z: scratch zero
  NYS_RETURN_IF(launch_fill(X64, 0.0, n * (int64_t)mtot, s));
  // P starts at zero: the first update is P = Z + P 0, which must not meet NaN garbage
  if constexpr (sizeof(T) == sizeof(float))
    NYS_RETURN_IF(launch_fill_f(reinterpret_cast<float *>(Pd), 0.0f, n * (int64_t)mtot, s));
  else
    NYS_RETURN_IF(launch_fill(reinterpret_cast<double *>(Pd), 0.0, n * (int64_t)mtot, s));
  NYS_RETURN_IF(colred<T>(0, R, R, nullptr, nullptr, n, mtot, nullptr, sp.red, s));
  NYS_RETURN_IF(colfinal(sp.red, n, mtot, 0, sp.tmpc, nullptr, nullptr, nullptr, nullptr, s));
  NYS_CHECK_HIP(hipMemcpyAsync(bb.data(), sp.tmpc, sizeof(double) * mtot, hipMemcpyDeviceToHost, s));
  NYS_CHECK_HIP(hipStreamSynchronize(s));
  for (int c = 0; c < mtot; ++c)
    if (!std::isfinite(bb[c])) {
      set_error("nyspcg_solve: NaN or Inf in the right-hand side");
      return NYS_ENUMERIC;
    }
  // |b| per (group slot, column); groups keep their original lambda index in gr[q].g
  auto bnorm = [&](int q, int j) { return bb[gr[q].g * S + j]; };

  // write the listed group slots' iterates to Xsol and drop them
  auto finish_and_compact = [&](const std::vector<int> &done) -> int32_t {
    if (done.empty()) return NYS_OK;
    std::vector<int> slots, orig, keep, keepg;
    std::vector<char> isdone(ga, 0);
    for (int q : done) isdone[q] = 1;
    for (int q : done)
      for (int j = 0; j < S; ++j) {
        slots.push_back(q * S + j);
        orig.push_back(gr[q].g * S + j);
      }
    NYS_CHECK_HIP(hipMemcpyAsync(sp.idx, slots.data(), sizeof(int) * slots.size(), hipMemcpyHostToDevice, s));
    NYS_CHECK_HIP(hipMemcpyAsync(sp.idx2, orig.data(), sizeof(int) * orig.size(), hipMemcpyHostToDevice, s));
    NYS_RETURN_IF(scatter_sol<double>(X64, nullptr, ma(), sp.idx, sp.idx2, (int)slots.size(), Xsol, mtot, n, s));
    for (int q = 0; q < ga; ++q)
      if (!isdone[q]) {
        keepg.push_back(q);
        for (int j = 0; j < S; ++j) keep.push_back(q * S + j);
      }
    const int mn = (int)keep.size();
    if (mn > 0) {
      // W is recomputed every iteration, so it serves as the rotating spare of the
      // vectors in the solve's precision; the float64 iterate rotates through the
      // float64 spare (low precision) or through W too (float64 solves)
      NYS_CHECK_HIP(hipMemcpyAsync(sp.idx, keep.data(), sizeof(int) * mn, hipMemcpyHostToDevice, s));
      NYS_RETURN_IF(gather_cols<T>(R, ma(), sp.idx, mn, W, n, s));
      std::swap(R, W);
      NYS_RETURN_IF(gather_cols<T>(Pd, ma(), sp.idx, mn, W, n, s));
      std::swap(Pd, W);
      NYS_RETURN_IF(gather_cols<T>(Z, ma(), sp.idx, mn, W, n, s));
      std::swap(Z, W);
      if (lowp) {
        NYS_RETURN_IF(gather_cols<double>(X64, ma(), sp.idx, mn, Sp64, n, s));
        std::swap(X64, Sp64);
      } else {
        double *w64 = reinterpret_cast<double *>(W);
        NYS_RETURN_IF(gather_cols<double>(X64, ma(), sp.idx, mn, w64, n, s));
        std::swap(X64, w64);
        W = reinterpret_cast<T *>(w64);
      }
    }
    std::vector<Group> ng;
    for (int q : keepg) ng.push_back(gr[q]);
    for (size_t q = 0; q < ng.size(); ++q) gr[q] = ng[q];
    ga = (int)ng.size();
    NYS_CHECK_HIP(hipStreamSynchronize(s));
    return upload_slots();
  };

  // float64 true residual of the listed group slots (low precision: R replaced by it)
  auto true_residual = [&](const std::vector<int> &qs) -> int32_t {
    std::vector<int> cols, bcs;
    std::vector<double> ls;
    for (int q : qs)
      for (int j = 0; j < S; ++j) {
        cols.push_back(q * S + j);
        bcs.push_back(j);
        ls.push_back(gr[q].lam);
      }
    const int ns = (int)cols.size();
    NYS_CHECK_HIP(hipMemcpyAsync(sp.idx, cols.data(), sizeof(int) * ns, hipMemcpyHostToDevice, s));
    NYS_CHECK_HIP(hipMemcpyAsync(sp.bcol2, bcs.data(), sizeof(int) * ns, hipMemcpyHostToDevice, s));
    NYS_CHECK_HIP(hipMemcpyAsync(sp.lam2, ls.data(), sizeof(double) * ns, hipMemcpyHostToDevice, s));
    NYS_RETURN_IF(gather_cols<double>(X64, ma(), sp.idx, ns, Sp64, n, s));
    NYS_RETURN_IF(op.apply64(Sp64, ns, ns, R64, ns, s));
    NYS_RETURN_IF(residual64(B, nrhs, sp.bcol2, sp.lam2, Sp64, R64, nullptr, n, ns, s));
    if (lowp) NYS_RETURN_IF(scatter_cols_d2f(R64, ns, sp.idx, reinterpret_cast<float *>(R), ma(), n, s));
    NYS_RETURN_IF(colred<double>(0, R64, R64, nullptr, nullptr, n, ns, nullptr, sp.red, s));
    NYS_RETURN_IF(colfinal(sp.red, n, ns, 0, sp.tmpc, nullptr, nullptr, nullptr, nullptr, s));
    NYS_CHECK_HIP(hipMemcpyAsync(rt.data(), sp.tmpc, sizeof(double) * ns, hipMemcpyDeviceToHost, s));
    NYS_CHECK_HIP(hipStreamSynchronize(s));
    for (int t = 0; t < ns; ++t) {
      const int q = cols[t] / S, j = cols[t] % S;
      const double b2 = bnorm(q, j);
      rt[t] = b2 > 0.0 ? std::sqrt(std::max(rt[t], 0.0) / b2) : 0.0;
    }
    return NYS_OK;
  };

  // a block with a zero right-hand side among non-zero ones is rank deficient from the
  // start; a group whose columns are all zero ends at once
  for (int q = 0; q < ga; ++q) {
    int zeros = 0;
    for (int j = 0; j < S; ++j) zeros += bnorm(q, j) == 0.0;
    if (zeros > 0 && zeros < S) {
      set_error("nyspcg_solve: block PCG needs the right-hand sides of a lambda all non-zero (or all zero)");
      return NYS_EINVAL;
    }
  }
  {
    std::vector<int> done;
    for (int q = 0; q < ga; ++q) {
      bool zero = true;
      for (int j = 0; j < S; ++j) zero = zero && bnorm(q, j) == 0.0;
      if (zero) {
        done.push_back(q);
        for (int j = 0; j < S; ++j) {
          nys_col_info &ci = info[gr[q].g * S + j];
          ci.status = NYS_OK;
          ci.relres_recursive = 0.0;
          ci.relres_true = 0.0;
        }
      }
    }
    NYS_RETURN_IF(finish_and_compact(done));
  }

  std::vector<double> Gh, Ch;
  // First-cycle drift constant: over the groups refined so far, the largest
  // (true - recursive) relative residual at the end of their first cycle times their
  // lambda.  The first cycle starts from x = 0, and its drift grows with the iterate,
  // whose norm reaches |b| / lambda in the directions K barely damps, so the drift a
  // first cycle accumulates scales as 1 / lambda.  Large lambdas converge first; a
  // group still in its first cycle ends it once its recursive residual reaches the
  // drift predicted for its lambda (iterating further lowers only the recursive
  // residual).
  double kap1 = 0.0;
  int iter = 0;
  bool breakdown = false;
  while (ga > 0) {
    // preconditioned residual; for restarted groups P = Z and R^T Z anew, else beta
    NYS_RETURN_IF(apply_precond_or_copy<T>(P, sp, R, ma(), Z, n, s));
    Gh.assign((size_t)ga * S * S, 0.0);
    for (int q = 0; q < ga; ++q)
      NYS_RETURN_IF(gemm_tn_to_double<T>(R + q * S, ma(), Z + q * S, ma(), n, S, S, bp.G + (size_t)q * S * S, S,
                                         bp.part, bp.splits, s));
    NYS_CHECK_HIP(hipMemcpyAsync(Gh.data(), bp.G, sizeof(double) * Gh.size(), hipMemcpyDeviceToHost, s));
    NYS_CHECK_HIP(hipStreamSynchronize(s));
    Ch.assign((size_t)ga * S * S, 0.0);
    for (int q = 0; q < ga; ++q) {
      Group &G = gr[q];
      std::vector<double> RZn(Gh.begin() + (size_t)q * S * S, Gh.begin() + (size_t)(q + 1) * S * S);
      if (!G.restart) {
        std::vector<double> A = G.RZ;
        std::vector<double> beta = RZn;
        if (chol_solve_host(A, beta.data(), S)) {
          std::copy(beta.begin(), beta.end(), Ch.begin() + (size_t)q * S * S);
        } else {
          G.restart = true;       // beta = 0: P = Z
          if (verbose) {
            std::fprintf(stderr, "[nys] block iter %d lambda %.4g: R^T Z lost rank, P = Z\n", iter, G.lam);
            std::fflush(stderr);
          }
        }
      }
      G.RZ = RZn;
    }
    NYS_CHECK_HIP(hipMemcpyAsync(bp.C, Ch.data(), sizeof(double) * Ch.size(), hipMemcpyHostToDevice, s));
    NYS_RETURN_IF((blk_apply<T, T>(2, Pd, bp.C, S, ga, ma(), Sp, Z, n, s)));   // Sp = Z + P beta
    std::swap(Pd, Sp);
    for (int q = 0; q < ga; ++q) gr[q].restart = false;

    // W = (K + lambda I) P
    NYS_RETURN_IF(op.apply(Pd, ma(), ma(), W, ma(), s));
    NYS_RETURN_IF(colred<T>(1, Pd, W, nullptr, nullptr, n, ma(), sp.lam, sp.red, s));
    for (int q = 0; q < ga; ++q)
      NYS_RETURN_IF(gemm_tn_to_double<T>(Pd + q * S, ma(), W + q * S, ma(), n, S, S, bp.G + (size_t)q * S * S, S,
                                         bp.part, bp.splits, s));
    NYS_CHECK_HIP(hipMemcpyAsync(Gh.data(), bp.G, sizeof(double) * (size_t)ga * S * S, hipMemcpyDeviceToHost, s));
    NYS_CHECK_HIP(hipStreamSynchronize(s));
    std::vector<int> failed;
    for (int q = 0; q < ga; ++q) {
      std::vector<double> A(Gh.begin() + (size_t)q * S * S, Gh.begin() + (size_t)(q + 1) * S * S);
      std::vector<double> alpha = gr[q].RZ;
      if (chol_solve_host(A, alpha.data(), S)) {
        std::copy(alpha.begin(), alpha.end(), Ch.begin() + (size_t)q * S * S);
      } else {
        std::fill(Ch.begin() + (size_t)q * S * S, Ch.begin() + (size_t)(q + 1) * S * S, 0.0);
        failed.push_back(q);
      }
    }
    NYS_CHECK_HIP(hipMemcpyAsync(bp.C, Ch.data(), sizeof(double) * (size_t)ga * S * S, hipMemcpyHostToDevice, s));
    NYS_RETURN_IF((blk_apply<T, double>(0, Pd, bp.C, S, ga, ma(), X64, nullptr, n, s)));   // x += P alpha
    NYS_RETURN_IF((blk_apply<T, T>(1, W, bp.C, S, ga, ma(), R, nullptr, n, s)));          // R -= W alpha
    ++iter;
    NYS_RETURN_IF(colred<T>(0, R, R, nullptr, nullptr, n, ma(), nullptr, sp.red, s));
    NYS_RETURN_IF(colfinal(sp.red, n, ma(), 0, sp.tmpc, nullptr, nullptr, nullptr, nullptr, s));
    NYS_CHECK_HIP(hipMemcpyAsync(rel.data(), sp.tmpc, sizeof(double) * ma(), hipMemcpyDeviceToHost, s));
    NYS_CHECK_HIP(hipStreamSynchronize(s));

    std::vector<int> done, refine_q;
    std::vector<char> isfailed(ga, 0);
    for (int q : failed) isfailed[q] = 1;
    double lo = 1e300, hi = 0.0;
    for (int q = 0; q < ga; ++q) {
      Group &G = gr[q];
      G.iters += 1;
      double worst = 0.0;
      bool finite = true;
      for (int j = 0; j < S; ++j) {
        const double b2 = bnorm(q, j);
        const double r = b2 > 0.0 ? std::sqrt(std::max(rel[q * S + j], 0.0) / b2) : 0.0;
        finite = finite && std::isfinite(r);
        rel[q * S + j] = r;
        worst = std::max(worst, r);
        lo = std::min(lo, r);
        hi = std::max(hi, r);
        nys_col_info &ci = info[G.g * S + j];
        ci.iters = G.iters;
        ci.relres_recursive = r;
      }
      if (!finite) {
        breakdown = true;
        for (int j = 0; j < S; ++j) info[G.g * S + j].status = NYS_ENUMERIC;
        done.push_back(q);
        continue;
      }
      const bool capped = G.iters >= o.max_iters;
      if (isfailed[q]) {
        G.fails += 1;
        if (G.fails >= 2) {
          breakdown = true;
          for (int j = 0; j < S; ++j) info[G.g * S + j].status = NYS_ENOTPD;
          done.push_back(q);
          continue;
        }
      } else {
        G.fails = 0;
      }
      if (!lowp) {
        if (worst <= tol) {
          for (int j = 0; j < S; ++j) info[G.g * S + j].status = NYS_OK;
          done.push_back(q);
        } else if (capped) {
          done.push_back(q);
        } else if (isfailed[q]) {
          G.restart = true;
        }
        continue;
      }
      double delta = G.delta;
      if (delta > 0.0 && G.refs == 0 && kap1 > 0.0 && G.lam > 0.0) delta = std::max(delta, std::min(0.5, kap1 / G.lam));
      double thr = delta > 0.0 ? delta * G.rstart : tol;
      if (G.delta > 0.0 && thr < 10.0 * 0.3 * tol) thr = 0.3 * tol;
      if (worst <= thr || capped || isfailed[q]) {
        refine_q.push_back(q);
        if (verbose) {
          std::fprintf(stderr, "[nys] block iter %d lambda %.4g (%d its): refine at recursive %.3e%s\n", iter,
                       G.lam, G.iters, worst, isfailed[q] ? " (P^T W lost rank)" : (capped ? " (cap)" : ""));
          std::fflush(stderr);
        }
      }
    }
    if (verbose && (iter % 10 == 0 || iter == 1)) {
      std::fprintf(stderr, "[nys] block iter %d groups %d relres [%.3e, %.3e]\n", iter, ga, lo, hi);
      std::fflush(stderr);
    }
    if (!refine_q.empty()) {
      NYS_RETURN_IF(true_residual(refine_q));
      double worst_all = 0.0;
      for (size_t t = 0; t < refine_q.size(); ++t) {
        const int q = refine_q[t];
        Group &G = gr[q];
        const bool first = G.refs == 0;
        G.refs += 1;
        double worst = 0.0, drift = 0.0;
        for (int j = 0; j < S; ++j) {
          const double r = rt[t * S + j];
          worst = std::max(worst, r);
          drift = std::max(drift, r - rel[q * S + j]);
          nys_col_info &ci = info[G.g * S + j];
          ci.refinements = G.refs;
          ci.relres_true = r;
        }
        worst_all = std::max(worst_all, worst);
        if (first && G.lam > 0.0) kap1 = std::max(kap1, drift / G.rstart * G.lam);
        if (verbose) {
          std::fprintf(stderr, "[nys] block iter %d lambda %.4g: true %.3e (cycle factor was %.3e)\n", iter, G.lam,
                       worst, G.delta);
          std::fflush(stderr);
        }
        if (worst <= tol) {
          for (int j = 0; j < S; ++j) info[G.g * S + j].status = NYS_OK;
          done.push_back(q);
          continue;
        }
        if (G.iters >= o.max_iters || G.refs >= max_refs) {
          done.push_back(q);
          continue;
        }
        const double g = worst / G.rstart;
        G.rstart = worst;
        if (delta0 > 0.0) G.delta = std::max(delta0, std::min(0.5, g));
        G.restart = true;
      }
      if (verbose) {
        std::fprintf(stderr, "[nys] block iter %d refined %zu of %d groups, max true relres %.3e\n", iter,
                     refine_q.size(), ga, worst_all);
        std::fflush(stderr);
      }
    }
    std::sort(done.begin(), done.end());
    done.erase(std::unique(done.begin(), done.end()), done.end());
    NYS_RETURN_IF(finish_and_compact(done));
  }
  if (o.check_true && !lowp) {
    // float64 true residuals of the solution (one product over all columns)
    NYS_RETURN_IF(op.apply64(Xsol, mtot, mtot, R64, mtot, s));
    std::vector<int> bc(mtot);
    std::vector<double> lm(mtot);
    for (int c = 0; c < mtot; ++c) {
      bc[c] = c % nrhs;
      lm[c] = lambdas[c / nrhs];
    }
    NYS_CHECK_HIP(hipMemcpyAsync(sp.bcol2, bc.data(), sizeof(int) * mtot, hipMemcpyHostToDevice, s));
    NYS_CHECK_HIP(hipMemcpyAsync(sp.lam2, lm.data(), sizeof(double) * mtot, hipMemcpyHostToDevice, s));
    NYS_RETURN_IF(residual64(B, nrhs, sp.bcol2, sp.lam2, Xsol, R64, nullptr, n, mtot, s));
    NYS_RETURN_IF(colred<double>(0, R64, R64, nullptr, nullptr, n, mtot, nullptr, sp.red, s));
    NYS_RETURN_IF(colfinal(sp.red, n, mtot, 0, sp.tmpc, nullptr, nullptr, nullptr, nullptr, s));
    std::vector<double> t2(mtot);
    NYS_CHECK_HIP(hipMemcpyAsync(t2.data(), sp.tmpc, sizeof(double) * mtot, hipMemcpyDeviceToHost, s));
    NYS_CHECK_HIP(hipStreamSynchronize(s));
    for (int c = 0; c < mtot; ++c) info[c].relres_true = bb[c] > 0 ? std::sqrt(std::max(t2[c], 0.0) / bb[c]) : 0.0;
  }
  if (breakdown) {
    for (int c = 0; c < mtot; ++c)
      if (info[c].status == NYS_ENOTPD || info[c].status == NYS_ENUMERIC) {
        set_error("nyspcg_solve: block PCG lost rank or met a non-finite value in a group");
        return info[c].status;
      }
  }
  for (int c = 0; c < mtot; ++c)
    if (info[c].status != NYS_OK) return NYS_NOT_CONVERGED;
  return NYS_OK;
}
