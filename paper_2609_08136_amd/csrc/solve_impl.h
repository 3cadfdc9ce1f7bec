// The PCG driver over a block of independent columns.  Included by api.hip
// inside its anonymous namespace (uses SolvePlan and apply_precond_or_copy
// defined there); the operator is a template argument (the kernel matrix, or the
// ridge normal matrix).
//
// Columns are kept compacted: slot q < ma holds original column sl[q].orig;
// finished columns are written to Xsol and removed, so the kernel product
// always runs on the active columns only.
//
// Low-precision solves (FP32 / BF16X3 products, float32 vectors) accept a
// column only on its float64 true residual (eq. experiment-relative-residual).
// The recursion of a low-precision product solves a perturbed system, so its
// residual drifts from the true one by about |E x| (E the product error).
// Refinement therefore works in cycles: a column is refined (x64 += x,
// r = b - (K + lambda I) x64 in float64, replacing the recursive residual) once
// its recursive residual has fallen by its cycle factor delta since the last
// refinement; delta follows the reduction the previous cycle actually achieved,
// so iterations are not spent below the precision floor.  Mode 1 restarts the
// recurrence (p = z) after every refinement; mode 0 keeps the search direction
// when the replaced residual is within 25% of the recursive one.  Mode 2 measures
// the drift q = |r_true - r_rec| / |r_rec| at each refinement, keeps p unless
// q > 0.5, and rescales the next cycle factor by q / 0.1: the drift accumulated
// over a cycle grows with the reduction the cycle makes, so cycles are sized to
// end with about a 10% replacement, which the recurrence absorbs without a restart.
#pragma once

struct Slot {
  int orig = 0, bcol = 0;
  double lam = 0.0, bb = 0.0;   // lambda, |b|^2
  double rstart = 1.0;          // relative true residual at the start of the cycle
  double rmin = 1e300;          // smallest recursive residual of the cycle
  double delta = 0.0;           // cycle factor
  int iters = 0, refs = 0, restart = 0;
};

// Op supplies the operator K of (K + lambda I) on n-vectors: prepare(s) once, then
// apply(V, m, ldv, Out, ldo, s) (Out = K V in the solve's precision) and apply64
// (the same in float64, for refinement residuals and the true-residual check).
template <class T, class Op>
int32_t solve_columns(Op &op, int64_t n, const double *B, int nrhs,
                      const double *lambdas, int nlam, const nys_precond *P, const nys_pcg_opts &o,
                      double *Xsol, nys_col_info *info, SolvePlan &sp, hipStream_t s) {
  const int mtot = nlam * nrhs;
  const int prec = sp.prec;
  const bool lowp = sp.lowp;
  const bool refine = lowp && o.refine_every >= 0;
  const int max_refs = o.max_refinements > 0 ? o.max_refinements : 50;
  const double join = o.refine_join > 0.0 ? o.refine_join : 3.0;
  const double tol = o.tol;
  const double delta0 = o.refine_reduction > 0.0 ? std::min(o.refine_reduction, 0.5) : 0.0;
  const bool verbose = std::getenv("NYS_VERBOSE") != nullptr;
  T *X = reinterpret_cast<T *>(sp.X), *R = reinterpret_cast<T *>(sp.R), *Z = reinterpret_cast<T *>(sp.Z);
  T *Pd = reinterpret_cast<T *>(sp.P), *W = reinterpret_cast<T *>(sp.W), *Sp = reinterpret_cast<T *>(sp.Spare);
  double *X64 = sp.X64, *R64 = sp.R64, *Sp64 = sp.Spare64;

  NYS_RETURN_IF(op.prepare(s));

  std::vector<Slot> sl(mtot);
  std::vector<int> ih(mtot);
  std::vector<double> dh(mtot);
  for (int c = 0; c < mtot; ++c) {
    sl[c].orig = c;
    sl[c].bcol = c % nrhs;
    sl[c].lam = lambdas[c / nrhs];
    sl[c].delta = delta0;
    info[c] = nys_col_info{0, 0, NYS_NOT_CONVERGED, 0, 1.0, -1.0};
  }
  int ma = mtot;
  // per-slot device arrays (bcol, lambda) from the host slots
  auto upload_slots = [&]() -> int32_t {
    if (ma == 0) return NYS_OK;
    for (int q = 0; q < ma; ++q) {
      ih[q] = sl[q].bcol;
      dh[q] = sl[q].lam;
    }
    NYS_CHECK_HIP(hipMemcpyAsync(sp.bcol, ih.data(), sizeof(int) * ma, hipMemcpyHostToDevice, s));
    NYS_CHECK_HIP(hipMemcpyAsync(sp.lam, dh.data(), sizeof(double) * ma, hipMemcpyHostToDevice, s));
    NYS_CHECK_HIP(hipStreamSynchronize(s));
    return NYS_OK;
  };
  NYS_RETURN_IF(upload_slots());
  NYS_CHECK_HIP(hipMemsetAsync(sp.restart, 0, sizeof(int) * mtot, s));
  NYS_CHECK_HIP(hipMemsetAsync(sp.flag, 0, sizeof(int) * mtot, s));
  NYS_RETURN_IF(init_rhs<T>(B, nrhs, sp.bcol, R, X, n, mtot, s));
  if (X64) NYS_RETURN_IF(launch_fill(X64, 0.0, n * (int64_t)mtot, s));
  NYS_RETURN_IF(colred<T>(0, R, R, nullptr, nullptr, n, mtot, nullptr, sp.red, s));
  NYS_RETURN_IF(colfinal(sp.red, n, mtot, 0, sp.tmpc, nullptr, nullptr, nullptr, nullptr, s));
  std::vector<double> bb(mtot);
  NYS_CHECK_HIP(hipMemcpyAsync(bb.data(), sp.tmpc, sizeof(double) * mtot, hipMemcpyDeviceToHost, s));
  NYS_CHECK_HIP(hipStreamSynchronize(s));
  for (int c = 0; c < mtot; ++c) {
    if (!std::isfinite(bb[c])) {
      set_error("nyspcg_solve: NaN or Inf in the right-hand side");
      return NYS_ENUMERIC;
    }
    sl[c].bb = bb[c];
  }

  std::vector<double> rr_h(mtot), rt_h(mtot), gap_h(mtot);
  const bool drift = o.refine_mode == 2;
  std::vector<int> flag_h(mtot);
  bool breakdown = false;

  // keep slots kp (in order): gather the device state, select the host slots
  auto compact = [&](const std::vector<int> &kp) -> int32_t {
    const int mn = (int)kp.size();
    if (mn == ma) return NYS_OK;
    if (mn > 0) {
      NYS_CHECK_HIP(hipMemcpyAsync(sp.idx, kp.data(), sizeof(int) * mn, hipMemcpyHostToDevice, s));
      NYS_RETURN_IF(gather_cols<T>(X, ma, sp.idx, mn, Sp, n, s));
      std::swap(X, Sp);
      NYS_RETURN_IF(gather_cols<T>(R, ma, sp.idx, mn, Sp, n, s));
      std::swap(R, Sp);
      NYS_RETURN_IF(gather_cols<T>(Pd, ma, sp.idx, mn, Sp, n, s));
      std::swap(Pd, Sp);
      if (X64) {
        NYS_RETURN_IF(gather_cols<double>(X64, ma, sp.idx, mn, Sp64, n, s));
        std::swap(X64, Sp64);
      }
      NYS_RETURN_IF(gather_cols<double>(sp.rho, ma, sp.idx, mn, sp.tmpc, 1, s));
      NYS_CHECK_HIP(hipMemcpyAsync(sp.rho, sp.tmpc, sizeof(double) * mn, hipMemcpyDeviceToDevice, s));
    }
    std::vector<Slot> ns(mn);
    for (int q = 0; q < mn; ++q) ns[q] = sl[kp[q]];
    for (int q = 0; q < mn; ++q) sl[q] = ns[q];
    ma = mn;
    return upload_slots();
  };
  // write finished slots to Xsol
  auto finish = [&](const std::vector<int> &slots) -> int32_t {
    if (slots.empty()) return NYS_OK;
    std::vector<int> og(slots.size());
    for (size_t q = 0; q < slots.size(); ++q) og[q] = sl[slots[q]].orig;
    NYS_CHECK_HIP(hipMemcpyAsync(sp.idx, slots.data(), sizeof(int) * slots.size(), hipMemcpyHostToDevice, s));
    NYS_CHECK_HIP(hipMemcpyAsync(sp.idx2, og.data(), sizeof(int) * og.size(), hipMemcpyHostToDevice, s));
    NYS_RETURN_IF(scatter_sol<T>(X, X64, ma, sp.idx, sp.idx2, (int)slots.size(), Xsol, mtot, n, s));
    NYS_CHECK_HIP(hipStreamSynchronize(s));
    return NYS_OK;
  };
  // float64 residual of the listed slots (x64 += x first); relative norms into rt_h
  auto refine_slots = [&](const std::vector<int> &sel) -> int32_t {
    const int ns = (int)sel.size();
    NYS_RETURN_IF(flush_x(reinterpret_cast<float *>(X), X64, n * (int64_t)ma, s));
    if (ns < ma) {
      std::vector<int> bs(ns);
      std::vector<double> ls(ns);
      for (int t = 0; t < ns; ++t) {
        bs[t] = sl[sel[t]].bcol;
        ls[t] = sl[sel[t]].lam;
      }
      NYS_CHECK_HIP(hipMemcpyAsync(sp.idx, sel.data(), sizeof(int) * ns, hipMemcpyHostToDevice, s));
      NYS_CHECK_HIP(hipMemcpyAsync(sp.bcol2, bs.data(), sizeof(int) * ns, hipMemcpyHostToDevice, s));
      NYS_CHECK_HIP(hipMemcpyAsync(sp.lam2, ls.data(), sizeof(double) * ns, hipMemcpyHostToDevice, s));
      NYS_RETURN_IF(gather_cols<double>(X64, ma, sp.idx, ns, Sp64, n, s));
      NYS_RETURN_IF(op.apply64(Sp64, ns, ns, R64, ns, s));
      NYS_RETURN_IF(residual64(B, nrhs, sp.bcol2, sp.lam2, Sp64, R64, nullptr, n, ns, s));
      if (drift) NYS_RETURN_IF(gapnorm<T>(R64, ns, R, ma, sp.idx, n, sp.red, s));
      if (drift) NYS_RETURN_IF(colfinal(sp.red, n, ns, 0, sp.tmpc, nullptr, nullptr, nullptr, nullptr, s));
      if (drift) NYS_CHECK_HIP(hipMemcpyAsync(gap_h.data(), sp.tmpc, sizeof(double) * ns, hipMemcpyDeviceToHost, s));
      NYS_RETURN_IF(scatter_cols_d2f(R64, ns, sp.idx, reinterpret_cast<float *>(R), ma, n, s));
    } else {
      NYS_RETURN_IF(op.apply64(X64, ma, ma, R64, ma, s));
      NYS_RETURN_IF(residual64(B, nrhs, sp.bcol, sp.lam, X64, R64, drift ? nullptr : reinterpret_cast<float *>(R),
                               n, ma, s));
      if (drift) {
        NYS_RETURN_IF(gapnorm<T>(R64, ma, R, ma, nullptr, n, sp.red, s));
        NYS_RETURN_IF(colfinal(sp.red, n, ma, 0, sp.tmpc, nullptr, nullptr, nullptr, nullptr, s));
        NYS_CHECK_HIP(hipMemcpyAsync(gap_h.data(), sp.tmpc, sizeof(double) * ma, hipMemcpyDeviceToHost, s));
        NYS_RETURN_IF(launch_copy_d2f(R64, reinterpret_cast<float *>(R), n * (int64_t)ma, s));
      }
    }
    NYS_RETURN_IF(colred<double>(0, R64, R64, nullptr, nullptr, n, ns, nullptr, sp.red, s));
    NYS_RETURN_IF(colfinal(sp.red, n, ns, 0, sp.tmpc, nullptr, nullptr, nullptr, nullptr, s));
    NYS_CHECK_HIP(hipMemcpyAsync(rt_h.data(), sp.tmpc, sizeof(double) * ns, hipMemcpyDeviceToHost, s));
    NYS_CHECK_HIP(hipStreamSynchronize(s));
    for (int t = 0; t < ns; ++t) {
      rt_h[t] = std::sqrt(std::max(rt_h[t], 0.0) / sl[sel[t]].bb);
      if (drift) gap_h[t] = std::sqrt(std::max(gap_h[t], 0.0) / sl[sel[t]].bb);   // relative to |b|
    }
    return NYS_OK;
  };

  // zero right-hand sides: x = 0 after 0 iterations
  {
    std::vector<int> z, kp;
    for (int c = 0; c < ma; ++c) (sl[c].bb == 0.0 ? z : kp).push_back(c);
    for (int c : z) {
      info[sl[c].orig].status = NYS_OK;
      info[sl[c].orig].relres_recursive = 0.0;
      info[sl[c].orig].relres_true = 0.0;
    }
    NYS_RETURN_IF(finish(z));
    NYS_RETURN_IF(compact(kp));
  }
  if (ma > 0 && o.max_iters > 0) {
    NYS_RETURN_IF(apply_precond_or_copy<T>(P, sp, R, ma, Z, n, s));
    NYS_RETURN_IF(colred<T>(0, R, Z, nullptr, nullptr, n, ma, nullptr, sp.red, s));
    NYS_RETURN_IF(colfinal(sp.red, n, ma, 0, sp.rho, nullptr, nullptr, nullptr, nullptr, s));
    NYS_CHECK_HIP(hipMemcpyAsync(Pd, Z, sizeof(T) * n * ma, hipMemcpyDeviceToDevice, s));
  }

  int iter = 0;
  while (ma > 0 && iter < o.max_iters) {
    ++iter;
    // w = K p + lambda p ; alpha = rho / p^T w
    NYS_RETURN_IF(op.apply(Pd, ma, ma, W, ma, s));
    NYS_RETURN_IF(colred<T>(1, Pd, W, nullptr, nullptr, n, ma, sp.lam, sp.red, s));
    NYS_RETURN_IF(colfinal(sp.red, n, ma, 1, nullptr, sp.rho, sp.ab, nullptr, sp.flag, s));
    // x += alpha p ; r -= alpha w ; rr = r^T r   (low precision: x accumulated in float64)
    NYS_RETURN_IF(colred<T>(X64 ? 3 : 2, Pd, W, X, R, n, ma, sp.ab, sp.red, s, X64));
    NYS_RETURN_IF(colfinal(sp.red, n, ma, 0, sp.rr, nullptr, nullptr, nullptr, nullptr, s));
    NYS_CHECK_HIP(hipMemcpyAsync(rr_h.data(), sp.rr, sizeof(double) * ma, hipMemcpyDeviceToHost, s));
    NYS_CHECK_HIP(hipMemcpyAsync(flag_h.data(), sp.flag, sizeof(int) * ma, hipMemcpyDeviceToHost, s));
    NYS_CHECK_HIP(hipStreamSynchronize(s));

    std::vector<char> conv(ma, 0), stop(ma, 0);
    std::vector<double> rel(ma), thr(ma);
    std::vector<char> dv(ma, 0);
    double lo = 1e300, hi = 0.0;
    bool any_due = false;
    for (int q = 0; q < ma; ++q) {
      Slot &c = sl[q];
      c.iters += 1;
      rel[q] = std::sqrt(std::max(rr_h[q], 0.0) / c.bb);
      info[c.orig].iters = c.iters;
      info[c.orig].relres_recursive = rel[q];
      lo = std::min(lo, rel[q]);
      hi = std::max(hi, rel[q]);
      if (flag_h[q] || !std::isfinite(rel[q])) {
        stop[q] = 1;
        breakdown = true;
        info[c.orig].status = NYS_ENOTPD;
        continue;
      }
      // cycle target: delta times the residual the cycle started from (may lie
      // below tol: acceptance is on the true residual), or tol without cycles
      // The last cycle aims at 0.3 tol (the true residual ends a little above the
      // recursive one); a cycle whose target is within 10x of that becomes the last.
      if (c.delta > 0.0) {
        const double last = 0.3 * tol;
        thr[q] = c.delta * c.rstart;
        if (thr[q] < 10.0 * last) thr[q] = last;
      } else {
        thr[q] = tol;
      }
      // a recursion whose residual grew 100x above its best of the cycle and 10x above
      // the residual the cycle started from has lost its footing: refine (and restart)
      // it now.  (CG residuals are not monotone: smaller excursions are normal.)
      const bool diverging = refine && rel[q] > 100.0 * c.rmin && rel[q] > 10.0 * c.rstart && rel[q] > tol;
      c.rmin = std::min(c.rmin, rel[q]);
      dv[q] = diverging;
      if (diverging) thr[q] = rel[q];
      if (rel[q] <= thr[q]) any_due = true;
      if (!refine && rel[q] <= tol) conv[q] = 1;
    }
    if (verbose && (iter % 10 == 0 || iter == 1)) {
      std::fprintf(stderr, "[nys] iter %d active %d relres [%.3e, %.3e]\n", iter, ma, lo, hi);
      std::fflush(stderr);
    }

    if (refine) {
      std::vector<int> sel;
      const bool periodic = o.refine_every > 0 && iter % o.refine_every == 0;
      for (int q = 0; q < ma; ++q) {
        if (stop[q]) continue;
        const bool capped = sl[q].iters >= o.max_iters;   // report its true residual before it stops
        const bool take = periodic || capped || dv[q] ? true
                        : (o.refine_every > 0 ? rel[q] <= tol : (any_due && rel[q] <= join * thr[q]));
        if (take) sel.push_back(q);
      }
      if (!sel.empty()) {
        NYS_RETURN_IF(refine_slots(sel));
        double worst = 0.0;
        for (int t = 0; t < (int)sel.size(); ++t) {
          const int q = sel[t];
          Slot &c = sl[q];
          const double rt = rt_h[t];
          worst = std::max(worst, rt);
          c.refs += 1;
          info[c.orig].refinements = c.refs;
          info[c.orig].relres_true = rt;
          if (rt <= tol) {
            conv[q] = 1;
            continue;
          }
          const double g = rt / c.rstart;
          c.rstart = rt;
          c.rmin = rt;
          if (drift) {
            // drift relative to the recursive residual it replaced
            const double qd = gap_h[t] / std::max(rel[q], 1e-300);
            if (delta0 > 0.0) c.delta = std::min(0.5, std::max(1e-4, c.delta * std::max(qd, 1e-3) / 0.1));
            c.restart = qd > 0.5 ? 1 : 0;
          } else {
            if (delta0 > 0.0) c.delta = std::max(delta0, std::min(0.5, g));
            // keeping p is only sound when the replacement barely moved the residual
            c.restart = (o.refine_mode == 1 || rt > 1.25 * rel[q] || rt < 0.8 * rel[q]) ? 1 : 0;
          }
          if (c.refs >= max_refs) stop[q] = 1;
        }
        if (verbose) {
          std::fprintf(stderr, "[nys] iter %d refined %zu of %d columns, max true relres %.3e\n", iter,
                       sel.size(), ma, worst);
          std::fflush(stderr);
        }
      }
    }

    // finished columns leave the active set
    std::vector<int> fin, kp;
    for (int q = 0; q < ma; ++q) {
      const bool over = sl[q].iters >= o.max_iters;
      if (conv[q]) info[sl[q].orig].status = NYS_OK;
      if (conv[q] || stop[q] || over) fin.push_back(q);
      else kp.push_back(q);
    }
    if (!fin.empty()) {
      NYS_RETURN_IF(finish(fin));
      NYS_RETURN_IF(compact(kp));
      NYS_CHECK_HIP(hipMemsetAsync(sp.flag, 0, sizeof(int) * std::max(ma, 1), s));
    }
    if (ma == 0) break;
    bool any_restart = false;
    for (int q = 0; q < ma; ++q) {
      ih[q] = sl[q].restart;
      any_restart |= sl[q].restart != 0;
      sl[q].restart = 0;
    }
    if (any_restart) {
      NYS_CHECK_HIP(hipMemcpyAsync(sp.restart, ih.data(), sizeof(int) * ma, hipMemcpyHostToDevice, s));
      NYS_CHECK_HIP(hipStreamSynchronize(s));
    }
    // z = P^{-1} r ; beta = r^T z / rho (0 on restart) ; p = z + beta p
    NYS_RETURN_IF(apply_precond_or_copy<T>(P, sp, R, ma, Z, n, s));
    NYS_RETURN_IF(colred<T>(0, R, Z, nullptr, nullptr, n, ma, nullptr, sp.red, s));
    NYS_RETURN_IF(colfinal(sp.red, n, ma, 2, nullptr, sp.rho, sp.ab, any_restart ? sp.restart : nullptr,
                           nullptr, s));
    NYS_RETURN_IF(p_update<T>(Pd, Z, sp.ab, n, ma, s));
    if (any_restart) NYS_CHECK_HIP(hipMemsetAsync(sp.restart, 0, sizeof(int) * ma, s));
  }
  // columns still active hit the iteration cap
  if (ma > 0) {
    std::vector<int> all(ma);
    for (int q = 0; q < ma; ++q) all[q] = q;
    if (refine && o.max_iters > 0) {
      // report their float64 true residual (refine_slots leaves X zero and x in X64)
      NYS_RETURN_IF(refine_slots(all));
      for (int q = 0; q < ma; ++q) {
        info[sl[q].orig].relres_true = rt_h[q];
        if (rt_h[q] <= tol) info[sl[q].orig].status = NYS_OK;
      }
    } else if (X64) {
      NYS_RETURN_IF(flush_x(reinterpret_cast<float *>(X), X64, n * (int64_t)ma, s));
      NYS_CHECK_HIP(hipMemsetAsync(X, 0, sizeof(T) * n * ma, s));
    }
    NYS_RETURN_IF(finish(all));
  }
  // optional float64 true residual of every column
  if (o.check_true && R64) {
    NYS_RETURN_IF(op.apply64(Xsol, mtot, mtot, R64, mtot, s));
    std::vector<int> bc(mtot);
    std::vector<double> lm(mtot);
    for (int c = 0; c < mtot; ++c) {
      bc[c] = c % nrhs;
      lm[c] = lambdas[c / nrhs];
    }
    NYS_CHECK_HIP(hipMemcpyAsync(sp.bcol, bc.data(), sizeof(int) * mtot, hipMemcpyHostToDevice, s));
    NYS_CHECK_HIP(hipMemcpyAsync(sp.lam, lm.data(), sizeof(double) * mtot, hipMemcpyHostToDevice, s));
    NYS_RETURN_IF(residual64(B, nrhs, sp.bcol, sp.lam, Xsol, R64, nullptr, n, mtot, s));
    NYS_RETURN_IF(colred<double>(0, R64, R64, nullptr, nullptr, n, mtot, nullptr, sp.red, s));
    NYS_RETURN_IF(colfinal(sp.red, n, mtot, 0, sp.tmpc, nullptr, nullptr, nullptr, nullptr, s));
    std::vector<double> rt(mtot);
    NYS_CHECK_HIP(hipMemcpyAsync(rt.data(), sp.tmpc, sizeof(double) * mtot, hipMemcpyDeviceToHost, s));
    NYS_CHECK_HIP(hipStreamSynchronize(s));
    for (int c = 0; c < mtot; ++c)
      info[c].relres_true = bb[c] > 0 ? std::sqrt(std::max(rt[c], 0.0) / bb[c]) : 0.0;
  }
  NYS_CHECK_HIP(hipStreamSynchronize(s));
  if (breakdown) {
    set_error("nyspcg_solve: PCG breakdown (p^T A p <= 0 or non-finite) in at least one column");
    return NYS_ENOTPD;
  }
  for (int c = 0; c < mtot; ++c)
    if (info[c].status != NYS_OK) return NYS_NOT_CONVERGED;
  return NYS_OK;
}
