"""Writes closed_forms.json: kernel values and 2x2 solves derived by hand from the
definitions (eq. rlaopt-krr with the RBF / Laplacian kernels, and the regularised
system of eq. rlaopt-regularized-linear-system).  Uses only the math module; nothing
here calls the library or the oracle."""
import json
import math
import os

cases = {}
# Points (0,0) and (3,4): |x-y| = 5, |x-y|^2 = 25.  sigma = 5.
s = 5.0
cases["triangle_3_4_5"] = {
    "x": [0.0, 0.0], "y": [3.0, 4.0], "sigma": s,
    "rbf": math.exp(-25.0 / (2.0 * s * s)),            # exp(-1/2)
    "laplacian": math.exp(-5.0 / s),                     # exp(-1)
    "rbf_dsigma": math.exp(-25.0 / (2.0 * s * s)) * 25.0 / s ** 3,
    "laplacian_dsigma": math.exp(-5.0 / s) * 5.0 / s ** 2,
}
# Two points at distance 1 on a line, RBF with sigma = 1: k = exp(-1/2).
# (K + lam I) x = b with K = [[1, k], [k, 1]]:
#   x1 = ((1+lam) b1 - k b2) / ((1+lam)^2 - k^2),  x2 = ((1+lam) b2 - k b1) / ((1+lam)^2 - k^2)
k = math.exp(-0.5)
lam = 0.25
b1, b2 = 1.0, -2.0
den = (1 + lam) ** 2 - k * k
cases["two_point_solve"] = {
    "X": [[0.0], [1.0]], "sigma": 1.0, "lam": lam, "b": [b1, b2],
    "x": [((1 + lam) * b1 - k * b2) / den, ((1 + lam) * b2 - k * b1) / den],
}
# Relative residual (eq. experiment-relative-residual) of the same 2x2 system at
# perturbed iterates: column 0 is x + e with e = (0.01, -0.03), so the residual is
# (K + lam I) e; column 1 solves for the right-hand side 3 b with the perturbation
# 2 e (relative residual 2/3 of column 0's); column 2 has b = 0 and x = e, for which
# the relative residual is undefined and the absolute norm |(K + lam I) e| is
# reported instead.  |b| = sqrt(5), so dividing by |b|^2 or leaving out the square
# roots changes every value.
e1, e2 = 0.01, -0.03
r1, r2 = (1 + lam) * e1 + k * e2, k * e1 + (1 + lam) * e2
xs = cases["two_point_solve"]["x"]
rn = math.sqrt(r1 * r1 + r2 * r2)
cases["two_point_relative_residual"] = {
    "X": [[0.0], [1.0]], "sigma": 1.0, "lam": lam,
    "B": [[b1, 3 * b1, 0.0], [b2, 3 * b2, 0.0]],
    "Xsol": [[xs[0] + e1, 3 * xs[0] + 2 * e1, e1], [xs[1] + e2, 3 * xs[1] + 2 * e2, e2]],
    "relres": [rn / math.sqrt(b1 * b1 + b2 * b2), 2 * rn / (3 * math.sqrt(b1 * b1 + b2 * b2)), rn],
}
# Eigenvalues of the 2x2 kernel matrix: 1 + k and 1 - k.
cases["two_point_eigs"] = {"X": [[0.0], [1.0]], "sigma": 1.0, "eigs": [1.0 + k, 1.0 - k]}

with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "closed_forms.json"), "w") as f:
    json.dump(cases, f, indent=1, sort_keys=True)
