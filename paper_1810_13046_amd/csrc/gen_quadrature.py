"""Generate the tetrahedral quadrature rules used by the integration kernels
(quadrature.inc).

Every integrand on a sub-tetrahedron of a clipped piece is a polynomial of
degree <= 4 (λ_i N_j and the shape-derivative products; the paper's
assembly integrates the mortar products with quadrature on the
intersection, Section 2.3).  Two fully symmetric rules are written:

* 14 points, degree 5, positive weights (a rule of this family is due to
  Walkington, "Quadrature on simplices of arbitrary dimension", 2000): two
  S31 orbits (a, a, a, 1-3a) of 4 points and one S22 orbit
  (b, b, 1/2-b, 1/2-b) of 6 points.  Used where the products themselves are
  integrated.
* 11 points, degree 4 (the structure of Keast's rule, 1986): the centroid
  with a negative weight, one S31 orbit and one S22 orbit.  Used for the 35
  piece moments (degree <= 4); Σ|w| / Σw = 1.16 bounds the extra rounding.
  No symmetric degree-4 rule with fewer than 14 points has positive
  weights and interior points, so the saving costs that negative weight.

The parameters are not typed in: they are solved here from the moment
equations  Σ_q w_q λ^α(q) = 3! α! / (|α|+3)!  for every barycentric monomial
of the rule's degree, by Levenberg–Marquardt from a coarse start, and the
script refuses to write the file unless every equation holds to 1e-15.

Run:  python gen_quadrature.py  (writes quadrature.inc next to this file).
"""
from __future__ import annotations

import itertools
import math
import os

import numpy as np
from scipy.optimize import least_squares


def points_weights(p):
    a1, a2, b, w1, w2 = p
    w3 = (1.0 - 4 * w1 - 4 * w2) / 6.0
    pts, wts = [], []
    for a, w in ((a1, w1), (a2, w2)):
        for k in range(4):
            q = [a] * 4
            q[k] = 1 - 3 * a
            pts.append(q)
            wts.append(w)
    for k, l in itertools.combinations(range(4), 2):
        q = [0.5 - b] * 4
        q[k] = b
        q[l] = b
        pts.append(q)
        wts.append(w3)
    return np.array(pts), np.array(wts)


def exponents(maxdeg):
    for e in itertools.product(range(maxdeg + 1), repeat=4):
        if sum(e) <= maxdeg:
            yield e


def exact(e):
    # ∫_T λ^e dV / |T| = 3! Π e_k! / (|e|+3)!
    return 6.0 * math.prod(math.factorial(k) for k in e) / math.factorial(sum(e) + 3)


def residual(p):
    pts, wts = points_weights(p)
    r = []
    for e in exponents(5):
        r.append(np.sum(wts * np.prod(pts ** np.array(e), axis=1)) - exact(e))
    return np.array(r)


def solve():
    best = None
    for start in ([0.09, 0.31, 0.045, 0.07, 0.11], [0.1, 0.3, 0.05, 0.05, 0.1]):
        sol = least_squares(residual, start, xtol=3e-16, ftol=3e-16, gtol=3e-16,
                            method="lm", max_nfev=20000)
        x = sol.x
        for _ in range(8):                        # Gauss–Newton polish
            r = residual(x)
            J = np.empty((r.size, x.size))
            for k in range(x.size):
                dx = np.zeros_like(x)
                dx[k] = 1e-7
                J[:, k] = (residual(x + dx) - residual(x - dx)) / 2e-7
            x = x - np.linalg.lstsq(J, r, rcond=None)[0]
        if best is None or np.max(np.abs(residual(x))) < np.max(np.abs(residual(best))):
            best = x
    p = best
    pts, wts = points_weights(p)
    err = np.max(np.abs(residual(p)))
    if err > 1e-15 or np.any(wts <= 0) or np.any(pts < 0):
        raise SystemExit(f"rule not found: max moment error {err:.3e}")
    return p, pts, wts, err


def points_weights4(p):
    w0, a, wa, b = p
    wb = (1.0 - w0 - 4 * wa) / 6.0
    pts, wts = [[0.25] * 4], [w0]
    for k in range(4):
        q = [a] * 4
        q[k] = 1 - 3 * a
        pts.append(q)
        wts.append(wa)
    for k, l in itertools.combinations(range(4), 2):
        q = [0.5 - b] * 4
        q[k] = b
        q[l] = b
        pts.append(q)
        wts.append(wb)
    return np.array(pts), np.array(wts)


def residual4(p):
    pts, wts = points_weights4(p)
    return np.array([np.sum(wts * np.prod(pts ** np.array(e), axis=1)) - exact(e)
                     for e in exponents(4)])


def solve4():
    """The 11-point degree-4 rule (S4 + S31 + S22), b < 1/4 branch."""
    sol = least_squares(residual4, [-0.08, 0.07, 0.045, 0.1], xtol=3e-16, ftol=3e-16,
                        gtol=3e-16, method="lm", max_nfev=20000)
    x = sol.x
    for _ in range(8):                            # Gauss–Newton polish
        r = residual4(x)
        J = np.empty((r.size, x.size))
        for k in range(x.size):
            dx = np.zeros_like(x)
            dx[k] = 1e-7
            J[:, k] = (residual4(x + dx) - residual4(x - dx)) / 2e-7
        x = x - np.linalg.lstsq(J, r, rcond=None)[0]
    pts, wts = points_weights4(x)
    err = np.max(np.abs(residual4(x)))
    if err > 1e-15 or np.any(pts < 0) or np.any(wts[1:] <= 0):
        raise SystemExit(f"degree-4 rule not found: max moment error {err:.3e}")
    return x, pts, wts, err


def main():
    p, pts, wts, err = solve()
    a1, a2, b, w1, w2 = p
    w3 = (1.0 - 4 * w1 - 4 * w2) / 6.0
    q4, pts4, wts4, err4 = solve4()
    w0, a, wa, b4 = q4
    wb = (1.0 - w0 - 4 * wa) / 6.0
    here = os.path.dirname(os.path.abspath(__file__))
    with open(os.path.join(here, "quadrature.inc"), "w") as f:
        f.write("// Generated by gen_quadrature.py: symmetric 14-point tetrahedral rule,\n")
        f.write("// degree 5, positive weights (weights sum to 1; multiply by the volume).\n")
        f.write(f"// Max moment error over all barycentric monomials of degree <= 5: {err:.2e}\n")
        f.write("// S31 orbits: (a, a, a, 1-3a);  S22 orbit: (b, b, 1/2-b, 1/2-b).\n")
        for name, v in (("kQA1", a1), ("kQA2", a2), ("kQB", b), ("kQW1", w1), ("kQW2", w2),
                        ("kQW3", w3)):
            f.write(f"constexpr double {name} = {float(v)!r};\n")
        f.write("// Symmetric 11-point rule, degree 4: centroid (weight kQ4W0 < 0), S31 orbit\n")
        f.write("// (a, a, a, 1-3a), S22 orbit (b, b, 1/2-b, 1/2-b); weights sum to 1.\n")
        f.write(f"// Max moment error over all barycentric monomials of degree <= 4: {err4:.2e}\n")
        for name, v in (("kQ4W0", w0), ("kQ4A", a), ("kQ4WA", wa), ("kQ4B", b4),
                        ("kQ4WB", wb)):
            f.write(f"constexpr double {name} = {float(v)!r};\n")
    print("a1 a2 b w1 w2 w3 =", a1, a2, b, w1, w2, w3, "err", err)
    print("w0 a wa b wb =", w0, a, wa, b4, wb, "err", err4, "sum|w|", np.abs(wts4).sum())


if __name__ == "__main__":
    main()
