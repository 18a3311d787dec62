"""Independent numerical integration used only by the tests to pin the oracle.

Stroud's conical-product (collapsed-coordinate) Gauss rule on a tetrahedron:
the unit cube (u, v, w) maps to the reference simplex by
x = u, y = v (1-u), z = w (1-u)(1-v), Jacobian (1-u)^2 (1-v); Gauss–Jacobi
points absorb the Jacobian.  With n points per direction it is exact for
polynomials of degree <= 2n-1.  Nodes come from scipy, not from any table.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np
from scipy.special import roots_jacobi


def _gj01(n, alpha):
    x, w = roots_jacobi(n, alpha, 0.0)      # weight (1-x)^alpha on [-1, 1]
    t = 0.5 * (1.0 + x)
    return t, w / 2.0 ** (alpha + 1)


def stroud_rule(n=5):
    """Points (barycentric, (m,4)) and weights (sum 1) on any tetrahedron."""
    u, wu = _gj01(n, 2.0)
    v, wv = _gj01(n, 1.0)
    w, ww = _gj01(n, 0.0)
    U, V, Wc = np.meshgrid(u, v, w, indexing="ij")
    WU, WV, WW = np.meshgrid(wu, wv, ww, indexing="ij")
    x = U
    y = V * (1 - U)
    z = Wc * (1 - U) * (1 - V)
    wt = (WU * WV * WW).ravel() * 6.0       # reference volume 1/6 -> weights sum to 1
    bary = np.stack([1 - x - y - z, x, y, z], axis=-1).reshape(-1, 4)
    return bary, wt


def tet_integral(P, f, n=5):
    """∫_T f for T with vertices P (4x3); f maps (m,3) points to (m, ...)."""
    bary, wt = stroud_rule(n)
    pts = bary @ np.asarray(P, dtype=np.float64)
    a = P[1] - P[0]
    b = P[2] - P[0]
    c = P[3] - P[0]
    vol = abs(np.dot(a, np.cross(b, c))) / 6.0
    vals = f(pts)
    return vol * np.tensordot(wt, vals, axes=(0, 0))


def hat_integral_exact(nodes, k, a, b):
    """∫_a^b of the 1D hat of node k on `nodes` (piecewise-linear, exact)."""
    nodes = [float(t) for t in nodes]
    total = 0.0
    segs = []
    if k > 0:
        segs.append((nodes[k - 1], nodes[k], 0.0, 1.0))
    if k < len(nodes) - 1:
        segs.append((nodes[k], nodes[k + 1], 1.0, 0.0))
    for s0, s1, f0, f1 in segs:
        lo, hi = max(s0, a), min(s1, b)
        if hi <= lo:
            continue
        g0 = f0 + (f1 - f0) * (lo - s0) / (s1 - s0)
        g1 = f0 + (f1 - f0) * (hi - s0) / (s1 - s0)
        total += 0.5 * (hi - lo) * (g0 + g1)
    return total


def ref_simplex_monomial(a, b, c):
    """∫ over {x,y,z>=0, x+y+z<=1} of x^a y^b z^c = a! b! c! / (a+b+c+3)!"""
    from math import factorial
    return Fraction(factorial(a) * factorial(b) * factorial(c), factorial(a + b + c + 3))


def triangle_rule(n=6):
    """Conical-product Gauss rule on a triangle: (u, v) in the unit square
    maps to x = u, y = v (1-u), Jacobian (1-u); Gauss–Jacobi points in u
    absorb it.  Exact for degree <= 2n-1.  Returns barycentric points (m,3)
    and weights summing to 1."""
    u, wu = _gj01(n, 1.0)
    v, wv = _gj01(n, 0.0)
    U, V = np.meshgrid(u, v, indexing="ij")
    WU, WV = np.meshgrid(wu, wv, indexing="ij")
    x = U
    y = V * (1 - U)
    wt = (WU * WV).ravel() * 2.0            # reference area 1/2 -> weights sum to 1
    bary = np.stack([1 - x - y, x, y], axis=-1).reshape(-1, 3)
    return bary, wt


def tri_integral(P, f, n=6):
    """∫_T f for triangle T with vertices P (3x2); f maps (m,2) points to (m, ...)."""
    P = np.asarray(P, dtype=np.float64)
    bary, wt = triangle_rule(n)
    pts = bary @ P
    a = P[1] - P[0]
    b = P[2] - P[0]
    area = 0.5 * abs(a[0] * b[1] - a[1] * b[0])
    return area * np.tensordot(wt, f(pts), axes=(0, 0))


def ref_triangle_monomial(a, b):
    """∫ over {x,y>=0, x+y<=1} of x^a y^b = a! b! / (a+b+2)!"""
    from math import factorial
    return Fraction(factorial(a) * factorial(b), factorial(a + b + 2))
