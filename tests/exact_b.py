"""Exact rational coupling entries B^d_ij = ∫ λ_i N^d_j (Section 2.3) for
small meshes, in Python's Fraction arithmetic: test infrastructure that
pins the FP64 oracle, sharing no code with it.

Floats are dyadic rationals, so the mesh and the grid faces convert
exactly, and every cut point of an axis plane with a tet edge is rational.
The route differs from the oracle's at each step:
  * a piece is the tet clipped by the cell's six half-spaces as a list of
    face polygons (each face clipped as a polygon; the cut points on the
    plane close the piece with a cap ordered around its centroid);
  * a piece is cut into tetrahedra from one of its vertices across the
    faces that do not contain it;
  * λ_i N_j (four affine factors: λ_i and the three 1D hats of corner j)
    is written in the barycentric coordinates ξ of each sub-tetrahedron,
    expanded into monomials ξ^α, and integrated with
    ∫_ref ξ^α = α1! α2! α3! / (|α| + 3)! times the Jacobian.
Ties follow the method's rule: a point with signed distance >= 0 is inside.
Pieces of volume <= drop_rel |T| are left out, as in the method."""
from fractions import Fraction as Q
import functools
import math

DROP_REL = Q(1, 10 ** 14)


def lattice(faces, d):
    """Component d's node coordinates per axis: the faces along axis d, the
    face midpoints along the others."""
    out = []
    for e in range(3):
        f = [Q(float(x)) for x in faces[e]]
        out.append(f if e == d else [(f[k] + f[k + 1]) / 2 for k in range(len(f) - 1)])
    return out


def det3(a, b, c):
    return (a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) +
            a[2] * (b[0] * c[1] - b[1] * c[0]))


def sub(p, q):
    return (p[0] - q[0], p[1] - q[1], p[2] - q[2])


def barycentric(P):
    """Affine λ_i(x) = c_i + g_i·x of the tet with vertices P (exact)."""
    # solve [1 x y z] rows: M a = e_i for each i
    M = [[Q(1), P[k][0], P[k][1], P[k][2]] for k in range(4)]
    # invert M by Gauss-Jordan
    A = [row[:] + [Q(int(i == k)) for i in range(4)] for k, row in enumerate(M)]
    for col in range(4):
        piv = next(r for r in range(col, 4) if A[r][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        pv = A[col][col]
        A[col] = [v / pv for v in A[col]]
        for r in range(4):
            if r != col and A[r][col] != 0:
                f = A[r][col]
                A[r] = [a - f * b for a, b in zip(A[r], A[col])]
    inv = [row[4:] for row in A]
    # λ_i = Σ_m inv[m][i] · (1, x, y, z)_m
    return [(inv[0][i], (inv[1][i], inv[2][i], inv[3][i])) for i in range(4)]


def tet_faces(P):
    return [[P[1], P[2], P[3]], [P[0], P[3], P[2]], [P[0], P[1], P[3]], [P[0], P[2], P[1]]]


def dedupe(poly):
    out = []
    for p in poly:
        if not out or out[-1] != p:
            out.append(p)
    while len(out) > 1 and out[0] == out[-1]:
        out.pop()
    return out


def order_in_plane(pts, e):
    """Points of a convex polygon in the plane x_e = const, in cyclic order
    (angle about their centroid, compared exactly)."""
    a, b = [k for k in range(3) if k != e]
    ca = sum(p[a] for p in pts) / len(pts)
    cb = sum(p[b] for p in pts) / len(pts)

    def half(p):
        u, v = p[a] - ca, p[b] - cb
        return 0 if (v > 0 or (v == 0 and u > 0)) else 1

    def cmp(p, q):
        hp, hq = half(p), half(q)
        if hp != hq:
            return hp - hq
        cr = (p[a] - ca) * (q[b] - cb) - (p[b] - cb) * (q[a] - ca)
        return -1 if cr > 0 else (1 if cr < 0 else 0)

    return sorted(pts, key=functools.cmp_to_key(cmp))


def clip(faces, e, c, sign):
    """Keep sign·(x_e − c) >= 0 of the convex polyhedron given by faces."""
    out_faces = []
    on_plane = []
    for face in faces:
        n = len(face)
        out = []
        for k in range(n):
            p, q = face[k], face[(k + 1) % n]
            sp, sq = sign * (p[e] - c), sign * (q[e] - c)
            if sp >= 0:
                out.append(p)
            if (sp >= 0) != (sq >= 0):
                t = sp / (sp - sq)
                r = [p[m] + t * (q[m] - p[m]) for m in range(3)]
                r[e] = c
                out.append(tuple(r))
        out = dedupe(out)
        if len(out) >= 3:
            out_faces.append(out)
    for f in out_faces:
        for p in f:
            if p[e] == c and p not in on_plane:
                on_plane.append(p)
    has_face = any(all(p[e] == c for p in f) for f in out_faces)
    if not has_face and len(on_plane) >= 3:
        out_faces.append(order_in_plane(on_plane, e))
    return out_faces


def volume6(faces):
    """6 |piece| by the tets from the first vertex over the other faces."""
    verts = [p for f in faces for p in f]
    if not verts:
        return Q(0), []
    apex = verts[0]
    tets = []
    v6 = Q(0)
    for f in faces:
        if apex in f:
            continue
        for k in range(1, len(f) - 1):
            t = (apex, f[0], f[k], f[k + 1])
            dv = abs(det3(sub(t[1], t[0]), sub(t[2], t[0]), sub(t[3], t[0])))
            if dv != 0:
                tets.append((t, dv))
                v6 += dv
    return v6, tets


def poly_mul(A, B):
    out = {}
    for ka, va in A.items():
        for kb, vb in B.items():
            k = (ka[0] + kb[0], ka[1] + kb[1], ka[2] + kb[2])
            out[k] = out.get(k, Q(0)) + va * vb
    return out


def affine_in_xi(vals):
    """An affine function with values vals at the 4 vertices, in ξ."""
    return {(0, 0, 0): vals[0], (1, 0, 0): vals[1] - vals[0], (0, 1, 0): vals[2] - vals[0],
            (0, 0, 1): vals[3] - vals[0]}


@functools.lru_cache(maxsize=None)
def ref_moment(a, b, c):
    """∫ over the reference tetrahedron of ξ1^a ξ2^b ξ3^c."""
    return Q(math.factorial(a) * math.factorial(b) * math.factorial(c),
             math.factorial(a + b + c + 3))


def cell_values(tets6, lam, lo, hi):
    """The 4 x 8 integrals ∫ λ_i N_j over the piece (sub-tets with their
    6-volumes), corner j = a + 2b + 4c.  On a sub-tet, with P_j the product
    of corner j's three hats in ξ, λ_i = l_0 + Σ_k (l_k − l_0) ξ_k gives
    ∫ λ_i P_j = l_0 ∫ P_j + Σ_k (l_k − l_0) ∫ ξ_k P_j."""
    b = [[Q(0)] * 8 for _ in range(4)]
    shift = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
    for t, dv in tets6:
        hats = []
        for e in range(3):
            h = hi[e] - lo[e]
            up = affine_in_xi([(p[e] - lo[e]) / h for p in t])
            dn = affine_in_xi([(hi[e] - p[e]) / h for p in t])
            hats.append((dn, up))
        lv = [[c + g[0] * p[0] + g[1] * p[1] + g[2] * p[2] for p in t] for c, g in lam]
        xy = [poly_mul(hats[0][j & 1], hats[1][(j >> 1) & 1]) for j in range(4)]
        for j in range(8):
            prod = poly_mul(xy[j & 3], hats[2][j >> 2])
            m = [sum((v * ref_moment(a + s[0], bb + s[1], c + s[2])
                      for (a, bb, c), v in prod.items()), Q(0)) for s in shift]
            for i in range(4):
                l = lv[i]
                b[i][j] += dv * (l[0] * m[0] + (l[1] - l[0]) * m[1] + (l[2] - l[0]) * m[2] +
                                 (l[3] - l[0]) * m[3])
    return b


def assemble_exact(faces, X, tets, drop_rel=DROP_REL):
    """{(d, i, j): B^d_ij} for the mesh (X: float vertices, tets: int
    indices), exact.  Zero-volume tets are left out."""
    B = {}
    lats = [lattice(faces, d) for d in range(3)]
    for tv in tets:
        P = [tuple(Q(float(x)) for x in X[v]) for v in tv]
        v6 = abs(det3(sub(P[1], P[0]), sub(P[2], P[0]), sub(P[3], P[0])))
        if v6 == 0:
            continue
        lam = barycentric(P)
        for d in range(3):
            L = lats[d]
            n = [len(L[0]), len(L[1]), len(L[2])]
            rng = []
            for e in range(3):
                mn = min(p[e] for p in P)
                mx = max(p[e] for p in P)
                cells = [k for k in range(n[e] - 1) if L[e][k] < mx and L[e][k + 1] > mn]
                rng.append(cells)
            for cz in rng[2]:
                for cy in rng[1]:
                    for cx in rng[0]:
                        ci = (cx, cy, cz)
                        lo = [L[e][ci[e]] for e in range(3)]
                        hi = [L[e][ci[e] + 1] for e in range(3)]
                        fc = tet_faces(P)
                        for e in range(3):
                            fc = clip(fc, e, lo[e], 1)
                            fc = clip(fc, e, hi[e], -1)
                            if not fc:
                                break
                        if not fc:
                            continue
                        pv6, sub_tets = volume6(fc)
                        if pv6 <= drop_rel * v6:
                            continue
                        vals = cell_values(sub_tets, lam, lo, hi)
                        for i in range(4):
                            for j in range(8):
                                if vals[i][j] == 0:
                                    continue
                                node = ((cx + (j & 1)) + n[0] * ((cy + ((j >> 1) & 1)) +
                                                                n[1] * (cz + (j >> 2))))
                                k = (d, int(tv[i]), node)
                                B[k] = B.get(k, Q(0)) + vals[i][j]
    return B
