"""FP64 CPU oracle of the two-dimensional coupling: Q1 (bilinear) hats on a
staggered rectilinear grid against a P1 triangle mesh.

TEST INFRASTRUCTURE ONLY, like the rest of this package.

This is the setting of the paper's 2D experiments (Section 4: Turek–Hron and
the inertia test), where bilinear Q1 hats are attached to the fluid grid and
the solid is meshed with linear triangles; the operators are those of
Section 2.3 with areas in place of volumes:

* B^d_ij = ∫ λ_i N^d_j dA for velocity components d = 0, 1 (C part, o2.c);
* S = the P1 mass M_il = |T|(1+δ_il)/12 per triangle, or its row sums
  m_i = Σ_{T∋i} |T|/3 (lumped);
* the dual multipliers of the pseudo-L2 variant: ψ_i = 4λ_i − 1 on each
  triangle (∫_T ψ_i λ_j = δ_ij |T|/3), so S = diag(m) and a piece's values
  become 4·b_i − Σ_k b_k;
* velocity w_s = S^{-1} B v_f (sparse direct solve, never CG) and force
  f_f = alpha B^T f_s (or the literal T^T = B^T S^{-1} on a load vector);
* the reverse mode with the shape derivative of B, as in three dimensions.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import DROP_REL, OutOfGrid

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "o2.c")
_LIB = os.path.join(_HERE, "_o2.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the 2D C part with gcc (plain C, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        dp, i64p, i32p = P(ctypes.c_double), P(ctypes.c_int64), P(ctypes.c_int32)
        lib.o2_pair_counts.argtypes = [P(dp), i64p, dp, i32p, i64p, ctypes.c_int64, i64p, i32p]
        lib.o2_pair_counts.restype = ctypes.c_int
        lib.o2_pairs.argtypes = [P(dp), i64p, dp, ctypes.c_int64, i32p, i64p, ctypes.c_int64, i32p,
                                 i64p, ctypes.c_double, ctypes.c_int, dp, dp,
                                 P(ctypes.c_uint8), i32p, dp, P(dp), dp, i64p, ctypes.c_int]
        lib.o2_pairs.restype = ctypes.c_int
        lib.o2_int3.argtypes = [dp] * 4
        lib.o2_int3.restype = ctypes.c_double
        lib.o2_clip_area.argtypes = [dp] * 3
        lib.o2_clip_area.restype = ctypes.c_double
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i64p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _i32p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


# ----------------------------------------------------------------------------
# Q1 lattices on the staggered 2D grid
# ----------------------------------------------------------------------------

def lattice(faces, d: int):
    """Node coordinates of velocity component d's Q1 lattice, per axis:
    face coordinates along axis d, cell centres along the other axis (the
    staggered arrangement of Section 2.2)."""
    out = []
    for e in range(2):
        f = np.asarray(faces[e], dtype=np.float64)
        out.append(f.copy() if e == d else 0.5 * (f[:-1] + f[1:]))
    return out


def lattice_shape(faces, d: int):
    """(n_x, n_y) nodes of component d's lattice."""
    return tuple(len(a) for a in lattice(faces, d))


def n_fluid(faces, d: int) -> int:
    nx, ny = lattice_shape(faces, d)
    return nx * ny


# ----------------------------------------------------------------------------
# P1 triangles
# ----------------------------------------------------------------------------

def tri_areas(X, tris):
    X = np.asarray(X, dtype=np.float64)
    a = X[tris[:, 1]] - X[tris[:, 0]]
    b = X[tris[:, 2]] - X[tris[:, 0]]
    return 0.5 * np.abs(a[:, 0] * b[:, 1] - a[:, 1] * b[:, 0])


def barycentric_gradients(X, tris):
    """grad λ_a per triangle: (n_t, 3, 2), from the inverse of [1 x y] rows."""
    X = np.asarray(X, dtype=np.float64)
    A = np.ones((tris.shape[0], 3, 3))
    A[:, :, 1:] = X[tris]
    inv = np.linalg.inv(A)
    return np.transpose(inv[:, 1:, :], (0, 2, 1))


def lumped_mass(X, tris, n_vert=None):
    """m_i = ∫ λ_i = Σ_{T∋i} |T|/3."""
    n_vert = X.shape[0] if n_vert is None else n_vert
    a = tri_areas(X, tris)
    m = np.zeros(n_vert)
    for k in range(3):
        np.add.at(m, tris[:, k], a / 3.0)
    return m


def consistent_mass(X, tris, n_vert=None):
    """P1 mass matrix M_il = ∫ λ_i λ_l = |T|(1+δ_il)/12 per triangle."""
    n_vert = X.shape[0] if n_vert is None else n_vert
    a = tri_areas(X, tris)
    rows, cols, vals = [], [], []
    for i in range(3):
        for l in range(3):
            rows.append(tris[:, i])
            cols.append(tris[:, l])
            vals.append(a * (2.0 if i == l else 1.0) / 12.0)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n_vert, n_vert))


# ----------------------------------------------------------------------------
# Pairs (triangle, component, cell) and the coupling matrices
# ----------------------------------------------------------------------------

@dataclass
class Pairs:
    subset: np.ndarray
    counts: np.ndarray          # (n_sub*2,)
    offsets: np.ndarray         # (n_sub*2+1,)
    ranges: np.ndarray          # (n_sub*2, 4)
    vals: np.ndarray            # (n_pairs, 12)
    areas: np.ndarray           # (n_pairs,)
    keep: np.ndarray            # (n_pairs,) bool
    cell: np.ndarray            # (n_pairs, 2)
    G: np.ndarray | None        # (n_pairs, 6)
    zero_tris: int
    seconds: float = 0.0

    def owner(self):
        """(subset position, component) of every pair."""
        sd = np.repeat(np.arange(self.counts.size), self.counts)
        return sd // 2, sd % 2


def _lat_arrays(faces):
    flat = [np.ascontiguousarray(lattice(faces, d)[e]) for d in range(2) for e in range(2)]
    ptrs = (ctypes.POINTER(ctypes.c_double) * 4)(*[_dp(a) for a in flat])
    nlat = np.array([a.size for a in flat], dtype=np.int64)
    return flat, ptrs, nlat


def pairs(faces, X, tris, subset=None, drop_rel=DROP_REL, nthreads=0, z=None, u_f=None,
          dual=False):
    """Integrate every (triangle, component, cell) pair of the selected triangles."""
    lib = _load()
    X = np.ascontiguousarray(X, dtype=np.float64)
    tris = np.ascontiguousarray(tris, dtype=np.int32)
    subset = (np.arange(tris.shape[0], dtype=np.int64) if subset is None
              else np.ascontiguousarray(subset, dtype=np.int64))
    flat, ptrs, nlat = _lat_arrays(faces)
    n_sub = subset.size
    counts = np.zeros(n_sub * 2, dtype=np.int64)
    ranges = np.zeros((n_sub * 2, 4), dtype=np.int32)
    st = lib.o2_pair_counts(ptrs, _i64p(nlat), _dp(X), _i32p(tris), _i64p(subset), n_sub,
                            _i64p(counts), _i32p(ranges))
    if st == -2:
        raise OutOfGrid("a triangle's bounding box leaves a velocity lattice")
    offsets = np.zeros(n_sub * 2 + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    n_pairs = int(offsets[-1])
    vals = np.zeros((n_pairs, 12))
    areas = np.zeros(n_pairs)
    keep = np.zeros(n_pairs, dtype=np.uint8)
    cell = np.zeros((n_pairs, 2), dtype=np.int32)
    zt = np.zeros(1, dtype=np.int64)
    G = None
    zp = ctypes.POINTER(ctypes.c_double)()
    up = ctypes.POINTER(ctypes.POINTER(ctypes.c_double))()
    Gp = ctypes.POINTER(ctypes.c_double)()
    keep_alive = []
    if z is not None:
        zc = np.ascontiguousarray(z, dtype=np.float64)
        uc = [np.ascontiguousarray(np.asarray(u, dtype=np.float64).ravel()) for u in u_f]
        keep_alive += [zc, uc]
        G = np.zeros((n_pairs, 6))
        zp = _dp(zc)
        up = (ctypes.POINTER(ctypes.c_double) * 2)(*[_dp(a) for a in uc])
        Gp = _dp(G)
    t0 = time.perf_counter()
    lib.o2_pairs(ptrs, _i64p(nlat), _dp(X), X.shape[0], _i32p(tris), _i64p(subset), n_sub,
                 _i32p(ranges), _i64p(offsets), float(drop_rel), int(nthreads), _dp(vals),
                 _dp(areas), keep.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), _i32p(cell),
                 zp, up, Gp, _i64p(zt), int(bool(dual)))
    dt = time.perf_counter() - t0
    return Pairs(subset, counts, offsets, ranges, vals, areas, keep.astype(bool), cell, G,
                 int(zt[0]), dt)


@dataclass
class Coupling:
    """B^d (n_vert x n_f,d, CSR) for d = 0, 1 plus what produced them."""
    faces: list
    X: np.ndarray
    tris: np.ndarray
    B: list
    pairs: Pairs
    stats: dict = field(default_factory=dict)
    dual: bool = False

    @property
    def n_vert(self):
        return self.X.shape[0]


def assemble(faces, X, tris, subset=None, drop_rel=DROP_REL, nthreads=0, dual=False) -> Coupling:
    """Mortar matrices B^d_ij = ∫ λ_i N^d_j over the selected triangles (all
    by default); with dual=True, B^d_ij = ∫ ψ_i N^d_j with ψ_i = 4λ_i − 1 =
    Σ_k (4δ_ik − 1) λ_k, so a piece's values are 4·b_i − Σ_k b_k."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    tris = np.ascontiguousarray(tris, dtype=np.int32)
    P = pairs(faces, X, tris, subset, drop_rel, nthreads)
    pvals = P.vals
    if dual:
        b = P.vals.reshape(-1, 3, 4)
        pvals = (4.0 * b - b.sum(axis=1, keepdims=True)).reshape(-1, 12)
    s_idx, comp = P.owner()
    t_idx = P.subset[s_idx]
    B = []
    for d in range(2):
        nx, ny = lattice_shape(faces, d)
        sel = np.nonzero((comp == d) & P.keep)[0]
        tv = tris[t_idx[sel]]                                     # (k, 3)
        c = P.cell[sel].astype(np.int64)
        rows = np.repeat(tv, 4, axis=1).reshape(-1)               # i major, corner minor
        corner = np.arange(4)
        a, b = corner & 1, (corner >> 1) & 1
        node = (c[:, 0:1] + a) + nx * (c[:, 1:2] + b)              # (k, 4)
        cols = np.tile(node, (1, 3)).reshape(-1)
        vals = pvals[sel].reshape(-1)
        B.append(sp.csr_matrix((vals, (rows, cols)), shape=(X.shape[0], nx * ny)))
    stats = dict(pairs=int(P.offsets[-1]), pieces=int(P.keep.sum()),
                 dropped=int(((P.areas > 0) & ~P.keep).sum()), zero_tris=P.zero_tris,
                 seconds=P.seconds)
    return Coupling(list(faces), X, tris, B, P, stats, dual)


def tri_bounds(X, tris):
    P = np.asarray(X)[tris]
    return P.min(axis=1), P.max(axis=1)


def tris_touching_node(faces, X, tris, d, node_ij, bounds=None):
    """Triangles whose bounding box meets the support of fluid node (i, j)
    of component d (a superset of those contributing to that column)."""
    lat = lattice(faces, d)
    lo = np.empty(2)
    hi = np.empty(2)
    for e in range(2):
        k = node_ij[e]
        lo[e] = lat[e][max(k - 1, 0)]
        hi[e] = lat[e][min(k + 1, lat[e].size - 1)]
    mn, mx = tri_bounds(X, tris) if bounds is None else bounds
    ok = np.all((mx >= lo) & (mn <= hi), axis=1)
    return np.nonzero(ok)[0]


# ----------------------------------------------------------------------------
# Transfers and their adjoints
# ----------------------------------------------------------------------------

def mass_solve(X, tris, rhs, mass: str):
    """S^{-1} rhs for each row of rhs (2, n_vert): lumped or consistent (direct)."""
    rhs = np.atleast_2d(rhs)
    if mass == "lumped":
        return rhs / lumped_mass(X, tris)[None, :]
    if mass == "consistent":
        lu = spla.splu(consistent_mass(X, tris).tocsc())
        return np.stack([lu.solve(r) for r in rhs])
    raise ValueError(mass)


def _mass_of(cpl: Coupling, mass: str) -> str:
    if cpl.dual:
        if mass == "consistent":
            raise ValueError("the dual basis has a diagonal S: use mass='lumped'")
        return "lumped"
    return mass


def transfer_velocity(cpl: Coupling, u_f, mass: str = "lumped"):
    """w_s = S^{-1} B v_f per component; u_f: 2 arrays of lattice shape
    (n_y, n_x).  Returns (2, n_vert)."""
    rhs = np.stack([cpl.B[d] @ np.asarray(u_f[d], dtype=np.float64).ravel() for d in range(2)])
    return mass_solve(cpl.X, cpl.tris, rhs, _mass_of(cpl, mass))


def transfer_force(cpl: Coupling, f_s, alpha: float = 1.0, load: bool = False, base=None):
    """f_f = base + alpha B^T f_s, or with load=True alpha B^T S^{-1} f_s
    (the literal transpose of the transfer on a load vector)."""
    f_s = np.asarray(f_s, dtype=np.float64)
    if load:
        f_s = mass_solve(cpl.X, cpl.tris, f_s, "lumped" if cpl.dual else "consistent")
    out = []
    for d in range(2):
        r = alpha * (cpl.B[d].T @ f_s[d])
        if base is not None:
            r = r + np.asarray(base[d], dtype=np.float64).ravel()
        out.append(r)
    return out


def _shape_pair_terms(faces, X, tris, z, u_f, nthreads=0, dual=False):
    P = pairs(faces, X, tris, None, DROP_REL, nthreads, z=z, u_f=u_f, dual=dual)
    s_idx, _ = P.owner()
    t_idx = P.subset[s_idx]
    g = np.zeros((X.shape[0], 2))
    Gk = P.G.reshape(-1, 3, 2) * P.keep[:, None, None]
    for a in range(3):
        np.add.at(g, tris[t_idx, a], Gk[:, a, :])
    return g


def _mass_shape_term(X, tris, z, u_s, mass):
    """Σ_d z^T (∂S/∂X) u_s^d as (n_vert, 2): ∂|T|/∂X_a = |T| ∇λ_a."""
    area = tri_areas(X, tris)
    grad = barycentric_gradients(X, tris)
    s = np.zeros(tris.shape[0])
    for d in range(2):
        zl = z[d][tris]
        ul = u_s[d][tris]
        if mass == "consistent":
            s += (np.einsum("ti,ti->t", zl, ul) + zl.sum(1) * ul.sum(1)) / 12.0
        else:
            s += np.einsum("ti,ti->t", zl, ul) / 3.0
    g = np.zeros((X.shape[0], 2))
    for a in range(3):
        np.add.at(g, tris[:, a], (area * s)[:, None] * grad[:, a, :])
    return g


def velocity_vjp(cpl: Coupling, u_f, g_us, mass: str = "lumped", nthreads=0):
    """Reverse mode of u_s = S^{-1} B u_f: (g_uf: 2 flat arrays, g_X (n_vert, 2))."""
    g_us = np.asarray(g_us, dtype=np.float64)
    mass = _mass_of(cpl, mass)
    z = mass_solve(cpl.X, cpl.tris, g_us, mass)
    u_s = transfer_velocity(cpl, u_f, mass)
    g_uf = [cpl.B[d].T @ z[d] for d in range(2)]
    gX = _shape_pair_terms(cpl.faces, cpl.X, cpl.tris, z, u_f, nthreads, cpl.dual)
    gX -= _mass_shape_term(cpl.X, cpl.tris, z, u_s, mass)
    return g_uf, gX


def force_vjp(cpl: Coupling, f_s, g_ff, alpha: float = 1.0, nthreads=0):
    """Reverse mode of f_f = alpha B^T f_s: (g_fs (2, n_vert), g_X)."""
    f_s = np.asarray(f_s, dtype=np.float64)
    g_fs = np.stack([alpha * (cpl.B[d] @ np.asarray(g_ff[d]).ravel()) for d in range(2)])
    gX = alpha * _shape_pair_terms(cpl.faces, cpl.X, cpl.tris, f_s, g_ff, nthreads, cpl.dual)
    return g_fs, gX


def velocity_loss(faces, X, tris, u_f, u_target, mass="lumped", dual=False):
    cpl = assemble(faces, X, tris, dual=dual)
    r = transfer_velocity(cpl, u_f, mass) - u_target
    return 0.5 * float(np.sum(r * r))


# ----------------------------------------------------------------------------
# Fixed-point (Picard) coupling of Section 3 in the plane
# ----------------------------------------------------------------------------

def fluid_lumped_volume(faces, d: int):
    """∫ N_j over the hull of component d's planar lattice for every node,
    shape (n_y, n_x): a product of two 1D hat integrals, each half the
    length of the node's neighbouring intervals."""
    w = []
    for L in lattice(faces, d):
        h = np.diff(L)
        we = np.zeros(L.size)
        we[:-1] += 0.5 * h
        we[1:] += 0.5 * h
        w.append(we)
    return np.outer(w[1], w[0])


def fsi_step(faces, X_ref, tris, u_hat0, v_f, solid, fluid, dt, alpha=1.0, eps_abs=0.0,
             eps_rel=1e-8, max_iter=50, mass="lumped", force_density=False, dual=False,
             f_prev=None):
    """One time step of the Picard iteration of Section 3 for a planar
    coupling, in the steps' order: T = S^{-1} B assembled at X_ref + u_hat0
    and held for the step; 1. w_s = T v_f; 2. u_hat = u_hat0 + dt w_s;
    3. f_fsi = solid(u_hat); 4. f_tilde = alpha B^T S^{-1} f_fsi (divided by
    the fluid nodes' lumped area with force_density); 5. v_f = fluid(f_tilde);
    6. stop when ||f_l − f_{l−1}||_inf < eps_abs or that over ||f_1||_inf <
    eps_rel; f_0 = f_prev (zeros by default).  Returns the last iteration's
    fields and the iteration count."""
    X = np.asarray(X_ref, dtype=np.float64) + np.asarray(u_hat0, dtype=np.float64).T
    cpl = assemble(faces, X, tris, dual=dual)
    S = _mass_of(cpl, mass)
    u_hat0 = np.asarray(u_hat0, dtype=np.float64)
    v = [np.asarray(a, dtype=np.float64).ravel().copy() for a in v_f]
    f_old = np.zeros_like(u_hat0) if f_prev is None else np.asarray(f_prev, dtype=np.float64)
    areas = [fluid_lumped_volume(faces, d).ravel() for d in range(2)] if force_density else None
    f1 = None
    out = {}
    for it in range(1, max_iter + 1):
        w_s = mass_solve(X, tris, np.stack([cpl.B[d] @ v[d] for d in range(2)]), S)
        u_hat = u_hat0 + dt * w_s
        f = np.asarray(solid(u_hat), dtype=np.float64)
        g = mass_solve(X, tris, f, S)
        f_tilde = [alpha * (cpl.B[d].T @ g[d]) for d in range(2)]
        if force_density:
            f_tilde = [f_tilde[d] / areas[d] for d in range(2)]
        v = [np.asarray(a, dtype=np.float64).ravel() for a in fluid(f_tilde)]
        res = float(np.max(np.abs(f - f_old)))
        if it == 1:
            f1 = float(np.max(np.abs(f)))
        rel = res / f1 if f1 > 0 else (np.inf if res > 0 else 0.0)
        f_old = f
        out = dict(iterations=it, w_s=w_s, u_hat=u_hat, f_fsi=f, f_tilde=f_tilde, v_f=v,
                   res_abs=res, res_rel=rel, f1_norm=f1, converged=False, B=cpl.B)
        if (eps_abs > 0 and res < eps_abs) or (eps_rel > 0 and rel < eps_rel):
            out["converged"] = True
            break
    return out


# ----------------------------------------------------------------------------
# Small helpers exposed for the pins
# ----------------------------------------------------------------------------

def int3(Y, f1, f2, f3) -> float:
    """∫_τ f1 f2 f3 for affine f_m given by vertex values (closed form)."""
    lib = _load()
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (Y, f1, f2, f3)]
    return lib.o2_int3(*[_dp(a) for a in arrs])


def clip_area(P, lo, hi) -> float:
    """Area of triangle P (3x2) ∩ box [lo, hi] (polygon clipping)."""
    lib = _load()
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (P, lo, hi)]
    return lib.o2_clip_area(*[_dp(a) for a in arrs])
