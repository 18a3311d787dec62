"""FP64 CPU oracle for the L2-projection fluid <-> solid transfer.

TEST INFRASTRUCTURE ONLY: the parity tests, the smoke check and the
benchmark's CPU-baseline leg use it; the product library never imports it.

It follows Section 2.3 of the paper ("Variational Transfer: the
L2-Projection Approach") directly:

* the auxiliary Q1 space on the staggered finite-difference grid (one node
  lattice per velocity component, Section 2.2 with its staggered-grid figure);
* the mortar integrals  B_ij = ∫ N_f,j N_fsi,i dV  (solid rows i, fluid
  columns j) and  S_ij = ∫ N_s,j N_fsi,i dV, with the standard multiplier
  space equal to the P1 solid space, so S is the P1 mass matrix M of
  Section 2.1 (Spatial Discretization);
* velocity transfer  w_s = S^{-1} B v_f  (S lumped or consistent), solved
  here with a sparse direct factorisation (never CG);
* force transfer with the transpose;
* the dual ("pseudo" L2) variant (eq. biorth): multipliers ψ_i biorthogonal
  to the P1 hats, here the element-local ψ_i = 5λ_i − 1 on each tet
  (∫_T λ_j ψ_i = δ_ij |T|/4), so S = diag(∫ψ_i) = the lumped P1 mass and
  B_ij = ∫ ψ_i N_j.

Readings where the paper is silent are listed in the design doc; the main ones:
lattice of component d = face coordinates along axis d and face midpoints
along the other two axes; lumped S = row sums of M; force transfer
f_f = alpha * B^T f_s with f_s as P1 nodal density coefficients (the
literal T^T on a load vector is available as `load=True`).

Parity is pinned by the tests in tests/test_oracle_pins.py (partition of
unity, exact box volumes and 1D closed forms of column sums, exact
reproduction of affine and trilinear fields, Monte Carlo brute force on tiny
meshes, exact-rational whole-tet integrals, finite differences of the
gradient).
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

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "o1.c")
_LIB = os.path.join(_HERE, "_o1.so")
_lib = None

DROP_REL = 1e-14


def build(force: bool = True) -> str:
    """Compile the C parts of the oracle (3D here, 2D in oracle.plane) with
    gcc (plain C, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    from . import plane, unstructured
    plane.build(force)
    unstructured.build(force)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        dp, i64p, i32p = P(ctypes.c_double), P(ctypes.c_int64), P(ctypes.c_int32)
        lib.o1_pair_counts.argtypes = [P(dp), i64p, dp, i32p, i64p, ctypes.c_int64, i64p, i32p]
        lib.o1_pair_counts.restype = ctypes.c_int
        lib.o1_pairs.argtypes = [P(dp), i64p, dp, ctypes.c_int64, i32p, i64p, ctypes.c_int64, i32p,
                                 i64p, ctypes.c_double, ctypes.c_int, dp, dp,
                                 P(ctypes.c_uint8), i32p, dp, P(dp), dp, i64p, ctypes.c_int]
        lib.o1_pairs.restype = ctypes.c_int
        lib.o1_int4.argtypes = [dp] * 5
        lib.o1_int4.restype = ctypes.c_double
        lib.o1_clip_volume.argtypes = [dp] * 3
        lib.o1_clip_volume.restype = ctypes.c_double
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i64p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _i32p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


class OutOfGrid(ValueError):
    pass


# ----------------------------------------------------------------------------
# Q1 lattices on the staggered grid
# ----------------------------------------------------------------------------

def lattice(faces, d: int):
    """Node coordinates of velocity component d's Q1 lattice, per axis.

    Staggered grid (Section 2.2): component d sits on the cell faces normal
    to axis d, i.e. at the face coordinates along axis d and at the cell
    centres (face midpoints) along the other two axes."""
    out = []
    for e in range(3):
        f = np.asarray(faces[e], dtype=np.float64)
        out.append(f.copy() if e == d else 0.5 * (f[:-1] + f[1:]))
    return out


def lattice_shape(faces, d: int):
    """(n_x, n_y, n_z) nodes of component d's lattice."""
    return tuple(len(a) for a in lattice(faces, d))


def n_fluid(faces, d: int) -> int:
    nx, ny, nz = lattice_shape(faces, d)
    return nx * ny * nz


def hat_1d(nodes, x):
    """All 1D piecewise-linear hats of `nodes` evaluated at points x:
    returns (len(x), len(nodes)).  Outside the node hull they are 0."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    H = np.zeros((x.size, nodes.size))
    for k in range(nodes.size):
        if k > 0:
            m = (x >= nodes[k - 1]) & (x <= nodes[k])
            H[m, k] = (x[m] - nodes[k - 1]) / (nodes[k] - nodes[k - 1])
        if k < nodes.size - 1:
            m = (x >= nodes[k]) & (x <= nodes[k + 1])
            H[m, k] = np.maximum(H[m, k], (nodes[k + 1] - x[m]) / (nodes[k + 1] - nodes[k]))
    return H


# ----------------------------------------------------------------------------
# P1 geometry
# ----------------------------------------------------------------------------

def tet_volumes(X, tets):
    X = np.asarray(X, dtype=np.float64)
    a = X[tets[:, 1]] - X[tets[:, 0]]
    b = X[tets[:, 2]] - X[tets[:, 0]]
    c = X[tets[:, 3]] - X[tets[:, 0]]
    return np.abs(np.einsum("ij,ij->i", a, np.cross(b, c))) / 6.0


def barycentric_gradients(X, tets):
    """grad λ_a per tet: (n_t, 4, 3), from the inverse of [1 x y z] rows."""
    X = np.asarray(X, dtype=np.float64)
    n_t = tets.shape[0]
    A = np.ones((n_t, 4, 4))
    A[:, :, 1:] = X[tets]
    inv = np.linalg.inv(A)            # column a = coefficients of λ_a
    return np.transpose(inv[:, 1:, :], (0, 2, 1))


def lumped_mass(X, tets, n_vert=None):
    """m_i = ∫ λ_i = Σ_{T∋i} |T|/4 (row sums of the P1 mass matrix)."""
    n_vert = X.shape[0] if n_vert is None else n_vert
    v = tet_volumes(X, tets)
    m = np.zeros(n_vert)
    for k in range(4):
        np.add.at(m, tets[:, k], v / 4.0)
    return m


def consistent_mass(X, tets, n_vert=None):
    """P1 mass matrix M_ij = ∫ λ_j λ_i (Section 2.1): |T|(1+δ_il)/20 per tet."""
    n_vert = X.shape[0] if n_vert is None else n_vert
    v = tet_volumes(X, tets)
    rows, cols, vals = [], [], []
    for i in range(4):
        for l in range(4):
            rows.append(tets[:, i])
            cols.append(tets[:, l])
            vals.append(v * (2.0 if i == l else 1.0) / 20.0)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n_vert, n_vert))


# ----------------------------------------------------------------------------
# Pairs (tet, component, cell) and the coupling matrices
# ----------------------------------------------------------------------------

@dataclass
class Pairs:
    subset: np.ndarray
    counts: np.ndarray          # (n_sub*3,)
    offsets: np.ndarray         # (n_sub*3+1,)
    ranges: np.ndarray          # (n_sub*3, 6)
    vals: np.ndarray            # (n_pairs, 32)
    vols: np.ndarray            # (n_pairs,)
    keep: np.ndarray            # (n_pairs,) bool
    cell: np.ndarray            # (n_pairs, 3)
    G: np.ndarray | None        # (n_pairs, 12)
    zero_tets: int
    seconds: float = 0.0

    def owner(self):
        """(subset position, component) of every pair."""
        sd = np.repeat(np.arange(self.counts.size), self.counts)
        return sd // 3, sd % 3


def _lat_arrays(faces):
    lats = [lattice(faces, d) for d in range(3)]
    flat = [np.ascontiguousarray(lats[d][e]) for d in range(3) for e in range(3)]
    ptrs = (ctypes.POINTER(ctypes.c_double) * 9)(*[_dp(a) for a in flat])
    nlat = np.array([a.size for a in flat], dtype=np.int64)
    return flat, ptrs, nlat


def pairs(faces, X, tets, subset=None, drop_rel=DROP_REL, nthreads=0, z=None, u_f=None,
          dual=False):
    """Integrate every (tet, component, cell) pair of the selected tets."""
    lib = _load()
    X = np.ascontiguousarray(X, dtype=np.float64)
    tets = np.ascontiguousarray(tets, dtype=np.int32)
    subset = (np.arange(tets.shape[0], dtype=np.int64) if subset is None
              else np.ascontiguousarray(subset, dtype=np.int64))
    flat, ptrs, nlat = _lat_arrays(faces)
    n_sub = subset.size
    counts = np.zeros(n_sub * 3, dtype=np.int64)
    ranges = np.zeros((n_sub * 3, 6), dtype=np.int32)
    st = lib.o1_pair_counts(ptrs, _i64p(nlat), _dp(X), _i32p(tets), _i64p(subset), n_sub,
                            _i64p(counts), _i32p(ranges))
    if st == -2:
        raise OutOfGrid("a tetrahedron's bounding box leaves a velocity lattice")
    offsets = np.zeros(n_sub * 3 + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    n_pairs = int(offsets[-1])
    vals = np.zeros((n_pairs, 32))
    vols = np.zeros(n_pairs)
    keep = np.zeros(n_pairs, dtype=np.uint8)
    cell = np.zeros((n_pairs, 3), dtype=np.int32)
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
        G = np.zeros((n_pairs, 12))
        zp = _dp(zc)
        up = (ctypes.POINTER(ctypes.c_double) * 3)(*[_dp(a) for a in uc])
        Gp = _dp(G)
    t0 = time.perf_counter()
    lib.o1_pairs(ptrs, _i64p(nlat), _dp(X), X.shape[0], _i32p(tets), _i64p(subset), n_sub,
                 _i32p(ranges), _i64p(offsets), float(drop_rel), int(nthreads), _dp(vals),
                 _dp(vols), keep.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), _i32p(cell),
                 zp, up, Gp, _i64p(zt), int(bool(dual)))
    dt = time.perf_counter() - t0
    return Pairs(subset, counts, offsets, ranges, vals, vols, keep.astype(bool), cell, G,
                 int(zt[0]), dt)


@dataclass
class Coupling:
    """B^d (n_vert x n_f,d, CSR) for d = 0, 1, 2 plus what produced them."""
    faces: list
    X: np.ndarray
    tets: np.ndarray
    B: list
    pairs: Pairs
    stats: dict = field(default_factory=dict)
    dual: bool = False

    @property
    def n_vert(self):
        return self.X.shape[0]


def assemble(faces, X, tets, subset=None, drop_rel=DROP_REL, nthreads=0, dual=False) -> Coupling:
    """Mortar matrices B^d_ij = ∫ λ_i N^d_j over the selected tets (all tets
    by default); with dual=True, B^d_ij = ∫ ψ_i N^d_j with the dual
    multipliers ψ_i = 5λ_i − 1 = Σ_k (5δ_ik − 1) λ_k of each tet, so a
    piece's values are 5·b_i − Σ_k b_k of its λ products b.  Rows of
    vertices not touched by the subset are zero."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    tets = np.ascontiguousarray(tets, dtype=np.int32)
    P = pairs(faces, X, tets, subset, drop_rel, nthreads)
    pvals = P.vals
    if dual:
        b = P.vals.reshape(-1, 4, 8)
        pvals = (5.0 * b - b.sum(axis=1, keepdims=True)).reshape(-1, 32)
    s_idx, comp = P.owner()
    t_idx = P.subset[s_idx]
    B = []
    for d in range(3):
        nx, ny, nz = lattice_shape(faces, d)
        sel = np.nonzero((comp == d) & P.keep)[0]
        tv = tets[t_idx[sel]]                                     # (k, 4)
        c = P.cell[sel].astype(np.int64)
        rows = np.repeat(tv, 8, axis=1).reshape(-1)               # i major, corner minor
        corner = np.arange(8)
        a, b, cc = corner & 1, (corner >> 1) & 1, (corner >> 2) & 1
        node = ((c[:, 0:1] + a) + nx * ((c[:, 1:2] + b) + ny * (c[:, 2:3] + cc)))  # (k, 8)
        cols = np.tile(node, (1, 4)).reshape(-1)
        vals = pvals[sel].reshape(-1)
        B.append(sp.csr_matrix((vals, (rows, cols)), shape=(X.shape[0], nx * ny * nz)))
    stats = dict(pairs=int(P.offsets[-1]), pieces=int(P.keep.sum()),
                 dropped=int(((P.vols > 0) & ~P.keep).sum()), zero_tets=P.zero_tets,
                 seconds=P.seconds)
    return Coupling(list(faces), X, tets, B, P, stats, dual)


def vertex_star(tets, vertices):
    """Indices of the tets incident to any of `vertices`."""
    mask = np.isin(tets, np.asarray(vertices)).any(axis=1)
    return np.nonzero(mask)[0]


def tet_bounds(X, tets):
    """Per-tet bounding boxes (mn, mx), each (n_t, 3)."""
    P = np.asarray(X)[tets]
    return P.min(axis=1), P.max(axis=1)


def tets_touching_node(faces, X, tets, d, node_ijk, bounds=None):
    """Tets whose bounding box meets the support of fluid node (i,j,k) of
    component d (a superset of those contributing to that column)."""
    lat = lattice(faces, d)
    lo = np.empty(3)
    hi = np.empty(3)
    for e in range(3):
        k = node_ijk[e]
        lo[e] = lat[e][max(k - 1, 0)]
        hi[e] = lat[e][min(k + 1, lat[e].size - 1)]
    mn, mx = tet_bounds(X, tets) if bounds is None else bounds
    ok = np.all((mx >= lo) & (mn <= hi), axis=1)
    return np.nonzero(ok)[0]


# ----------------------------------------------------------------------------
# Transfers (Section 2.3) and their adjoints
# ----------------------------------------------------------------------------

def mass_solve(X, tets, rhs, mass: str):
    """S^{-1} rhs for each row of rhs (3, n_vert): lumped or consistent (direct)."""
    rhs = np.atleast_2d(rhs)
    if mass == "lumped":
        return rhs / lumped_mass(X, tets)[None, :]
    if mass == "consistent":
        M = consistent_mass(X, tets).tocsc()
        lu = spla.splu(M)
        return np.stack([lu.solve(r) for r in rhs])
    raise ValueError(mass)


def _mass_of(cpl: Coupling, mass: str) -> str:
    """The dual multipliers make S the lumped (diagonal) mass."""
    if cpl.dual:
        if mass == "consistent":
            raise ValueError("the dual basis has a diagonal S: use mass='lumped'")
        return "lumped"
    return mass


def transfer_velocity(cpl: Coupling, u_f, mass: str = "lumped"):
    """w_s = S^{-1} B v_f per component; u_f: 3 arrays of lattice shape
    (n_z, n_y, n_x).  Returns (3, n_vert)."""
    rhs = np.stack([cpl.B[d] @ np.asarray(u_f[d], dtype=np.float64).ravel() for d in range(3)])
    return mass_solve(cpl.X, cpl.tets, rhs, _mass_of(cpl, mass))


def transfer_force(cpl: Coupling, f_s, alpha: float = 1.0, load: bool = False, base=None):
    """f_f = base + alpha B^T f_s (f_s nodal density coefficients), or with
    load=True the literal transpose of the transfer operator on a load
    vector: alpha B^T S^{-1} f_s (consistent S).  Returns 3 flat arrays."""
    f_s = np.asarray(f_s, dtype=np.float64)
    if load:
        f_s = mass_solve(cpl.X, cpl.tets, f_s, "lumped" if cpl.dual else "consistent")
    out = []
    for d in range(3):
        r = alpha * (cpl.B[d].T @ f_s[d])
        if base is not None:
            r = r + np.asarray(base[d], dtype=np.float64).ravel()
        out.append(r)
    return out


def _shape_pair_terms(faces, X, tets, z, u_f, nthreads=0, dual=False):
    """Σ over pairs of the B shape-derivative terms, contracted with z (3,n_v)
    and u_f: returns (n_vert, 3)."""
    P = pairs(faces, X, tets, None, DROP_REL, nthreads, z=z, u_f=u_f, dual=dual)
    s_idx, _ = P.owner()
    t_idx = P.subset[s_idx]
    g = np.zeros((X.shape[0], 3))
    Gk = P.G.reshape(-1, 4, 3) * P.keep[:, None, None]
    for a in range(4):
        np.add.at(g, tets[t_idx, a], Gk[:, a, :])
    return g


def _mass_shape_term(X, tets, z, u_s, mass):
    """Σ_d z^T (∂S/∂X) u_s^d as (n_vert, 3): ∂|T|/∂X_a = |T| ∇λ_a."""
    vol = tet_volumes(X, tets)
    grad = barycentric_gradients(X, tets)                   # (n_t, 4, 3)
    s = np.zeros(tets.shape[0])
    for d in range(3):
        zl = z[d][tets]                                     # (n_t, 4)
        ul = u_s[d][tets]
        if mass == "consistent":
            s += (np.einsum("ti,ti->t", zl, ul) + zl.sum(1) * ul.sum(1)) / 20.0
        else:
            s += np.einsum("ti,ti->t", zl, ul) / 4.0
    g = np.zeros((X.shape[0], 3))
    for a in range(4):
        np.add.at(g, tets[:, a], (vol * s)[:, None] * grad[:, a, :])
    return g


def velocity_vjp(cpl: Coupling, u_f, g_us, mass: str = "lumped", nthreads=0):
    """Reverse mode of u_s = S^{-1} B u_f.  Returns (g_uf: 3 flat arrays,
    g_X: (n_vert, 3)).  z = S^{-1} g; g_uf = B^T z; g_X from the shape
    derivative of B (moving P1 hats over the fixed Q1 hats) minus that of S."""
    g_us = np.asarray(g_us, dtype=np.float64)
    mass = _mass_of(cpl, mass)
    z = mass_solve(cpl.X, cpl.tets, g_us, mass)
    u_s = transfer_velocity(cpl, u_f, mass)
    g_uf = [cpl.B[d].T @ z[d] for d in range(3)]
    gX = _shape_pair_terms(cpl.faces, cpl.X, cpl.tets, z, u_f, nthreads, cpl.dual)
    gX -= _mass_shape_term(cpl.X, cpl.tets, z, u_s, mass)
    return g_uf, gX


def force_vjp(cpl: Coupling, f_s, g_ff, alpha: float = 1.0, nthreads=0):
    """Reverse mode of f_f = alpha B^T f_s.  Returns (g_fs (3, n_vert), g_X)."""
    f_s = np.asarray(f_s, dtype=np.float64)
    g_fs = np.stack([alpha * (cpl.B[d] @ np.asarray(g_ff[d]).ravel()) for d in range(3)])
    gX = alpha * _shape_pair_terms(cpl.faces, cpl.X, cpl.tets, f_s, g_ff, nthreads, cpl.dual)
    return g_fs, gX


def velocity_loss(faces, X, tets, u_f, u_target, mass="lumped", dual=False):
    """L = 1/2 ||u_s - u_target||^2 with u_s = S^{-1} B u_f (reassembled at X)."""
    cpl = assemble(faces, X, tets, dual=dual)
    u_s = transfer_velocity(cpl, u_f, mass)
    r = u_s - u_target
    return 0.5 * float(np.sum(r * r))


# ----------------------------------------------------------------------------
# Fixed-point (Picard) coupling, Section 3 Steps 1-6
# ----------------------------------------------------------------------------

def fluid_lumped_volume(faces, d: int):
    """∫ N_j over the hull of component d's lattice for every node (the Q1
    lumped mass of the fluid lattice), shape (n_z, n_y, n_x): a product of
    1D hat integrals, each half the length of the node's neighbouring
    intervals."""
    w = []
    for L in lattice(faces, d):
        h = np.diff(L)
        we = np.zeros(L.size)
        we[:-1] += 0.5 * h
        we[1:] += 0.5 * h
        w.append(we)
    return np.einsum("k,j,i->kji", w[2], w[1], w[0])


def fsi_step(faces, X_ref, tets, u_hat0, v_f, solid, fluid, dt, alpha=1.0, eps_abs=0.0,
             eps_rel=1e-8, max_iter=50, mass="lumped", force_density=False, dual=False,
             f_prev=None):
    """One time step of the Picard iteration of Section 3, in the steps'
    order: T = S^{-1} B assembled at X_ref + u_hat0 and held for the step;
      1. w_s = T v_f;  2. u_hat = u_hat0 + dt w_s;  3. f_fsi = solid(u_hat);
      4. f_tilde = alpha T^T f_fsi = alpha B^T S^{-1} f_fsi (divided by the
         fluid nodes' lumped volume with force_density);
      5. v_f = fluid(f_tilde);
      6. stop when ||f_l − f_{l−1}||_inf < eps_abs (eq. AC) or that norm over
         ||f_1||_inf < eps_rel (eq. RC); f_0 = f_prev (zeros by default).
    solid and fluid are numpy callables.  Returns a dict with the last
    iteration's fields and the iteration count."""
    X = np.asarray(X_ref, dtype=np.float64) + np.asarray(u_hat0, dtype=np.float64).T
    cpl = assemble(faces, X, tets, dual=dual)
    S = _mass_of(cpl, mass)
    u_hat0 = np.asarray(u_hat0, dtype=np.float64)
    v = [np.asarray(a, dtype=np.float64).ravel().copy() for a in v_f]
    f_old = np.zeros_like(u_hat0) if f_prev is None else np.asarray(f_prev, dtype=np.float64)
    vols = [fluid_lumped_volume(faces, d).ravel() for d in range(3)] if force_density else None
    f1 = None
    out = {}
    for it in range(1, max_iter + 1):
        w_s = mass_solve(X, tets, np.stack([cpl.B[d] @ v[d] for d in range(3)]), S)
        u_hat = u_hat0 + dt * w_s
        f = np.asarray(solid(u_hat), dtype=np.float64)
        g = mass_solve(X, tets, f, S)
        f_tilde = [alpha * (cpl.B[d].T @ g[d]) for d in range(3)]
        if force_density:
            f_tilde = [f_tilde[d] / vols[d] for d in range(3)]
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

def int4(Y, f1, f2, f3, f4) -> float:
    """∫_τ f1 f2 f3 f4 for affine f_m given by vertex values (closed form)."""
    lib = _load()
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (Y, f1, f2, f3, f4)]
    return lib.o1_int4(*[_dp(a) for a in arrs])


def clip_volume(P, lo, hi) -> float:
    """Volume of tetrahedron P (4x3) ∩ box [lo, hi] (face-list clipping)."""
    lib = _load()
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (P, lo, hi)]
    return lib.o1_clip_volume(*[_dp(a) for a in arrs])
