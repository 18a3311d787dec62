"""FP64 CPU oracle of the coupling with an unstructured background mesh: a
P1 tetrahedral fluid mesh against the P1 tetrahedral solid mesh.

TEST INFRASTRUCTURE ONLY, like the rest of this package.

Section 2.3 assembles the transfer for meshes that need not be structured:
(I) the overlapping elements are found by a tree search, (II)-(III) the
products of the two element bases are integrated on the intersections
(piecewise affine meshes), (IV) the mortar matrices are assembled.  Here
the fluid space is P1 on the fluid tets (collocated: every velocity
component uses the same nodes and the same B):

* candidate pairs: every (solid tet, fluid tet) with overlapping bounding
  boxes (a k-d tree ball query on the box centres gives a superset, the
  exact box test filters it; the GPU builds its own bounding-volume tree);
* B_ij = ∫ λ_i μ_j dV per pair (C part, o3.c), summed;
* S, the transfers and the dual multipliers as in the structured case
  (oracle/__init__.py);
* reverse mode: z = S^{-1} g, B^T z, and the shape derivative with respect
  to the solid vertices (the transport form of the structured case with the
  fluid P1 hats in place of the Q1 hats; ∫ λ_a λ_i per piece is the second
  integral it needs);
* the Picard step of Section 3 over this coupling (fsi_step).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

from . import (DROP_REL, _mass_shape_term, barycentric_gradients, consistent_mass, lumped_mass,
               mass_solve, tet_volumes)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "o3.c")
_LIB = os.path.join(_HERE, "_o3.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C part with gcc (plain C, OpenMP)."""
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
        lib.o3_pairs.argtypes = [dp, i32p, dp, i32p, i64p, ctypes.c_int64, ctypes.c_double,
                                 ctypes.c_int, dp, dp, dp, P(ctypes.c_uint8)]
        lib.o3_pairs.restype = ctypes.c_int
        lib.o3_clip_volume.argtypes = [dp, dp]
        lib.o3_clip_volume.restype = ctypes.c_double
        lib.o3_int2.argtypes = [dp, dp, dp]
        lib.o3_int2.restype = ctypes.c_double
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def tet_bounds(X, tets):
    P = np.asarray(X)[tets]
    return P.min(axis=1), P.max(axis=1)


def candidate_pairs(Xs, tets_s, Xf, tets_f):
    """(solid tet, fluid tet) pairs with overlapping closed bounding boxes,
    sorted by solid tet then fluid tet.  Boxes that overlap have centres
    closer than the sum of their half-diagonals, so a k-d tree ball query on
    the fluid box centres gives a superset, which the exact box test then
    filters."""
    from scipy.spatial import cKDTree
    mns, mxs = tet_bounds(Xs, tets_s)
    mnf, mxf = tet_bounds(Xf, tets_f)
    cs, cf = 0.5 * (mns + mxs), 0.5 * (mnf + mxf)
    hs = 0.5 * np.linalg.norm(mxs - mns, axis=1)
    hf = 0.5 * np.linalg.norm(mxf - mnf, axis=1)
    tree = cKDTree(cf)
    out = []
    for s in range(tets_s.shape[0]):
        cand = np.asarray(tree.query_ball_point(cs[s], hs[s] + hf.max() + 1e-12), dtype=np.int64)
        ok = np.all((mxs[s] >= mnf[cand]) & (mns[s] <= mxf[cand]), axis=1)
        f = np.sort(cand[ok])
        out.append(np.stack([np.full(f.size, s, dtype=np.int64), f], axis=1))
    if not out:
        return np.zeros((0, 2), dtype=np.int64)
    return np.ascontiguousarray(np.concatenate(out))


@dataclass
class Coupling:
    """B (n_vert_solid x n_vert_fluid, CSR) plus what produced it."""
    Xf: np.ndarray
    tets_f: np.ndarray
    X: np.ndarray
    tets: np.ndarray
    B: sp.csr_matrix
    pairs: np.ndarray
    vals: np.ndarray
    keep: np.ndarray
    stats: dict = field(default_factory=dict)
    dual: bool = False


def pair_values(Xs, tets_s, Xf, tets_f, pairs, drop_rel=DROP_REL, nthreads=0, with_lam=False):
    """vals (n, 16): ∫ λ_i μ_j per pair (i*4 + j); vols; keep; and with
    with_lam also lams (n, 16): ∫ λ_a λ_i per pair (a*4 + i)."""
    lib = _load()
    Xs = np.ascontiguousarray(Xs, dtype=np.float64)
    Xf = np.ascontiguousarray(Xf, dtype=np.float64)
    ts = np.ascontiguousarray(tets_s, dtype=np.int32)
    tf = np.ascontiguousarray(tets_f, dtype=np.int32)
    pairs = np.ascontiguousarray(pairs, dtype=np.int64)
    n = pairs.shape[0]
    vals = np.zeros((n, 16))
    lams = np.zeros((n, 16)) if with_lam else None
    vols = np.zeros(n)
    keep = np.zeros(n, dtype=np.uint8)
    lib.o3_pairs(_dp(Xs), ts.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(Xf),
                 tf.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                 pairs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), n, float(drop_rel),
                 int(nthreads), _dp(vals), _dp(lams) if with_lam else None, _dp(vols),
                 keep.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    if with_lam:
        return vals, lams, vols, keep.astype(bool)
    return vals, vols, keep.astype(bool)


def assemble(Xf, tets_f, Xs, tets_s, drop_rel=DROP_REL, dual=False, nthreads=0) -> Coupling:
    """B_ij = ∫ λ_i μ_j (solid vertex i, fluid vertex j); with dual=True the
    dual multipliers ψ_i = 5λ_i − 1 of each solid tet (a piece's values
    become 5·b_i − Σ_k b_k)."""
    Xs = np.ascontiguousarray(Xs, dtype=np.float64)
    Xf = np.ascontiguousarray(Xf, dtype=np.float64)
    tets_s = np.ascontiguousarray(tets_s, dtype=np.int32)
    tets_f = np.ascontiguousarray(tets_f, dtype=np.int32)
    t0 = time.perf_counter()
    pairs = candidate_pairs(Xs, tets_s, Xf, tets_f)
    vals, vols, keep = pair_values(Xs, tets_s, Xf, tets_f, pairs, drop_rel, nthreads)
    pv = vals
    if dual:
        b = vals.reshape(-1, 4, 4)
        pv = (5.0 * b - b.sum(axis=1, keepdims=True)).reshape(-1, 16)
    sel = np.nonzero(keep)[0]
    rows = np.repeat(tets_s[pairs[sel, 0]], 4, axis=1).reshape(-1)       # i major
    cols = np.tile(tets_f[pairs[sel, 1]], (1, 4)).reshape(-1)            # j minor
    B = sp.csr_matrix((pv[sel].reshape(-1), (rows, cols)), shape=(Xs.shape[0], Xf.shape[0]))
    stats = dict(pairs=int(pairs.shape[0]), pieces=int(keep.sum()),
                 dropped=int(((vols > 0) & ~keep).sum()),
                 zero_tets=int((tet_volumes(Xs, tets_s) == 0).sum()),
                 seconds=time.perf_counter() - t0)
    return Coupling(Xf, tets_f, Xs, tets_s, B, pairs, vals, keep, stats, dual)


def transfer_velocity(cpl: Coupling, u_f, mass="lumped"):
    """w_s = S^{-1} B v_f for each component (u_f: (nc, n_vert_fluid))."""
    if cpl.dual and mass == "consistent":
        raise ValueError("the dual basis has a diagonal S: use mass='lumped'")
    u_f = np.atleast_2d(np.asarray(u_f, dtype=np.float64))
    rhs = np.stack([cpl.B @ u for u in u_f])
    return mass_solve(cpl.X, cpl.tets, rhs, "lumped" if cpl.dual else mass)


def transfer_force(cpl: Coupling, f_s, alpha=1.0, load=False, base=None):
    """f_f = base + alpha B^T f_s per component, or alpha B^T S^{-1} f_s."""
    f_s = np.atleast_2d(np.asarray(f_s, dtype=np.float64))
    if load:
        f_s = mass_solve(cpl.X, cpl.tets, f_s, "lumped" if cpl.dual else "consistent")
    out = alpha * np.stack([cpl.B.T @ f for f in f_s])
    if base is not None:
        out = out + np.asarray(base, dtype=np.float64)
    return out


def _mass_kind(cpl: Coupling, mass: str) -> str:
    if cpl.dual and mass == "consistent":
        raise ValueError("the dual basis has a diagonal S: use mass='lumped'")
    return "lumped" if cpl.dual else mass


def _shape_terms(cpl: Coupling, z, u):
    """Σ over the pieces of the shape-derivative terms of B contracted with
    the solid weights z (nc, n_vert) and the fluid nodal fields u (nc,
    n_vert_fluid), as (n_vert, 3).  Moving vertex a of a solid tet moves its
    points by λ_a e_k while the fluid hats μ_j stay where they are, so
        ∂B_ij/∂X_{a,k} = Σ_{T∋a} ∫_T (λ_a λ_i ∂_k μ_j + ∂_k λ_a λ_i μ_j)
    (the same transport form as for the grid).  On a piece inside fluid tet
    F the interpolant U = Σ_j u_j μ_j has the constant gradient Σ_j u_j ∇μ_j,
    so a piece adds ∂_k U · Σ_i z_i ∫ λ_a λ_i + ∂_k λ_a · Σ_ij z_i u_j ∫ λ_i μ_j.
    With dual multipliers the weights are 5 z_i − Σ_k z_k."""
    z = np.atleast_2d(np.asarray(z, dtype=np.float64))
    u = np.atleast_2d(np.asarray(u, dtype=np.float64))
    vals, lams, _, keep = pair_values(cpl.X, cpl.tets, cpl.Xf, cpl.tets_f, cpl.pairs, with_lam=True)
    sel = np.nonzero(keep)[0]
    ps, pf = cpl.pairs[sel, 0], cpl.pairs[sel, 1]
    V = vals[sel].reshape(-1, 4, 4)                       # [p, i, j]
    L = lams[sel].reshape(-1, 4, 4)                       # [p, a, i]
    grad_l = barycentric_gradients(cpl.X, cpl.tets)[ps]   # [p, a, k]
    grad_m = barycentric_gradients(cpl.Xf, cpl.tets_f)[pf]
    vs, vf = cpl.tets[ps], cpl.tets_f[pf]
    g = np.zeros((cpl.X.shape[0], 3))
    for d in range(z.shape[0]):
        zl = z[d][vs]
        if cpl.dual:
            zl = 5.0 * zl - zl.sum(axis=1, keepdims=True)
        ul = u[d][vf]
        grad_u = np.einsum("pj,pjk->pk", ul, grad_m)
        zL = np.einsum("pi,pai->pa", zl, L)
        zVu = np.einsum("pi,pij,pj->p", zl, V, ul)
        term = zL[:, :, None] * grad_u[:, None, :] + grad_l * zVu[:, None, None]
        for a in range(4):
            np.add.at(g, vs[:, a], term[:, a, :])
    return g


def velocity_vjp(cpl: Coupling, u_f, g_us, mass="lumped"):
    """Reverse mode of u_s = S^{-1} B(X) u_f: z = S^{-1} g_us; returns
    (g_uf = B^T z per component, g_X = Σ_d z_d^T (∂B/∂X) u_f,d − Σ_d z_d^T
    (∂S/∂X) u_s,d)."""
    mk = _mass_kind(cpl, mass)
    z = mass_solve(cpl.X, cpl.tets, np.atleast_2d(np.asarray(g_us, dtype=np.float64)), mk)
    u_f = np.atleast_2d(np.asarray(u_f, dtype=np.float64))
    u_s = transfer_velocity(cpl, u_f, mass)
    g_uf = np.stack([cpl.B.T @ zd for zd in z])
    g_X = _shape_terms(cpl, z, u_f) - _mass_shape_term(cpl.X, cpl.tets, z, u_s, mk)
    return g_uf, g_X


def force_vjp(cpl: Coupling, f_s, g_ff, alpha=1.0):
    """Reverse mode of f_f = alpha B(X)^T f_s: returns (g_fs = alpha B g_ff,
    g_X = alpha Σ_d f_s,d^T (∂B/∂X) g_ff,d)."""
    f_s = np.atleast_2d(np.asarray(f_s, dtype=np.float64))
    g_ff = np.atleast_2d(np.asarray(g_ff, dtype=np.float64))
    g_fs = alpha * np.stack([cpl.B @ g for g in g_ff])
    return g_fs, alpha * _shape_terms(cpl, f_s, g_ff)


def velocity_loss(Xf, tets_f, X, tets, u_f, u_target, mass="lumped", dual=False):
    """L = 1/2 ||u_s − u_target||^2 with u_s = S^{-1} B u_f assembled at X."""
    cpl = assemble(Xf, tets_f, X, tets, dual=dual)
    r = transfer_velocity(cpl, u_f, mass) - u_target
    return 0.5 * float(np.sum(r * r))


def fsi_step(Xf, tets_f, X_ref, tets, u_hat0, v_f, solid, fluid, dt, alpha=1.0, eps_abs=0.0,
             eps_rel=1e-8, max_iter=50, mass="lumped", force_density=False, dual=False,
             f_prev=None):
    """One time step of the Picard iteration of Section 3 with the P1 fluid
    mesh as the background, in the steps' order: T = S^{-1} B assembled at
    X_ref + u_hat0 and held for the step; 1. w_s = T v_f; 2. u_hat = u_hat0
    + dt w_s; 3. f_fsi = solid(u_hat); 4. f_tilde = alpha B^T S^{-1} f_fsi
    (divided by the fluid nodes' lumped volume ∫ μ_j with force_density);
    5. v_f = fluid(f_tilde); 6. stop when ||f_l − f_{l−1}||_inf < eps_abs or
    that over ||f_1||_inf < eps_rel; f_0 = f_prev (zeros by default).
    v_f: three nodal arrays of the fluid mesh."""
    X = np.asarray(X_ref, dtype=np.float64) + np.asarray(u_hat0, dtype=np.float64).T
    cpl = assemble(Xf, tets_f, X, tets, dual=dual)
    S = _mass_kind(cpl, mass)
    u_hat0 = np.asarray(u_hat0, dtype=np.float64)
    v = [np.asarray(a, dtype=np.float64).ravel().copy() for a in v_f]
    f_old = np.zeros_like(u_hat0) if f_prev is None else np.asarray(f_prev, dtype=np.float64)
    vol = lumped_mass(Xf, tets_f, Xf.shape[0]) if force_density else None
    f1 = None
    out = {}
    for it in range(1, max_iter + 1):
        w_s = mass_solve(X, tets, np.stack([cpl.B @ v[d] for d in range(3)]), S)
        u_hat = u_hat0 + dt * w_s
        f = np.asarray(solid(u_hat), dtype=np.float64)
        g = mass_solve(X, tets, f, S)
        f_tilde = [alpha * (cpl.B.T @ g[d]) for d in range(3)]
        if force_density:
            # a fluid vertex no tet touches has no volume and receives no
            # load; its density is taken as zero
            f_tilde = [np.divide(f_tilde[d], vol, out=np.zeros_like(f_tilde[d]), where=vol > 0)
                       for d in range(3)]
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


def clip_volume(S, F) -> float:
    lib = _load()
    a = np.ascontiguousarray(S, dtype=np.float64)
    b = np.ascontiguousarray(F, dtype=np.float64)
    return lib.o3_clip_volume(_dp(a), _dp(b))


def int2(Y, f, g) -> float:
    lib = _load()
    arrs = [np.ascontiguousarray(x, dtype=np.float64) for x in (Y, f, g)]
    return lib.o3_int2(*[_dp(x) for x in arrs])


__all__ = ["build", "candidate_pairs", "Coupling", "pair_values", "assemble",
           "transfer_velocity", "transfer_force", "velocity_vjp", "force_vjp", "velocity_loss",
           "clip_volume", "int2", "tet_bounds", "lumped_mass", "consistent_mass"]
