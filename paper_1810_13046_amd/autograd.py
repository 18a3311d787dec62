"""torch.autograd forms of the two transfers (hand-written backward).

TransferVelocity:  u_s = S^{-1} B(X) u_f
    backward: z = S^{-1} g_us;  g_uf = B^T z;  g_X = shape derivative
TransferForce:     f_f = alpha B(X)^T f_s          (a new fluid field)
    backward: g_fs = alpha B g_ff;  g_X = alpha * shape derivative

Both call the C ABI (transfer_velocity / transfer_force and their
_vjp entry points); no numerical step runs in Python.  With dual=True the
multipliers are the dual basis of Section 2.3 (eq. biorth) and S is the
lumped mass.  With
recompute_B=True a 3D grid coupling is built without stored matrices
(IBVT_NO_STORE_B): the forward and the backward pass clip and integrate the
pieces again, so neither B, B^T nor any per-pair data is ever held (the
force-spreading products then add with atomics: equal to the stored form to
rounding, not bit for bit).  A planar coupling is instead freed after the
forward pass and assembled again from the saved X in the backward pass.  Planar couplings (two face
arrays, X (n_vert, 2), triangles) take two fluid components: pass
u_f = (u0, u1) and get two force arrays back.  An unstructured coupling
(Coupling(None, X, tets, fluid_mesh=...)) is passed as `coupling` (faces
None; fluid fields are nodal arrays of the fluid mesh); it is not
reassembled by recompute_B.
"""
from __future__ import annotations

import torch

from .ibvt import Coupling


class _Ctx:
    def __init__(self, faces, tets, precision, mass, rtol, maxit, dual=False):
        self.faces, self.tets, self.precision = faces, tets, precision
        self.mass, self.rtol, self.maxit, self.dual = mass, rtol, maxit, dual


def _coupling(meta, X, existing, store_B=True):
    if existing is not None:
        return existing
    return Coupling(meta.faces, X.detach().contiguous(), meta.tets, precision=meta.precision,
                    consistent=(meta.mass == "consistent"), dual=meta.dual, store_B=store_B)


def _matrix_free(meta, recompute, existing):
    """recompute_B on a 3D grid: a coupling that keeps no matrices, held
    between the passes (it holds per-tet data only)."""
    return recompute and existing is None and meta.faces is not None and len(meta.faces) == 3


class TransferVelocity(torch.autograd.Function):
    """u_s = TransferVelocity.apply(u_f0, u_f1, u_f2, X, faces, tets, precision,
    mass, rtol, maxit, coupling, recompute_B, dual) -> (nc, n_vert); u_f2 is
    None for a planar coupling."""

    @staticmethod
    def forward(ctx, u0, u1, u2, X, faces, tets, precision="fp64", mass="lumped", rtol=1e-12,
                maxit=500, coupling=None, recompute_B=False, dual=False):
        meta = _Ctx(faces, tets, precision, mass, rtol, maxit, dual)
        mf = _matrix_free(meta, recompute_B, coupling)
        c = _coupling(meta, X, coupling, store_B=not mf)
        u = [v.contiguous() for v in (u0, u1, u2) if v is not None]
        us = c.velocity(u, mass=mass, rtol=rtol, maxit=maxit)
        ctx.meta = meta
        ctx.nc = len(u)
        ctx.recompute = recompute_B and coupling is None and not mf
        ctx.coupling = None if ctx.recompute else c
        ctx.save_for_backward(X, us, *u)
        if ctx.recompute:
            c.free()
        return us

    @staticmethod
    def backward(ctx, g_us):
        X, us, *u = ctx.saved_tensors
        meta = ctx.meta
        c = ctx.coupling if ctx.coupling is not None else _coupling(meta, X, None)
        need_u = any(ctx.needs_input_grad[:3])
        need_X = ctx.needs_input_grad[3]
        g_uf = [torch.zeros_like(v) for v in u] if need_u else None
        g_X = (torch.zeros((X.shape[0], X.shape[1]), dtype=torch.float64, device=X.device)
               if need_X else None)
        c.velocity_vjp(g_us.contiguous().to(us.dtype), u_f=u, u_s=us, mass=meta.mass, g_uf=g_uf,
                       g_X=g_X, rtol=meta.rtol, maxit=meta.maxit)
        if ctx.coupling is None:
            c.free()
        gu = (g_uf if need_u else []) + [None] * (3 - (ctx.nc if need_u else 0))
        return (gu[0], gu[1], gu[2], g_X.to(X.dtype) if need_X else None,
                None, None, None, None, None, None, None, None, None)


class TransferForce(torch.autograd.Function):
    """f_f = TransferForce.apply(f_s, X, faces, tets, precision, alpha,
    coupling, recompute_B, dual) -> tuple of nc fluid arrays."""

    @staticmethod
    def forward(ctx, f_s, X, faces, tets, precision="fp64", alpha=1.0, coupling=None,
                recompute_B=False, dual=False):
        meta = _Ctx(faces, tets, precision, "lumped", 1e-12, 500, dual)
        mf = _matrix_free(meta, recompute_B, coupling)
        c = _coupling(meta, X, coupling, store_B=not mf)
        out = [torch.zeros(s, dtype=c.dtype, device=f_s.device) for s in
               [tuple(reversed(ls)) for ls in c.lattice_shapes]]
        c.force(f_s.contiguous(), out, alpha=alpha)
        ctx.meta = meta
        ctx.alpha = alpha
        ctx.recompute = recompute_B and coupling is None and not mf
        ctx.coupling = None if ctx.recompute else c
        ctx.save_for_backward(f_s, X)
        if ctx.recompute:
            c.free()
        return tuple(out)

    @staticmethod
    def backward(ctx, *grads):
        f_s, X = ctx.saved_tensors
        c = ctx.coupling if ctx.coupling is not None else _coupling(ctx.meta, X, None)
        g_ff = []
        for g, s in zip(grads, c.lattice_shapes):
            g_ff.append(torch.zeros(tuple(reversed(s)), dtype=c.dtype, device=X.device)
                        if g is None else g.contiguous().to(c.dtype))
        g_fs = torch.zeros_like(f_s) if ctx.needs_input_grad[0] else None
        g_X = (torch.zeros((X.shape[0], X.shape[1]), dtype=torch.float64, device=X.device)
               if ctx.needs_input_grad[1] else None)
        c.force_vjp(g_ff, f_s=f_s.contiguous(), alpha=ctx.alpha, g_fs=g_fs, g_X=g_X)
        if ctx.coupling is None:
            c.free()
        return (g_fs, g_X.to(X.dtype) if g_X is not None else None,
                None, None, None, None, None, None, None)


def transfer_velocity(u_f, X, faces, tets, precision="fp64", mass="lumped", rtol=1e-12,
                      maxit=500, coupling=None, recompute_B=False, dual=False):
    u2 = u_f[2] if len(u_f) > 2 else None
    return TransferVelocity.apply(u_f[0], u_f[1], u2, X, faces, tets, precision, mass, rtol,
                                  maxit, coupling, recompute_B, dual)


def transfer_force(f_s, X, faces, tets, precision="fp64", alpha=1.0, coupling=None,
                   recompute_B=False, dual=False):
    return TransferForce.apply(f_s, X, faces, tets, precision, alpha, coupling, recompute_B,
                               dual)
