#!/usr/bin/env python3
"""Throughput of the L2-projection transfer hot path on one MI355X.

Workload (default): the large three-body case on a 512 x 256 x 256
staggered grid, y-stretched (ratio 4) about y = 1/2, domain [0,2]x[0,1]x[0,1];
beam 1,975,392 + plate 1,500,282 + curved shell 1,027,728 = 4,503,402 P1
tets, 832,517 vertices, assembled in one launch sequence.  Inputs are seeded
and synthetic (see workloads/gen.py), resident in HBM before timing.

One step = the whole hot path on that input:
  reassemble B^d (all three velocity lattices) for the current positions,
  velocity transfer with the consistent mass (solved to 1e-10),
  force transfer,
  reverse mode of both transfers (fluid cotangents and the shape gradient).
The headline `value` is solid tets per second of that step in the
mixed-precision path (double clipping, float quadrature and applies); the
same step in FP64 is reported beside it.

Also reported (not the headline): the same step with the dual multipliers,
one Picard coupling step, and the planar coupling (Q1 quadrilateral lattice
x P1 triangles) on the Turek–Hron-like reference mesh (43,824 triangles in a
4608 x 762 grid, workloads/plane.py) in both precisions, with the 2D oracle
timed on the same step.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_VEC_PEAK_TFLOPS = 157.3
FP64_VEC_PEAK_TFLOPS = 78.6

# Algorithmic FP64 flops of the clip step (double arithmetic only; the
# vertex graph bookkeeping is integer work and not counted):
#   signed distance of a vertex to a plane       2  (subtract, sign)
#   cut point on an edge                        11  (t = s_v/(s_v - s_u): 2;
#                                                    p = v + t(u - v): 3 x 3)
#   sub-tetrahedron record                      47  (12 cell-local coordinates
#                                                    x 2, determinant 23)
#   pair set-up                                 50  (cell box, λ in cell-local
#                                                    coordinates, drop test)
CLIP_FLOPS = dict(dist=2, cut=11, subtet=47, pair=50)
# The survey's pricing of the clip for the roofline: 150-300 FP64 flops per
# plane cut (one tet piece clipped by one cell plane: signed distances of its
# vertices, cut points, bookkeeping); the midpoint is reported as `frac`,
# the range beside it.
FLOPS_PER_PLANE_CUT = (150, 225, 300)
FLUSH_BYTES = 1 << 30   # cold-cache protocol: >= 1 GiB written between repetitions
# flops per quadrature point of the 32 piece moments: point 6, powers 6,
# partial products 12, 32 multiply-adds 64; 11 points (degree 4) per
# sub-tetrahedron
MOM_FLOPS_PER_POINT = 88
POINTS_PER_SUBTET = 11

# HBM traffic of the clip step (all launches of one assembly) on
# the three-body workload, from rocprofv3 FETCH_SIZE and WRITE_SIZE counter
# passes, scaled by the copy-kernel calibration (FETCH x 2, WRITE x 1): the
# summary and its commands are in profiles/.  Reported only while the clip
# sources are the ones the counters were taken on.
CLIP_TRAFFIC = dict(sources_sha256="3800264d4994daa2c74c70a25de4942cd18f307be5a10b65554dee672c5342f0",
                    bytes_mixed=25436929408)
CLIP_SOURCES = ["paper_1810_13046_amd/csrc/assemble.hip", "paper_1810_13046_amd/csrc/geometry.hpp",
                "paper_1810_13046_amd/csrc/common.hpp"]
# HBM traffic of one lumped velocity apply and one force apply (all three
# components, mixed precision) on the three-body workload, from the same
# counter passes (profiles/hbm_traffic_three_bodies4.5M_mixed.txt);
# reported while apply.hip is the source they were taken on.
APPLY_TRAFFIC = dict(sources_sha256="2364d30cd6bae5f50fd603c4ed7fdc3e6a156ff37b34dcc7efd560032113be06",
                     velocity_bytes=972426558, force_bytes=980883005)
APPLY_SOURCES = ["paper_1810_13046_amd/csrc/apply.hip"]


def sources_sha256(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_inputs(cfg, dev):
    import torch
    import workloads as wl
    from paper_1810_13046_amd import lattice_coords
    t0 = time.time()
    W = wl.workload(cfg)
    k, phi = wl.fourier_modes(W.n_modes, W.kmax, 2000 + cfg)
    u64 = []
    for d in range(3):
        xs, ys, zs = lattice_coords(W.faces, d)
        u64.append(wl.fourier_field(k[d], phi[d], xs, ys, zs, device=dev).contiguous())
    X = torch.as_tensor(W.X, device=dev).contiguous()
    T = torch.as_tensor(W.tets, device=dev).contiguous()
    f_s = torch.as_tensor(W.f_s(), device=dev).contiguous()
    u_t = torch.as_tensor(W.u_target(), device=dev).contiguous()
    torch.cuda.synchronize()
    log(f"[bench] inputs for workload {cfg} ({W.name}) in {time.time() - t0:.1f}s: "
        f"{W.tets.shape[0]} tets, {W.X.shape[0]} vertices, grid {W.n_cells}")
    return W, X, T, u64, f_s, u_t


class Step:
    """Buffers and one full pass of the hot path for one precision.  With
    dual=True the multipliers are the dual basis (S = lumped mass), so the
    velocity transfer and its adjoint need no mass solve."""

    def __init__(self, W, X, T, u64, f_s, u_t, precision, dual=False, store_B=True):
        import torch
        from paper_1810_13046_amd import Coupling
        self.dual = dual
        self.mass = "lumped" if dual else "consistent"
        self.c = Coupling(W.faces, X, T, precision=precision, consistent=not dual, dual=dual,
                          store_B=store_B)
        dt = self.c.dtype
        self.X = X
        self.u = [u.to(dt).contiguous() for u in u64]
        self.f_s = f_s.to(dt).contiguous()
        self.u_t = u_t.to(dt).contiguous()
        self.us = torch.empty((self.c.nc, X.shape[0]), dtype=dt, device=X.device)
        self.ff = [torch.zeros_like(u) for u in self.u]
        self.g_uf = [torch.zeros_like(u) for u in self.u]
        self.g_fs = torch.zeros_like(self.f_s)
        self.g_X = torch.zeros((X.shape[0], X.shape[1]), dtype=torch.float64, device=X.device)

    def run(self):
        c = self.c
        c.reassemble(self.X)
        c.velocity(self.u, mass=self.mass, rtol=1e-10, maxit=500, out=self.us)
        c.force(self.f_s, self.ff, alpha=1.0)
        g_us = self.us - self.u_t
        # both adjoints (velocity: cotangent g_us; force: cotangent u_f) in
        # one call, so their shape terms share one pass over the moments
        c.vjp(g_us, self.u, u_f=self.u, u_s=self.us, f_s=self.f_s, mass=self.mass, alpha=1.0,
              g_uf=self.g_uf, g_fs=self.g_fs, g_X=self.g_X, rtol=1e-10, maxit=500)


def make_inputs_planar(dev):
    """The Turek–Hron-like reference mesh and grid (workloads/plane.py)."""
    import torch
    import workloads as wl
    from paper_1810_13046_amd import lattice_coords
    P2 = wl.plane
    W = P2.workload2(5)
    k, phi = P2.fourier_modes2(W.n_modes, W.kmax, 2100 + W.key)
    u64 = [torch.as_tensor(P2.fourier_field2(k[d], phi[d], *lattice_coords(W.faces, d),
                                             scale=W.extent), device=dev).contiguous()
           for d in range(2)]
    X = torch.as_tensor(W.X, device=dev).contiguous()
    T = torch.as_tensor(W.tris, device=dev).contiguous()
    f_s = torch.as_tensor(W.f_s(), device=dev).contiguous()
    u_t = torch.as_tensor(W.u_target(), device=dev).contiguous()
    torch.cuda.synchronize()
    return W, X, T, u64, f_s, u_t


def planar_oracle_step(W):
    """The 2D oracle on the same step (assembly, consistent velocity by sparse
    LU, force, both adjoints): seconds for the whole mesh."""
    from oracle import plane as pl
    import workloads as wl
    P2 = wl.plane
    k, phi = P2.fourier_modes2(W.n_modes, W.kmax, 2100 + W.key)
    u = [P2.fourier_field2(k[d], phi[d], *pl.lattice(W.faces, d), scale=W.extent)
         for d in range(2)]
    t0 = time.perf_counter()
    cpl = pl.assemble(W.faces, W.X, W.tris)
    us = pl.transfer_velocity(cpl, u, "consistent")
    pl.transfer_force(cpl, W.f_s(), 1.0)
    pl.velocity_vjp(cpl, u, us - W.u_target(), "consistent")
    pl.force_vjp(cpl, W.f_s(), [a.ravel() for a in u], 1.0)
    return time.perf_counter() - t0


def planar_leg(dev, steps, warmup, with_cpu):
    W, X, T, u64, f_s, u_t = make_inputs_planar(dev)
    n_tri = W.tris.shape[0]
    out = dict(workload=W.name, n_tri=int(n_tri), n_vert=int(W.X.shape[0]),
               grid_cells=list(W.n_cells), unit="solid triangles/s (same step as 3D)")
    for prec in ("fp32", "fp64"):
        log(f"[bench] planar {prec} step")
        st = Step(W, X, T, u64, f_s, u_t, prec)
        ms, wall = time_steps(st, steps, warmup)
        prof = kernel_profile(st)
        info = st.c.info()
        out[prec] = dict(ms_per_step=ms, wall_ms_per_step=wall, value=n_tri / (ms * 1e-3),
                         kernels_ms={k: v[1] for k, v in prof.items()},
                         kernel_launches={k: v[0] for k, v in prof.items()},
                         pairs=info["pairs"], pieces=info["pieces"], nnz=info["nnz"][:2])
        log(f"[bench] planar {prec} {ms:.3f} ms/step")
        del st
    if with_cpu:
        sec = planar_oracle_step(W)
        out["cpu_oracle"] = dict(value=n_tri / sec, seconds=sec, kind="oracle",
                                 cores=int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
                                 sample="the whole mesh, one step")
    return out


class UStep:
    """One pass over the unstructured coupling (P1 tetrahedral fluid mesh):
    reassembly against the kept fluid tree, consistent velocity transfer,
    force transfer and both adjoints with the shape gradient (the same step
    as on the grid)."""

    def __init__(self, W, X, T, Xf, Tf, u_f, f_s, precision):
        import torch
        from paper_1810_13046_amd import Coupling
        self.c = Coupling(None, X, T, precision=precision, consistent=True, fluid_mesh=(Xf, Tf))
        dt = self.c.dtype
        self.X = X
        self.u = [u.to(dt).contiguous() for u in u_f]
        self.f_s = f_s.to(dt).contiguous()
        self.us = torch.empty((3, X.shape[0]), dtype=dt, device=X.device)
        self.ff = [torch.zeros_like(u) for u in self.u]
        self.g_uf = [torch.zeros_like(u) for u in self.u]
        self.g_fs = torch.zeros_like(self.f_s)
        self.g_X = torch.zeros((X.shape[0], 3), dtype=torch.float64, device=X.device)

    def run(self):
        c = self.c
        c.reassemble(self.X)
        c.velocity(self.u, mass="consistent", rtol=1e-10, maxit=500, out=self.us)
        c.force(self.f_s, self.ff, alpha=1.0)
        c.vjp(self.us, self.u, u_f=self.u, u_s=self.us, f_s=self.f_s, mass="consistent",
              alpha=1.0, g_uf=self.g_uf, g_fs=self.g_fs, g_X=self.g_X, rtol=1e-10, maxit=500)


def unstructured_oracle_rate(W, n_sample):
    """The oracle's assembly (candidate search, clipping, integration, B) on
    the first n_sample solid tets of the same meshes: solid tets/s."""
    from oracle import unstructured as un
    un.build(force=False)
    t0 = time.perf_counter()
    un.assemble(W.Xf, W.tets_f, W.X, W.tets[:n_sample])
    return n_sample / (time.perf_counter() - t0)


def unstructured_leg(dev, steps, warmup, with_cpu):
    import torch
    import workloads as wl
    W = wl.unstructured.workload_u(3)
    X = torch.as_tensor(W.X, device=dev).contiguous()
    T = torch.as_tensor(W.tets, device=dev).contiguous()
    Xf = torch.as_tensor(W.Xf, device=dev).contiguous()
    Tf = torch.as_tensor(W.tets_f, device=dev).contiguous()
    u_f = [torch.as_tensor(u, device=dev).contiguous() for u in W.u_f()]
    f_s = torch.as_tensor(W.f_s(), device=dev).contiguous()
    n_tet = W.tets.shape[0]
    out = dict(workload=W.name, n_tet=int(n_tet), n_vert=int(W.X.shape[0]),
               fluid_tets=int(W.tets_f.shape[0]), fluid_vertices=int(W.Xf.shape[0]),
               unit="solid tets/s (reassembly + consistent velocity + force + both adjoints)")
    for prec in ("fp32", "fp64"):
        log(f"[bench] unstructured {prec} step")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = UStep(W, X, T, Xf, Tf, u_f, f_s, prec)
        torch.cuda.synchronize()
        first = (time.perf_counter() - t0) * 1e3
        ms, wall = time_steps(st, steps, warmup)
        prof = kernel_profile(st)
        info = st.c.info()
        out[prec] = dict(ms_per_step=ms, wall_ms_per_step=wall, value=n_tet / (ms * 1e-3),
                         first_assembly_with_tree_ms=first,
                         kernels_ms={k: v[1] for k, v in prof.items()},
                         kernel_launches={k: v[0] for k, v in prof.items()},
                         pairs=info["pairs"], pieces=info["pieces"], nnz=info["nnz"][0])
        log(f"[bench] unstructured {prec} {ms:.3f} ms/step")
        del st
    if with_cpu:
        n_sample = 3000
        rate = unstructured_oracle_rate(W, n_sample)
        out["cpu_oracle"] = dict(value=rate, kind="oracle", unit="solid tets/s (assembly only)",
                                 cores=int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
                                 sample=f"assembly of the first {n_sample} solid tets")
    return out


def time_steps(step, steps, warmup):
    import torch
    for _ in range(warmup):
        step.run()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for k in range(steps):
        step.run()
        log(f"[bench]   step {k + 1}/{steps}")
    e1.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps * 1e3
    return e0.elapsed_time(e1) / steps, wall


def kernel_profile(step):
    import torch
    from paper_1810_13046_amd import profile_enable, profile_read
    torch.cuda.synchronize()
    profile_read()
    profile_enable(True)
    step.run()
    torch.cuda.synchronize()
    prof = profile_read()
    profile_enable(False)
    return prof


def apply_bytes(c):
    """Algorithmic bytes of one lumped velocity apply and one force apply
    (three components): s value bytes, int32 indices, nnz_d nonzeros, t_d
    touched fluid nodes, n solid vertices."""
    info = c.info()
    s = 8 if c.precision == "fp64" else 4
    n = info["n_vert"]
    nnz, t = info["nnz"], info["touched"]
    vel = sum(nnz[d] * (s + 4) + 4 * (n + 1) + s * t[d] + s * n for d in range(3)) + s * n
    frc = sum(nnz[d] * (s + 4) + 4 * (t[d] + 1) + 4 * t[d] + 2 * s * t[d] + s * n
              for d in range(3))
    return vel, frc


def _one_launch_ms(run, name):
    """Device time of the library kernel `name` in one call of run()
    (HIP events the library records on its stream)."""
    from paper_1810_13046_amd import profile_enable, profile_read
    profile_read()
    profile_enable(True)
    run()
    prof = profile_read()
    profile_enable(False)
    launches, ms = prof[name]
    return ms / launches


def apply_rates(step, reps=20, warm=3):
    """Lumped velocity apply and force apply, ms per launch and GB/s of
    algorithmic bytes.  Cold: a >= 1 GiB write between repetitions evicts
    the caches, 3 warm-ups, median of `reps`; warm: back to back, median of
    `reps`."""
    import torch
    c = step.c
    vel_bytes, frc_bytes = apply_bytes(c)
    flush = torch.empty(FLUSH_BYTES // 4, dtype=torch.float32, device=step.X.device)
    vel = lambda: c.velocity(step.u, mass="lumped", out=step.us)
    frc = lambda: c.force(step.f_s, step.ff)
    out = dict(velocity_bytes=vel_bytes, force_bytes=frc_bytes, reps=reps,
               protocol="cold: 1 GiB written between repetitions, 3 warm-ups, median of 20; "
                        "warm: back to back, median of 20")
    for key, run, name, nbytes in (("velocity", vel, "spmv_B", vel_bytes),
                                   ("force", frc, "spmv_Bt", frc_bytes)):
        for _ in range(warm):
            run()
        cold = []
        for _ in range(reps):
            flush.fill_(1.0)
            cold.append(_one_launch_ms(run, name))
        hot = [_one_launch_ms(run, name) for _ in range(reps)]
        cms, hms = float(np.median(cold)), float(np.median(hot))
        out[f"{key}_ms"] = cms
        out[f"{key}_GBs"] = nbytes / cms / 1e6
        out[f"{key}_warm_ms"] = hms
        out[f"{key}_warm_GBs"] = nbytes / hms / 1e6
    del flush
    return out


def copy_ceiling(dev, reps=20):
    """Device-copy bandwidth (read + write bytes over time) of a 1 GiB copy,
    median of `reps`: the practical ceiling for streaming kernels."""
    import torch
    n = FLUSH_BYTES // 4
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    ms = float(np.median(ts))
    del a, b
    return dict(bytes=2 * FLUSH_BYTES, ms=ms, GBs=2 * FLUSH_BYTES / ms / 1e6,
                frac_of_peak=2 * FLUSH_BYTES / ms / 1e6 / HBM_PEAK_GBS)


def assembly_rate(step, n_tet, reps=10):
    """Reassembly alone (B, B^T, masses for the current positions): median
    ms over `reps` calls, HIP events around each."""
    import torch
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        step.c.reassemble(step.X)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    ms = float(np.median(ts))
    return dict(ms=ms, tets_per_s=n_tet / (ms * 1e-3), reps=reps)


def gpu_sample(step, W, seed=77, n_rows=48):
    """GPU values at sampled vertices (rows of B^d, the lumped velocity) and
    sampled fluid nodes (the force), for the error against the oracle."""
    import torch
    c = step.c
    rng = np.random.default_rng(seed)
    verts = np.sort(rng.choice(W.X.shape[0], n_rows, replace=False))
    us = c.velocity(step.u, mass="lumped").cpu().numpy().astype(np.float64)
    ff = [torch.zeros_like(u) for u in step.u]
    c.force(step.f_s, ff, alpha=1.0)
    out = dict(verts=verts, rows=[], us=us[:, verts], cols=[], ff=[])
    for d in range(3):
        rp, col, val = c.export_csr(d)
        import scipy.sparse as sp
        G = sp.csr_matrix((val, col, rp), shape=(W.X.shape[0], c.n_fluid[d]))[verts]
        cols = np.unique(G.indices)
        pick = np.sort(rng.choice(cols, min(24, cols.size), replace=False))
        out["rows"].append(G)
        out["cols"].append(pick)
        out["ff"].append(ff[d].cpu().numpy().astype(np.float64).ravel()[pick])
    return out


def fsi_rate(step, iters=6):
    """One Picard time step (Section 3) through fsi_step with stub solvers
    (a spring solid, a fluid whose velocity follows the force): ms of a step
    with 1 and with `iters` iterations; their difference per extra iteration
    is the cost of one Picard iteration (Steps 1-6 without real solvers)."""
    import torch
    c = step.c
    n = c.n_vert
    u0 = torch.zeros((3, n), dtype=c.dtype, device=step.X.device)
    vf = [u.clone() for u in step.u]

    def solid(u_hat, f):
        torch.mul(u_hat, -10.0, out=f)

    def fluid(ft, v):
        for d in range(3):
            v[d].add_(ft[d], alpha=1e-3)

    def run(k):
        c.fsi_step(step.X, u0, vf, solid, fluid, dt=1e-3, alpha=1.0, eps_abs=0.0, eps_rel=0.0,
                   max_iter=k, mass=step.mass, raise_not_converged=False)

    out = {}
    for k in (1, iters):
        run(k)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        run(k)
        e1.record()
        torch.cuda.synchronize()
        out[k] = e0.elapsed_time(e1)
    return dict(step_ms_1_iteration=out[1], step_ms=out[iters], iterations=iters,
                ms_per_picard_iteration=(out[iters] - out[1]) / (iters - 1),
                mass=step.mass, note="stub solvers; T assembled once per step at X_ref + u_hat0")


def cpu_baseline(W, dev, tets_per_body, samples):
    """The oracle leg (the only part of this script that runs the oracle).

    * value: the FP64 oracle on a bounded sample, the first `tets_per_body`
      tets of each body (a sub-mesh on the same grid), one full step, with
      the host's threads (OMP_NUM_THREADS for its C part).
    * the oracle's assembly alone at 1 thread and at the host's threads on
      the first 1000 tets of each body;
    * error_vs_oracle: the GPU's sampled full-size rows of B^d, lumped
      velocities there and forces at sampled fluid nodes (`samples`, per
      precision) against the oracle, which integrates only the tets that
      touch them."""
    import torch
    import oracle
    import scipy.sparse as sp
    import workloads as wl
    oracle.build(force=False)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))

    def sub_mesh(per_body):
        sel = []
        for b in range(len(W.bodies)):
            t0, t1 = int(W.body_tet_offsets[b]), int(W.body_tet_offsets[b + 1])
            sel.append(np.arange(t0, min(t1, t0 + per_body)))
        T = W.tets[np.concatenate(sel)]
        used, inv = np.unique(T, return_inverse=True)
        return W.X[used], inv.reshape(T.shape).astype(np.int32), used

    k, phi = wl.fourier_modes(W.n_modes, W.kmax, 2000 + W.cfg)
    u = []
    for d in range(3):
        xs, ys, zs = oracle.lattice(W.faces, d)
        u.append(wl.fourier_field(k[d], phi[d], xs, ys, zs, device=dev).cpu().numpy())
    X, T, used = sub_mesh(tets_per_body)
    f_s = W.f_s()[:, used]
    u_t = W.u_target()[:, used]
    t0 = time.perf_counter()
    cpl = oracle.assemble(W.faces, X, T)
    us = oracle.transfer_velocity(cpl, u, "consistent")
    oracle.transfer_force(cpl, f_s, 1.0)
    oracle.velocity_vjp(cpl, u, us - u_t, "consistent")
    oracle.force_vjp(cpl, f_s, [a.ravel() for a in u], 1.0)
    dt = time.perf_counter() - t0
    out = dict(value=T.shape[0] / dt, unit="solid tets/s", cores=cores, kind="oracle",
               sample=f"first {tets_per_body} tets of each of the {len(W.bodies)} bodies "
                      f"({T.shape[0]} tets, {X.shape[0]} vertices) on the full grid; one full "
                      f"step (assembly, consistent velocity by sparse LU, force, both adjoints) "
                      f"in {dt:.1f}s")
    # assembly alone at 1 thread and at `cores` threads
    Xa, Ta, _ = sub_mesh(1000)
    asm = {}
    for nth in (1, cores):
        t0 = time.perf_counter()
        oracle.assemble(W.faces, Xa, Ta, nthreads=nth)
        asm[nth] = Ta.shape[0] / (time.perf_counter() - t0)
    out["assembly_only"] = dict(unit="solid tets/s", sample=f"first 1000 tets of each body "
                                f"({Ta.shape[0]} tets)", threads_1=asm[1], **{f"threads_{cores}": asm[cores]})
    # error of the GPU's full-size results against the oracle, sampled
    errs = {prec: sampled_errors(W, u, smp, prec) for prec, smp in (samples or {}).items()}
    out["error_vs_oracle"] = errs
    return out


def sampled_errors(W, u, smp, prec):
    """Relative Frobenius errors of a GPU sample (gpu_sample) against the
    oracle, which integrates only the tets that touch the sampled rows and
    fluid nodes (oracle use: the measurement legs only)."""
    import oracle
    import scipy.sparse as sp
    bounds = oracle.tet_bounds(W.X, W.tets)
    verts = smp["verts"]
    star = oracle.vertex_star(W.tets, verts)
    R = oracle.assemble(W.faces, W.X, W.tets, subset=star)
    m = oracle.lumped_mass(W.X, W.tets[star], n_vert=W.X.shape[0])
    f_full = W.f_s()
    e = dict(rows=0.0, velocity=0.0, force=0.0)
    for d in range(3):
        Rs = R.B[d][verts]
        G = smp["rows"][d]
        e["rows"] = max(e["rows"], float(sp.linalg.norm(G - Rs) / sp.linalg.norm(Rs)))
        want = (Rs @ u[d].ravel()) / m[verts]
        e["velocity"] = max(e["velocity"], float(np.linalg.norm(smp["us"][d] - want) /
                                                 np.linalg.norm(want)))
        pick = smp["cols"][d]
        nx, ny, _ = oracle.lattice_shape(W.faces, d)
        sub = np.unique(np.concatenate([
            oracle.tets_touching_node(W.faces, W.X, W.tets, d,
                                      (j % nx, (j // nx) % ny, j // (nx * ny)), bounds)
            for j in pick]))
        Rc = oracle.assemble(W.faces, W.X, W.tets, subset=sub).B[d].tocsc()[:, pick]
        wantf = Rc.T @ f_full[d]
        e["force"] = max(e["force"], float(np.linalg.norm(smp["ff"][d] - wantf) /
                                           np.linalg.norm(wantf)))
    e["tolerance"] = 1e-12 if prec == "fp64" else 1e-5
    e["sample"] = (f"{len(verts)} seeded vertices (rows of B^d, lumped velocity), 24 fluid "
                   f"nodes per component (force); relative Frobenius, max over components")
    return e


def backward_ms(step, reps=5):
    """The velocity adjoint with the shape derivative (consistent mass): median
    ms of `reps` calls after one warm-up, HIP events around each."""
    import torch
    c = step.c
    c.velocity(step.u, mass="consistent", rtol=1e-10, maxit=500, out=step.us)
    g_us = step.us - step.u_t

    def run():
        c.velocity_vjp(g_us, u_f=step.u, u_s=step.us, mass="consistent", g_uf=step.g_uf,
                       g_X=step.g_X, rtol=1e-10, maxit=500)
    run()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        run()
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def per_config(dev, with_cpu):
    """Every workload (1..5) at its full size: reassembly rate and the apply
    rates (cold protocol) in both precisions, the error against the oracle
    (whole B and transfers for the two small workloads, sampled rows and
    nodes otherwise), the velocity adjoint with and without stored matrices
    for the differentiable and time-series workloads, and the oracle's own
    assembly rate at 1 thread and at the host's threads."""
    import torch
    import oracle
    import scipy.sparse as sp
    if with_cpu:
        oracle.build(force=False)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    rows = []
    for cfg in (1, 2, 3, 4, 5):
        W, X, T, u64, f_s, u_t = make_inputs(cfg, dev)
        n_tet = int(W.tets.shape[0])
        u_np = [u.cpu().numpy() for u in u64]
        R = None
        if with_cpu and n_tet <= 60000:
            R = oracle.assemble(W.faces, W.X, W.tets)
        row = dict(config=cfg, workload=W.name, n_tet=n_tet, n_vert=int(W.X.shape[0]),
                   grid_cells=list(W.n_cells))
        for prec in ("fp64", "fp32"):
            st = Step(W, X, T, u64, f_s, u_t, prec)
            asm = assembly_rate(st, n_tet, reps=5)
            rates = apply_rates(st)
            r = dict(assembly_ms=asm["ms"], assembly_tets_per_s=asm["tets_per_s"],
                     velocity_per_s=1e3 / rates["velocity_ms"], velocity_GBs=rates["velocity_GBs"],
                     velocity_frac=rates["velocity_GBs"] / HBM_PEAK_GBS,
                     force_per_s=1e3 / rates["force_ms"], force_GBs=rates["force_GBs"],
                     force_frac=rates["force_GBs"] / HBM_PEAK_GBS,
                     device_bytes=st.c.info()["device_bytes"])
            if with_cpu and R is not None:
                e = dict(B=0.0)
                for d in range(3):
                    rp, col, val = st.c.export_csr(d)
                    G = sp.csr_matrix((val, col, rp), shape=R.B[d].shape)
                    e["B"] = max(e["B"], float(sp.linalg.norm(G - R.B[d]) / sp.linalg.norm(R.B[d])))
                us = st.c.velocity(st.u, mass="lumped").cpu().numpy().astype(np.float64)
                want = oracle.transfer_velocity(R, u_np, "lumped")
                e["velocity"] = float(np.linalg.norm(us - want) / np.linalg.norm(want))
                ff = [torch.zeros_like(u) for u in st.u]
                st.c.force(st.f_s, ff, alpha=1.0)
                wantf = oracle.transfer_force(R, W.f_s(), 1.0)
                e["force"] = max(float(np.linalg.norm(ff[d].cpu().numpy().ravel() - wantf[d]) /
                                       np.linalg.norm(wantf[d])) for d in range(3))
                e["sample"] = "whole B^d, lumped velocity and force; relative Frobenius"
                r["error_vs_oracle"] = e
            elif with_cpu:
                r["error_vs_oracle"] = sampled_errors(W, u_np, gpu_sample(st, W), prec)
            if cfg in (3, 4):
                r["backward_stored_ms"] = backward_ms(st)
            del st
            if cfg in (3, 4):
                smf = Step(W, X, T, u64, f_s, u_t, prec, store_B=False)
                r["backward_recompute_ms"] = backward_ms(smf)
                r["recompute_device_bytes"] = smf.c.info()["device_bytes"]
                del smf
            row[prec] = r
            log(f"[bench] config {cfg} {prec}: assembly {asm['ms']:.3f} ms, velocity "
                f"{rates['velocity_GBs']:.0f} GB/s, force {rates['force_GBs']:.0f} GB/s")
        if with_cpu:
            n1 = min(n_tet, 2000)
            nn = min(n_tet, 40000)
            asm_cpu = {}
            for nth, n in ((1, n1), (cores, nn)):
                t0 = time.perf_counter()
                oracle.assemble(W.faces, W.X, W.tets[:n], nthreads=nth)
                asm_cpu[nth] = n / (time.perf_counter() - t0)
            row["oracle_assembly"] = dict(unit="solid tets/s", threads_1=asm_cpu[1],
                                          **{f"threads_{cores}": asm_cpu[cores]},
                                          sample=f"first {n1} tets (1 thread), first {nn} tets "
                                                 f"({cores} threads)", cores=cores)
        rows.append(row)
    return rows


def roofline(name, prof, info, precision):
    """Roofline object of kernel `name` over one profiled step: its
    algorithmic work in one assembly over the summed device time of its
    launches in that assembly (HIP events on the library's stream; the clip
    runs as one launch per (pair chunk, cut class), the integration as one
    per chunk).  The clip is priced at FLOPS_PER_PLANE_CUT FP64 flops per
    plane cut (midpoint as `frac`, the range beside it); the builder's own
    operation count (CLIP_FLOPS) is reported beside that."""
    launches, total_ms = prof
    ms = total_ms
    out = dict(kernel=name + " (all launches of one assembly)", bound="unknown", achieved=None,
               peak=None, unit=None, frac=None, traffic=None, launch_ms=ms,
               timed_launches=launches)
    if name == "clip":
        lo, mid, hi = (f * info["plane_cuts"] for f in FLOPS_PER_PLANE_CUT)
        achieved = mid / (ms * 1e-3) / 1e12
        own = (CLIP_FLOPS["dist"] * info["dist_evals"] + CLIP_FLOPS["cut"] * info["cut_points"] +
               CLIP_FLOPS["subtet"] * info["subtets"] + CLIP_FLOPS["pair"] * info["pairs"])
        traffic = None
        if (precision == "fp32" and CLIP_TRAFFIC["bytes_mixed"] is not None and
                CLIP_TRAFFIC["sources_sha256"] == sources_sha256(CLIP_SOURCES)):
            traffic = CLIP_TRAFFIC["bytes_mixed"]
        out.update(bound="alu", achieved=achieved, peak=FP64_VEC_PEAK_TFLOPS, unit="TFLOP/s",
                   frac=achieved / FP64_VEC_PEAK_TFLOPS, traffic=traffic,
                   precision="fp64 (clipping is double)",
                   plane_cuts=info["plane_cuts"], flops_per_plane_cut=FLOPS_PER_PLANE_CUT[1],
                   algorithmic_flops_per_launch=mid,
                   frac_range=[lo / (ms * 1e-3) / 1e12 / FP64_VEC_PEAK_TFLOPS,
                               hi / (ms * 1e-3) / 1e12 / FP64_VEC_PEAK_TFLOPS],
                   own_count=dict(flops=own, frac=own / (ms * 1e-3) / 1e12 / FP64_VEC_PEAK_TFLOPS,
                                  dist_evals=info["dist_evals"], cut_points=info["cut_points"],
                                  subtets=info["subtets"], pairs=info["pairs"]))
    elif name == "integrate":
        flops = info["subtets"] * POINTS_PER_SUBTET * MOM_FLOPS_PER_POINT
        peak = FP32_VEC_PEAK_TFLOPS if precision == "fp32" else FP64_VEC_PEAK_TFLOPS
        achieved = flops / (ms * 1e-3) / 1e12
        out.update(bound="alu", achieved=achieved, peak=peak, unit="TFLOP/s", frac=achieved / peak,
                   algorithmic_flops_per_launch=flops)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", type=int, default=5, help=argparse.SUPPRESS)
    ap.add_argument("--skip-fp64", action="store_true", help="do not time the FP64 step")
    ap.add_argument("--skip-cpu", action="store_true", help="do not time the oracle")
    ap.add_argument("--cpu-tets-per-body", type=int, default=8000)
    ap.add_argument("--profile-run", action="store_true",
                    help="one mixed-precision step and the applies only (for rocprofv3)")
    ap.add_argument("--planar-only", action="store_true",
                    help="only the planar leg (prints its JSON object; for rocprofv3)")
    ap.add_argument("--unstructured-only", action="store_true",
                    help="only the unstructured-background leg (prints its JSON object)")
    ap.add_argument("--clip-only", action="store_true",
                    help="only the mixed-precision assembly and one reassembly (counter runs)")
    ap.add_argument("--per-config", action="store_true",
                    help="every workload at full size (rates, errors, adjoints; JSON list)")
    ap.add_argument("--copy-gib", type=float, default=0.0,
                    help="only run a plain device copy of this many GiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the transfer is built and timed on a single MI355X; "
              "multi-GPU sharding is a design note only (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    if args.copy_gib > 0:
        n = int(args.copy_gib * (1 << 30) / 8)
        a = torch.ones(n, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n, "launches": 3}))
        return
    from paper_1810_13046_amd import load_library
    load_library()
    if args.planar_only:
        print(json.dumps(planar_leg(dev, args.steps, args.warmup, False)))
        return
    if args.per_config:
        print(json.dumps(per_config(dev, not args.skip_cpu)))
        return
    if args.unstructured_only:
        print(json.dumps(unstructured_leg(dev, args.steps, args.warmup, False)))
        return
    if args.profile_run:
        args.skip_fp64 = True
        args.skip_cpu = True

    W, X, T, u64, f_s, u_t = make_inputs(args.workload, dev)
    n_tet = W.tets.shape[0]
    if args.clip_only:
        from paper_1810_13046_amd import Coupling
        c = Coupling(W.faces, X, T, precision="fp32", consistent=True)
        c.reassemble(X)
        torch.cuda.synchronize()
        print(json.dumps({"assemblies": c.info()["assemblies"], "pairs": c.info()["pairs"]}))
        return

    log("[bench] mixed-precision step: build")
    mixed = Step(W, X, T, u64, f_s, u_t, "fp32")
    log("[bench] mixed-precision step: timing")
    ms_mixed, wall_mixed = time_steps(mixed, args.steps, args.warmup)
    prof_mixed = kernel_profile(mixed)
    rates_mixed = apply_rates(mixed)
    info = mixed.c.info()
    log(f"[bench] mixed {ms_mixed:.2f} ms/step; kernels {json.dumps(prof_mixed)}")
    asm_mixed = assembly_rate(mixed, n_tet, reps=3 if args.profile_run else 10)
    log(f"[bench] mixed assembly alone {asm_mixed['ms']:.2f} ms")
    copy = copy_ceiling(dev)
    log(f"[bench] device copy {copy['GBs']:.0f} GB/s")
    samples = {}
    if not args.skip_cpu:
        samples["fp32"] = gpu_sample(mixed, W)
    fsi = None
    if not args.profile_run:
        log("[bench] Picard coupling step (mixed)")
        fsi = fsi_rate(mixed)
        log(f"[bench] fsi {fsi['ms_per_picard_iteration']:.2f} ms per Picard iteration")

    # what the coupling holds once the assembly's scratch is released
    mixed.c.release_scratch()
    import torch
    torch.cuda.synchronize()
    bytes_released = mixed.c.info()["device_bytes"]
    fp64 = None
    if not args.skip_fp64:
        del mixed.c
        mixed_keep = mixed
        log("[bench] fp64 step: build")
        s64 = Step(W, X, T, u64, f_s, u_t, "fp64")
        log("[bench] fp64 step: timing")
        ms64, wall64 = time_steps(s64, args.steps, args.warmup)
        prof64 = kernel_profile(s64)
        rates64 = apply_rates(s64)
        asm64 = assembly_rate(s64, n_tet)
        fp64 = dict(ms_per_step=ms64, value=n_tet / (ms64 * 1e-3), kernels_ms=prof64,
                    applies=rates64, assembly_only=asm64,
                    device_bytes=s64.c.info()["device_bytes"])
        if not args.skip_cpu:
            samples["fp64"] = gpu_sample(s64, W)
        log(f"[bench] fp64 {ms64:.2f} ms/step")
        del s64
        del mixed_keep
    # device memory of the mixed-precision coupling without the moment store
    bytes_no_store = None
    if not args.profile_run:
        import torch
        from paper_1810_13046_amd import Coupling
        cns = Coupling(W.faces, X, T, precision="fp32", consistent=True, store_pieces=False)
        torch.cuda.synchronize()
        bytes_no_store = cns.info()["device_bytes"]
        cns.free()

    dual = None
    if not args.profile_run:
        log("[bench] dual-basis step (mixed): build")
        sd = Step(W, X, T, u64, f_s, u_t, "fp32", dual=True)
        ms_d, _ = time_steps(sd, args.steps, args.warmup)
        dual = dict(ms_per_step=ms_d, value=n_tet / (ms_d * 1e-3),
                    note="dual multipliers (S = lumped mass): reassembly, velocity, force, "
                         "both adjoints; no mass solve")
        log(f"[bench] dual {ms_d:.2f} ms/step")
        del sd

    matrix_free = None
    if not args.profile_run:
        log("[bench] step without stored matrices (mixed): build")
        smf = Step(W, X, T, u64, f_s, u_t, "fp32", store_B=False)
        ms_mf, _ = time_steps(smf, max(1, min(args.steps, 3)), 1)
        matrix_free = dict(ms_per_step=ms_mf, value=n_tet / (ms_mf * 1e-3),
                           device_bytes=smf.c.info()["device_bytes"],
                           note="IBVT_NO_STORE_B: no B, B^T or per-pair data held; the "
                                "consistent velocity, the force and both adjoints clip and "
                                "integrate every piece again")
        log(f"[bench] without stored matrices {ms_mf:.2f} ms/step")
        del smf

    # dominant kernel of the mixed step and its roofline
    per_kernel = {k: v[1] for k, v in prof_mixed.items()}
    dom = max(per_kernel, key=per_kernel.get)
    roof = roofline(dom, prof_mixed[dom], info, "fp32")
    apply_traffic = None
    if (APPLY_TRAFFIC["velocity_bytes"] is not None and
            APPLY_TRAFFIC["sources_sha256"] == sources_sha256(APPLY_SOURCES)):
        apply_traffic = APPLY_TRAFFIC["velocity_bytes"]
    roof_apply = dict(kernel="spmv_B (lumped velocity apply, cold cache)", bound="hbm",
                      achieved=rates_mixed["velocity_GBs"], peak=HBM_PEAK_GBS, unit="GB/s",
                      frac=rates_mixed["velocity_GBs"] / HBM_PEAK_GBS, traffic=apply_traffic,
                      launch_ms=rates_mixed["velocity_ms"],
                      algorithmic_bytes_per_launch=rates_mixed["velocity_bytes"],
                      frac_of_copy_ceiling=rates_mixed["velocity_GBs"] / copy["GBs"],
                      force_GBs=rates_mixed["force_GBs"],
                      force_frac=rates_mixed["force_GBs"] / HBM_PEAK_GBS)

    planar = None
    if not args.profile_run:
        planar = planar_leg(dev, max(args.steps, 10), args.warmup, not args.skip_cpu)
    unstructured = None
    if not args.profile_run:
        unstructured = unstructured_leg(dev, args.steps, args.warmup, not args.skip_cpu)

    cpu = None
    if not args.skip_cpu:
        log("[bench] cpu baseline (oracle)")
        cpu = cpu_baseline(W, dev, args.cpu_tets_per_body, samples)
        log(f"[bench] cpu baseline {cpu['value']:.1f} tets/s")

    out = {
        "metric": "B assembly (solid tets/s) + transfer applies/s, HBM % of peak; mixed vs FP64",
        "value": n_tet / (ms_mixed * 1e-3),
        "unit": "solid tets/s (full step: assembly + consistent velocity + force + both adjoints)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_mixed,
        "wall_ms_per_step": wall_mixed,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 quadrature/applies, f64 clipping and mass-solve residual",
        "data": "synthetic (seeded meshes and Fourier velocity fields)",
        "config": {
            "workload": W.name, "n_tet": int(n_tet), "n_vert": int(W.X.shape[0]),
            "grid_cells": list(W.n_cells), "y_stretch_ratio": 4.0, "bodies": len(W.bodies),
            "mass": "consistent", "solve_rtol": 1e-10, "parallelism": "single GPU",
        },
        "assembly": {"pairs": info["pairs"], "pieces": info["pieces"], "subtets": info["subtets"],
                     "plane_cuts": info["plane_cuts"], "dist_evals": info["dist_evals"],
                     "cut_points": info["cut_points"],
                     "nnz": info["nnz"], "touched": info["touched"],
                     "device_bytes": info["device_bytes"],
                     "device_bytes_after_release_scratch": bytes_released,
                     "device_bytes_no_piece_store": bytes_no_store},
        "assembly_only": {**asm_mixed, "unit": "solid tets/s (reassembly: B, B^T, masses)"},
        "copy_ceiling": copy,
        "error_vs_oracle": cpu["error_vs_oracle"] if cpu else None,
        "kernels_ms": {k: v[1] for k, v in prof_mixed.items()},
        "kernels_ms_note": "per stage, HIP events on the stream each stage runs on; the "
                           "12- and 16-slot clip classes run on a second stream inside 'clip', "
                           "and 'pair_order_beside_integrate' (the next chunk's order) beside "
                           "'integrate', so the stages overlap and their sum exceeds the step",
        "kernel_launches": {k: v[0] for k, v in prof_mixed.items()},
        "applies": {
            "velocity_per_s": 1e3 / rates_mixed["velocity_ms"],
            "force_per_s": 1e3 / rates_mixed["force_ms"],
            **rates_mixed,
        },
        "fp64": fp64,
        "speedup_mixed_vs_fp64": (fp64["ms_per_step"] / ms_mixed) if fp64 else None,
        "dual_basis": dual,
        "without_stored_matrices": matrix_free,
        "fsi_picard": fsi,
        "planar": planar,
        "unstructured": unstructured,
        "roofline": roof,
        "roofline_apply": roof_apply,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
