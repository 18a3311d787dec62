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
# flops per quadrature point of the 35 piece moments: point 6, powers 9,
# partial products 14, 35 multiply-adds 70; 11 points (degree 4) per
# sub-tetrahedron
MOM_FLOPS_PER_POINT = 99
POINTS_PER_SUBTET = 11

# HBM traffic of the clip step (both slot-class launches of one assembly) on
# the three-body workload, from rocprofv3 FETCH_SIZE and WRITE_SIZE counter
# passes, scaled by the copy-kernel calibration (FETCH x 2, WRITE x 1): the
# summary and its commands are in profiles/.  Reported only while the clip
# sources are the ones the counters were taken on.
CLIP_TRAFFIC = dict(sources_sha256="cabeb8d4ad35f8fbf2f6a963582c61d6b5051132c9182e61302edb9beedced2b",
                    bytes_mixed=35621912352)
CLIP_SOURCES = ["paper_1810_13046_amd/csrc/assemble.hip", "paper_1810_13046_amd/csrc/geometry.hpp",
                "paper_1810_13046_amd/csrc/common.hpp"]


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

    def __init__(self, W, X, T, u64, f_s, u_t, precision, dual=False):
        import torch
        from paper_1810_13046_amd import Coupling
        self.dual = dual
        self.mass = "lumped" if dual else "consistent"
        self.c = Coupling(W.faces, X, T, precision=precision, consistent=not dual, dual=dual)
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


def apply_rates(step, reps=20):
    """Lumped velocity apply and force apply: ms per launch (HIP events on
    the library's stream) and algorithmic bytes per apply."""
    import torch
    from paper_1810_13046_amd import profile_enable, profile_read
    c = step.c
    info = c.info()
    s = 8 if c.precision == "fp64" else 4
    n = info["n_vert"]
    nnz, t = info["nnz"], info["touched"]
    vel_bytes = sum(nnz[d] * (s + 4) + 4 * (n + 1) + s * t[d] + s * n for d in range(3)) + s * n
    frc_bytes = sum(nnz[d] * (s + 4) + 4 * (t[d] + 1) + 4 * t[d] + 2 * s * t[d] + s * n
                    for d in range(3))
    for _ in range(3):
        c.velocity(step.u, mass="lumped", out=step.us)
        c.force(step.f_s, step.ff)
    torch.cuda.synchronize()
    profile_read()
    profile_enable(True)
    for _ in range(reps):
        c.velocity(step.u, mass="lumped", out=step.us)
        c.force(step.f_s, step.ff)
    torch.cuda.synchronize()
    prof = profile_read()
    profile_enable(False)
    vel_ms = prof["spmv_B"][1] / prof["spmv_B"][0]
    frc_ms = prof["spmv_Bt"][1] / prof["spmv_Bt"][0]
    return dict(velocity_ms=vel_ms, force_ms=frc_ms, velocity_bytes=vel_bytes, force_bytes=frc_bytes,
                velocity_GBs=vel_bytes / vel_ms / 1e6, force_GBs=frc_bytes / frc_ms / 1e6)


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


def cpu_baseline(W, dev, tets_per_body):
    """The FP64 oracle on a bounded sample: the first `tets_per_body` tets of
    each body (a sub-mesh on the same grid), one full step."""
    import torch
    import oracle
    import workloads as wl
    oracle.build(force=False)
    sel = []
    for b in range(len(W.bodies)):
        t0, t1 = int(W.body_tet_offsets[b]), int(W.body_tet_offsets[b + 1])
        sel.append(np.arange(t0, min(t1, t0 + tets_per_body)))
    sel = np.concatenate(sel)
    T = W.tets[sel]
    used, inv = np.unique(T, return_inverse=True)
    T = inv.reshape(T.shape).astype(np.int32)
    X = W.X[used]
    k, phi = wl.fourier_modes(W.n_modes, W.kmax, 2000 + W.cfg)
    u = []
    for d in range(3):
        xs, ys, zs = oracle.lattice(W.faces, d)
        u.append(wl.fourier_field(k[d], phi[d], xs, ys, zs, device=dev).cpu().numpy())
    f_s = W.f_s()[:, used]
    u_t = W.u_target()[:, used]
    t0 = time.perf_counter()
    cpl = oracle.assemble(W.faces, X, T)
    us = oracle.transfer_velocity(cpl, u, "consistent")
    oracle.transfer_force(cpl, f_s, 1.0)
    oracle.velocity_vjp(cpl, u, us - u_t, "consistent")
    oracle.force_vjp(cpl, f_s, [a.ravel() for a in u], 1.0)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return dict(value=T.shape[0] / dt, unit="solid tets/s", cores=cores, kind="oracle",
                sample=f"first {tets_per_body} tets of each of the {len(W.bodies)} bodies "
                       f"({T.shape[0]} tets, {X.shape[0]} vertices) on the full grid; one full "
                       f"step (assembly, consistent velocity by sparse LU, force, both adjoints) "
                       f"in {dt:.1f}s")


def roofline(name, prof, info, precision):
    """Roofline object of one profiled step of kernel `name`: algorithmic
    work per launch (see the constants above) over its average launch time
    (HIP events on the library's stream)."""
    launches, total_ms = prof
    ms = total_ms / launches
    out = dict(kernel=name, bound="unknown", achieved=None, peak=None, unit=None, frac=None,
               traffic=None, launch_ms=ms)
    if name == "clip":
        flops = (CLIP_FLOPS["dist"] * info["dist_evals"] + CLIP_FLOPS["cut"] * info["cut_points"] +
                 CLIP_FLOPS["subtet"] * info["subtets"] + CLIP_FLOPS["pair"] * info["pairs"])
        achieved = flops / (ms * 1e-3) / 1e12
        traffic = None
        if (precision == "fp32" and CLIP_TRAFFIC["bytes_mixed"] is not None and
                CLIP_TRAFFIC["sources_sha256"] == sources_sha256(CLIP_SOURCES)):
            traffic = CLIP_TRAFFIC["bytes_mixed"]
        out.update(bound="alu", achieved=achieved, peak=FP64_VEC_PEAK_TFLOPS, unit="TFLOP/s",
                   frac=achieved / FP64_VEC_PEAK_TFLOPS, traffic=traffic,
                   algorithmic_flops_per_launch=flops, precision="fp64 (clipping is double)")
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
    if args.unstructured_only:
        print(json.dumps(unstructured_leg(dev, args.steps, args.warmup, False)))
        return
    if args.profile_run:
        args.skip_fp64 = True
        args.skip_cpu = True

    W, X, T, u64, f_s, u_t = make_inputs(args.workload, dev)
    n_tet = W.tets.shape[0]

    log("[bench] mixed-precision step: build")
    mixed = Step(W, X, T, u64, f_s, u_t, "fp32")
    log("[bench] mixed-precision step: timing")
    ms_mixed, wall_mixed = time_steps(mixed, args.steps, args.warmup)
    prof_mixed = kernel_profile(mixed)
    rates_mixed = apply_rates(mixed)
    info = mixed.c.info()
    log(f"[bench] mixed {ms_mixed:.2f} ms/step; kernels {json.dumps(prof_mixed)}")
    fsi = None
    if not args.profile_run:
        log("[bench] Picard coupling step (mixed)")
        fsi = fsi_rate(mixed)
        log(f"[bench] fsi {fsi['ms_per_picard_iteration']:.2f} ms per Picard iteration")

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
        fp64 = dict(ms_per_step=ms64, value=n_tet / (ms64 * 1e-3), kernels_ms=prof64,
                    applies=rates64)
        log(f"[bench] fp64 {ms64:.2f} ms/step")
        del s64
        del mixed_keep

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

    # dominant kernel of the mixed step and its roofline
    per_kernel = {k: v[1] for k, v in prof_mixed.items()}
    dom = max(per_kernel, key=per_kernel.get)
    roof = roofline(dom, prof_mixed[dom], info, "fp32")
    roof_apply = dict(kernel="spmv_B (lumped velocity apply)", bound="hbm",
                      achieved=rates_mixed["velocity_GBs"], peak=HBM_PEAK_GBS, unit="GB/s",
                      frac=rates_mixed["velocity_GBs"] / HBM_PEAK_GBS, traffic=None,
                      launch_ms=rates_mixed["velocity_ms"],
                      algorithmic_bytes_per_launch=rates_mixed["velocity_bytes"])

    planar = None
    if not args.profile_run:
        planar = planar_leg(dev, max(args.steps, 10), args.warmup, not args.skip_cpu)
    unstructured = None
    if not args.profile_run:
        unstructured = unstructured_leg(dev, args.steps, args.warmup, not args.skip_cpu)

    cpu = None
    if not args.skip_cpu:
        log("[bench] cpu baseline (oracle)")
        cpu = cpu_baseline(W, dev, args.cpu_tets_per_body)
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
                     "nnz": info["nnz"], "touched": info["touched"],
                     "device_bytes": info["device_bytes"]},
        "kernels_ms": {k: v[1] for k, v in prof_mixed.items()},
        "kernel_launches": {k: v[0] for k, v in prof_mixed.items()},
        "applies": {
            "velocity_per_s": 1e3 / rates_mixed["velocity_ms"],
            "force_per_s": 1e3 / rates_mixed["force_ms"],
            **rates_mixed,
        },
        "fp64": fp64,
        "speedup_mixed_vs_fp64": (fp64["ms_per_step"] / ms_mixed) if fp64 else None,
        "dual_basis": dual,
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
