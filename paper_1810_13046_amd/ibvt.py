"""Python binding of libibvt (argument marshalling only).

Every numerical step runs in the HIP library; this module only checks
shapes and dtypes of torch tensors and passes device pointers and the
current HIP stream through the C ABI declared in include/ibvt.h.  There is
no CPU fallback: if the library is missing or no GPU is present, calls
raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libibvt.so")

IBVT_OK = 0
INVALID = 1
NOT_CONVERGED = 5
STATUS_NAMES = {
    0: "IBVT_OK", 1: "IBVT_E_INVALID", 2: "IBVT_E_OUT_OF_GRID", 3: "IBVT_E_HIP",
    4: "IBVT_E_NOMEM", 5: "IBVT_E_NOT_CONVERGED", 6: "IBVT_E_CAPACITY", 7: "IBVT_E_UNSUPPORTED",
}
FP64, FP32_MIXED = 0, 1
LUMPED, CONSISTENT = 0, 1
BUILD_CONSISTENT_M = 1
NO_PIECE_STORE = 2
DUAL_BASIS = 4
NO_STORE_B = 8
FORCE_IS_LOAD = 1

EXPORTED = [
    "assemble_coupling", "reassemble_coupling", "transfer_velocity", "transfer_force",
    "transfer_velocity_vjp", "transfer_force_vjp", "coupling_info", "coupling_export_csr",
    "coupling_free", "ibvt_status_string", "ibvt_last_error", "ibvt_lattice_coords",
    "ibvt_profile_enable", "ibvt_profile_read", "fsi_step", "ibvt_fluid_lumped_volume",
    "assemble_coupling_2d", "ibvt_lattice_coords_2d", "assemble_coupling_unstructured",
    "transfer_vjp", "ibvt_fluid_lumped_volume_2d", "transfer_velocity_noalloc",
    "coupling_body_info", "ibvt_set_allocator", "coupling_release_scratch",
]


class IbvtError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        self.name = STATUS_NAMES.get(status, str(status))
        super().__init__(f"{where}: {self.name}: {detail}")


class _Grid(ctypes.Structure):
    _fields_ = [("n_cells", ctypes.c_int32 * 3), ("faces", ctypes.c_void_p * 3)]


class _Mesh(ctypes.Structure):
    _fields_ = [("n_vert", ctypes.c_int64), ("n_tet", ctypes.c_int64),
                ("X", ctypes.c_void_p), ("tets", ctypes.c_void_p)]


class _Grid2d(ctypes.Structure):
    _fields_ = [("n_cells", ctypes.c_int32 * 2), ("faces", ctypes.c_void_p * 2)]


class _Mesh2d(ctypes.Structure):
    _fields_ = [("n_vert", ctypes.c_int64), ("n_tri", ctypes.c_int64),
                ("X", ctypes.c_void_p), ("tris", ctypes.c_void_p)]


class _SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32 * 3), ("rel_residual", ctypes.c_double * 3)]


class _Info(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("has_consistent_mass", ctypes.c_int32),
                ("n_vert", ctypes.c_int64), ("n_tet", ctypes.c_int64),
                ("lattice", (ctypes.c_int64 * 3) * 3), ("n_fluid", ctypes.c_int64 * 3),
                ("pairs", ctypes.c_int64), ("pieces", ctypes.c_int64),
                ("dropped", ctypes.c_int64), ("zero_tets", ctypes.c_int64),
                ("nnz", ctypes.c_int64 * 3), ("touched", ctypes.c_int64 * 3),
                ("nnz_mass", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("assemblies", ctypes.c_int64), ("subtets", ctypes.c_int64),
                ("piece_store", ctypes.c_int64), ("dist_evals", ctypes.c_int64),
                ("cut_points", ctypes.c_int64), ("dual", ctypes.c_int64), ("dim", ctypes.c_int64),
                ("unstructured", ctypes.c_int64), ("plane_cuts", ctypes.c_int64),
                ("matrix_free", ctypes.c_int64)]


class _BodyInfo(ctypes.Structure):
    _fields_ = [("tets", ctypes.c_int64), ("zero_tets", ctypes.c_int64), ("pairs", ctypes.c_int64),
                ("pieces", ctypes.c_int64), ("volume", ctypes.c_double)]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class _Alloc(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("ctx", ctypes.c_void_p)]


_lib = None


class _FsiConfig(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("alpha", ctypes.c_double), ("eps_abs", ctypes.c_double),
                ("eps_rel", ctypes.c_double), ("max_iter", ctypes.c_int32), ("mass", ctypes.c_int32),
                ("force_density", ctypes.c_int32), ("cg_maxit", ctypes.c_int32),
                ("cg_rtol", ctypes.c_double)]


class _FsiBuffers(ctypes.Structure):
    _fields_ = [("X_ref", ctypes.c_void_p), ("u_hat0", ctypes.c_void_p), ("u_hat", ctypes.c_void_p),
                ("w_s", ctypes.c_void_p), ("f_fsi", ctypes.c_void_p), ("f_prev", ctypes.c_void_p),
                ("v_f", ctypes.c_void_p * 3), ("f_tilde", ctypes.c_void_p * 3)]


class _FsiReport(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("res_abs", ctypes.c_double), ("res_rel", ctypes.c_double),
                ("f1_norm", ctypes.c_double)]


_SOLID_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                             ctypes.c_void_p)
_FLUID_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                             ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p)


def load_library(path: str = LIB_PATH):
    """Load libibvt.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build it with `python -m paper_1810_13046_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, i64, u32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_double
    P = ctypes.POINTER
    lib.assemble_coupling.argtypes = [P(_Grid), P(_Mesh), ctypes.c_int, u32, vp, P(vp)]
    lib.reassemble_coupling.argtypes = [vp, vp, vp]
    lib.transfer_velocity.argtypes = [vp, P(vp), vp, ctypes.c_int, dbl, ctypes.c_int, vp, P(_SolveInfo)]
    lib.transfer_velocity_noalloc.argtypes = lib.transfer_velocity.argtypes
    lib.transfer_force.argtypes = [vp, vp, P(vp), dbl, u32, vp]
    lib.transfer_velocity_vjp.argtypes = [vp, vp, P(vp), vp, ctypes.c_int, dbl, ctypes.c_int, P(vp), vp, vp]
    lib.transfer_force_vjp.argtypes = [vp, P(vp), vp, dbl, vp, vp, vp]
    lib.coupling_info.argtypes = [vp, P(_Info)]
    lib.coupling_export_csr.argtypes = [vp, ctypes.c_int, ctypes.c_int, P(i64), P(i64), vp, vp, vp, vp]
    lib.coupling_free.argtypes = [vp]
    lib.coupling_free.restype = None
    lib.ibvt_status_string.argtypes = [ctypes.c_int]
    lib.ibvt_status_string.restype = ctypes.c_char_p
    lib.ibvt_last_error.argtypes = []
    lib.ibvt_last_error.restype = ctypes.c_char_p
    lib.ibvt_lattice_coords.argtypes = [P(_Grid), ctypes.c_int, ctypes.c_int, vp, P(i64)]
    lib.ibvt_profile_enable.argtypes = [ctypes.c_int]
    lib.ibvt_profile_enable.restype = None
    lib.ibvt_profile_read.argtypes = [P(ctypes.c_char_p), P(i64), P(dbl), ctypes.c_int]
    lib.ibvt_profile_read.restype = ctypes.c_int
    lib.fsi_step.argtypes = [vp, P(_FsiConfig), P(_FsiBuffers), _SOLID_FN, vp, _FLUID_FN, vp, vp,
                             P(_FsiReport)]
    lib.ibvt_fluid_lumped_volume.argtypes = [P(_Grid), ctypes.c_int, vp, vp]
    lib.ibvt_fluid_lumped_volume_2d.argtypes = [P(_Grid2d), ctypes.c_int, vp, vp]
    lib.assemble_coupling_2d.argtypes = [P(_Grid2d), P(_Mesh2d), ctypes.c_int, u32, vp, P(vp)]
    lib.ibvt_lattice_coords_2d.argtypes = [P(_Grid2d), ctypes.c_int, ctypes.c_int, vp, P(i64)]
    lib.assemble_coupling_unstructured.argtypes = [P(_Mesh), P(_Mesh), ctypes.c_int, u32, vp, P(vp)]
    lib.transfer_vjp.argtypes = [vp, vp, P(vp), vp, ctypes.c_int, dbl, ctypes.c_int, P(vp),
                                 P(vp), vp, dbl, vp, vp, vp]
    lib.coupling_body_info.argtypes = [vp, i32, P(i64), P(_BodyInfo), vp]
    lib.ibvt_set_allocator.argtypes = [P(_Alloc)]
    lib.coupling_release_scratch.argtypes = [vp, vp]
    for name in ("assemble_coupling", "reassemble_coupling", "transfer_velocity", "transfer_force",
                 "transfer_velocity_vjp", "transfer_force_vjp", "coupling_info",
                 "coupling_export_csr", "ibvt_lattice_coords", "fsi_step",
                 "ibvt_fluid_lumped_volume", "assemble_coupling_2d", "ibvt_lattice_coords_2d",
                 "assemble_coupling_unstructured", "transfer_vjp", "ibvt_fluid_lumped_volume_2d",
                 "transfer_velocity_noalloc", "coupling_body_info", "ibvt_set_allocator",
                 "coupling_release_scratch"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


# torch's caching allocator behind ibvt_set_allocator (the callbacks must
# outlive every coupling created while they are set)
def _torch_alloc(nbytes, stream, ctx):
    import torch
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(),
                                                  stream or 0)
    except Exception:
        return None


def _torch_free(ptr, stream, ctx):
    try:
        import torch
        torch.cuda.caching_allocator_delete(ptr)
    except Exception:
        pass


_TORCH_ALLOC = _Alloc(_ALLOC_FN(_torch_alloc), _FREE_FN(_torch_free), None)


def use_torch_allocator(enable: bool = True):
    """Couplings created after this call take their device buffers from
    torch's caching allocator (enable=True) or from hipMallocAsync
    (enable=False); each coupling frees with the allocator it was made with
    (ibvt_set_allocator)."""
    lib = load_library()
    _check(lib.ibvt_set_allocator(ctypes.byref(_TORCH_ALLOC) if enable else None),
           "ibvt_set_allocator")


def _check(st: int, where: str):
    if st != IBVT_OK:
        detail = _lib.ibvt_last_error().decode(errors="replace") if _lib else ""
        raise IbvtError(st, where, detail)


def _grid_struct(faces):
    """ibvt_grid (3 face arrays) or ibvt_grid2d (2 face arrays)."""
    faces = [np.ascontiguousarray(np.asarray(f, dtype=np.float64)) for f in faces]
    if len(faces) not in (2, 3):
        raise ValueError("faces: 3 arrays (3D grid) or 2 (planar grid)")
    g = _Grid() if len(faces) == 3 else _Grid2d()
    for e in range(len(faces)):
        g.n_cells[e] = faces[e].size - 1
        g.faces[e] = faces[e].ctypes.data
    return g, faces


def lattice_coords(faces, comp: int):
    """Node coordinates of component `comp`'s lattice along each axis (host)."""
    lib = load_library()
    g, keep = _grid_struct(faces)
    fn = lib.ibvt_lattice_coords if len(keep) == 3 else lib.ibvt_lattice_coords_2d
    out = []
    for e in range(len(keep)):
        n = ctypes.c_int64()
        _check(fn(ctypes.byref(g), comp, e, None, ctypes.byref(n)), "lattice")
        a = np.empty(n.value)
        _check(fn(ctypes.byref(g), comp, e, a.ctypes.data, ctypes.byref(n)), "lattice")
        out.append(a)
    del keep
    return out


def profile_enable(on: bool = True):
    """Record device time of the library's main kernels (HIP events)."""
    load_library().ibvt_profile_enable(1 if on else 0)


def profile_read() -> dict:
    """{kernel name: (launches, total ms)} since the last read (synchronizes)."""
    lib = load_library()
    n = 64
    names = (ctypes.c_char_p * n)()
    launches = (ctypes.c_int64 * n)()
    ms = (ctypes.c_double * n)()
    k = lib.ibvt_profile_read(names, launches, ms, n)
    if k < 0:
        raise IbvtError(-k, "profile_read", lib.ibvt_last_error().decode(errors="replace"))
    return {names[i].decode(): (int(launches[i]), float(ms[i])) for i in range(k)}


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, dtype, numel, what):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what}: expected a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{what}: expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what}: must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{what}: expected {numel} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


@dataclass
class FsiReport:
    iterations: int
    converged: bool
    res_abs: float
    res_rel: float
    f1_norm: float


def fluid_lumped_volume(faces, comp: int, device=None, stream=None):
    """Q1 lumped volume ∫ N_j of every node of component comp's lattice,
    shape (n_z, n_y, n_x) (with two face arrays the planar lumped area,
    shape (n_y, n_x)), float64 on the device."""
    import torch
    lib = load_library()
    g, keep = _grid_struct(faces)
    shape = tuple(reversed([len(a) for a in lattice_coords(faces, comp)]))
    out = torch.empty(shape, dtype=torch.float64, device=device or "cuda")
    fn = lib.ibvt_fluid_lumped_volume if len(keep) == 3 else lib.ibvt_fluid_lumped_volume_2d
    _check(fn(ctypes.byref(g), comp, ctypes.c_void_p(out.data_ptr()), _stream(stream)),
           "ibvt_fluid_lumped_volume")
    del keep
    return out


@dataclass
class SolveInfo:
    iterations: tuple
    rel_residual: tuple


class Coupling:
    """A coupling handle: B^d, B^dT, masses for one grid and mesh.

    Three face arrays, X (n_vert, 3) and tets (n_tet, 4) make a 3D coupling;
    two face arrays, X (n_vert, 2) and triangles (n_tri, 3) a planar one
    (assemble_coupling_2d), whose solid fields are (2, n_vert) and whose
    fluid fields are 2 arrays of shape (n_y, n_x).  With fluid_mesh =
    (X_f, tets_f) (device tensors, a P1 tetrahedral fluid mesh) and faces =
    None the background is unstructured (assemble_coupling_unstructured):
    the fluid fields are 3 nodal arrays of the fluid mesh's vertices.
    store_B=False (3D grids only) keeps no matrices: every transfer and
    adjoint clips and integrates the pieces again (IBVT_NO_STORE_B)."""

    def __init__(self, faces, X, tets, precision: str = "fp64", consistent: bool = True,
                 store_pieces: bool = True, dual: bool = False, stream=None, fluid_mesh=None,
                 store_B: bool = True):
        import torch
        lib = load_library()
        if precision not in ("fp64", "fp32"):
            raise ValueError("precision must be 'fp64' or 'fp32' (mixed)")
        self.precision = precision
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        self.dual = bool(dual)
        self.consistent = consistent
        if fluid_mesh is not None:
            if not store_B:
                raise ValueError("store_B=False is for grid couplings")
            self._init_unstructured(fluid_mesh, X, tets, precision, consistent, dual, stream)
            return
        self.faces = [np.ascontiguousarray(np.asarray(f, dtype=np.float64)) for f in faces]
        self.dim = len(self.faces)
        self.nc = self.dim
        k = self.dim + 1
        self.n_vert = int(X.shape[0])
        self.n_tet = int(tets.shape[0])
        if X.ndim != 2 or X.shape[1] != self.dim:
            raise ValueError(f"X must be (n_vert, {self.dim})")
        if tets.ndim != 2 or tets.shape[1] != k:
            raise ValueError(f"elements must be (n, {k})")
        g, keep = _grid_struct(self.faces)
        m = _Mesh() if self.dim == 3 else _Mesh2d()
        m.n_vert = self.n_vert
        Xp = _dev(X, torch.float64, self.dim * self.n_vert, "X")
        Tp = _dev(tets, torch.int32, k * self.n_tet, "elements") if self.n_tet else None
        if self.dim == 3:
            m.n_tet, m.X, m.tets = self.n_tet, Xp, Tp
        else:
            m.n_tri, m.X, m.tris = self.n_tet, Xp, Tp
        h = ctypes.c_void_p()
        flags = ((BUILD_CONSISTENT_M if consistent else 0) | (0 if store_pieces else NO_PIECE_STORE) |
                 (DUAL_BASIS if dual else 0) | (0 if store_B else NO_STORE_B))
        self.dual = bool(dual)
        fn = lib.assemble_coupling if self.dim == 3 else lib.assemble_coupling_2d
        _check(fn(ctypes.byref(g), ctypes.byref(m), FP64 if precision == "fp64" else FP32_MIXED,
                  flags, _stream(stream), ctypes.byref(h)),
               "assemble_coupling" if self.dim == 3 else "assemble_coupling_2d")
        self._h = h
        self.consistent = consistent
        del keep
        self.lattice_shapes = [tuple(len(a) for a in lattice_coords(self.faces, d))
                               for d in range(self.nc)]
        self.n_fluid = [int(np.prod(s)) for s in self.lattice_shapes]

    def _init_unstructured(self, fluid_mesh, X, tets, precision, consistent, dual, stream):
        import torch
        Xf, tets_f = fluid_mesh
        self.faces = None
        self.dim = self.nc = 3
        self.n_vert = int(X.shape[0])
        self.n_tet = int(tets.shape[0])
        if X.ndim != 2 or X.shape[1] != 3 or tets.ndim != 2 or tets.shape[1] != 4:
            raise ValueError("solid: X (n_vert, 3) and tets (n_tet, 4)")
        if Xf.ndim != 2 or Xf.shape[1] != 3 or tets_f.ndim != 2 or tets_f.shape[1] != 4:
            raise ValueError("fluid mesh: X_f (n_vert, 3) and tets_f (n_tet, 4)")
        mf, ms = _Mesh(), _Mesh()
        mf.n_vert, mf.n_tet = int(Xf.shape[0]), int(tets_f.shape[0])
        mf.X = _dev(Xf, torch.float64, 3 * mf.n_vert, "X_f")
        mf.tets = _dev(tets_f, torch.int32, 4 * mf.n_tet, "tets_f")
        ms.n_vert, ms.n_tet = self.n_vert, self.n_tet
        ms.X = _dev(X, torch.float64, 3 * self.n_vert, "X")
        ms.tets = _dev(tets, torch.int32, 4 * self.n_tet, "tets") if self.n_tet else None
        flags = (BUILD_CONSISTENT_M if consistent else 0) | (DUAL_BASIS if dual else 0)
        h = ctypes.c_void_p()
        _check(_lib.assemble_coupling_unstructured(
            ctypes.byref(mf), ctypes.byref(ms), FP64 if precision == "fp64" else FP32_MIXED,
            flags, _stream(stream), ctypes.byref(h)), "assemble_coupling_unstructured")
        self._h = h
        self.lattice_shapes = [(mf.n_vert,)] * 3
        self.n_fluid = [mf.n_vert] * 3

    # -- lifetime ---------------------------------------------------------
    def fsi_step(self, X_ref, u_hat0, v_f, solid, fluid, *, dt, alpha=1.0, eps_abs=0.0,
                 eps_rel=1e-8, max_iter=50, mass="lumped", force_density=False, cg_rtol=1e-10,
                 cg_maxit=500, f_prev=None, stream=None, raise_not_converged=True):
        """One time step of the Picard coupling (Section 3, Steps 1-6) through
        the C driver.  solid(u_hat, f_fsi) fills f_fsi (nc, n_vert) from the
        displacement u_hat; fluid(f_tilde, v_f) updates the nc fluid velocity
        arrays v_f in place from the transferred force (nc = 3, or 2 for a
        planar coupling, whose X_ref is (n_vert, 2); with an unstructured
        coupling the v_f are nodal arrays of the fluid mesh and the force
        density divides by the nodes' lumped volumes ∫ μ_j).  Both receive this
        call's tensors and must enqueue their work on the current stream
        (with an explicit `stream`, that stream is made current for the
        call, so the callbacks and the driver share it).  Returns (report, dict of u_hat, w_s, f_fsi, f_tilde)."""
        import torch
        dt_ = self.dtype
        dev = X_ref.device
        n, nc = self.n_vert, self.nc
        out = dict(u_hat=torch.empty((nc, n), dtype=dt_, device=dev),
                   w_s=torch.empty((nc, n), dtype=dt_, device=dev),
                   f_fsi=torch.empty((nc, n), dtype=dt_, device=dev),
                   f_tilde=[torch.empty_like(v) for v in v_f])
        fp = torch.zeros((nc, n), dtype=dt_, device=dev) if f_prev is None else f_prev
        cfg = _FsiConfig(float(dt), float(alpha), float(eps_abs), float(eps_rel), int(max_iter),
                         LUMPED if mass == "lumped" else CONSISTENT, int(bool(force_density)),
                         int(cg_maxit), float(cg_rtol))
        buf = _FsiBuffers()
        buf.X_ref = _dev(X_ref, torch.float64, self.dim * n, "X_ref")
        buf.u_hat0 = _dev(u_hat0, dt_, nc * n, "u_hat0")
        buf.u_hat = out["u_hat"].data_ptr()
        buf.w_s = out["w_s"].data_ptr()
        buf.f_fsi = out["f_fsi"].data_ptr()
        buf.f_prev = _dev(fp, dt_, nc * n, "f_prev")
        if len(v_f) != nc:
            raise IbvtError(INVALID, "fsi_step", f"v_f needs {nc} fluid arrays")
        for d in range(nc):
            buf.v_f[d] = _dev(v_f[d], dt_, self.n_fluid[d], f"v_f[{d}]")
            buf.f_tilde[d] = out["f_tilde"][d].data_ptr()
        errors = []

        def _solid(ctx, u_ptr, f_ptr, s):
            try:
                solid(out["u_hat"], out["f_fsi"])
                return 0
            except BaseException as e:          # reported after the C call returns
                errors.append(e)
                return INVALID

        def _fluid(ctx, ft_ptr, vf_ptr, s):
            try:
                fluid(out["f_tilde"], v_f)
                return 0
            except BaseException as e:
                errors.append(e)
                return INVALID

        cs, cf = _SOLID_FN(_solid), _FLUID_FN(_fluid)
        rep = _FsiReport()
        # the callbacks enqueue on torch's current stream: make it the
        # driver's stream for the duration of the call, so Steps 3 and 5
        # are ordered with the driver's own kernels
        import contextlib
        scope = torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext()
        with scope:
            st = _lib.fsi_step(self.handle, ctypes.byref(cfg), ctypes.byref(buf), cs, None, cf,
                               None, _stream(stream), ctypes.byref(rep))
        if errors:
            raise errors[0]
        report = FsiReport(int(rep.iterations), bool(rep.converged), float(rep.res_abs),
                           float(rep.res_rel), float(rep.f1_norm))
        if st != IBVT_OK and not (st == NOT_CONVERGED and not raise_not_converged):
            _check(st, "fsi_step")
        out["f_prev"] = fp
        return report, out

    def free(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.coupling_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("coupling was freed")
        return self._h

    def reassemble(self, X, stream=None):
        import torch
        _check(_lib.reassemble_coupling(self.handle,
                                        _dev(X, torch.float64, self.dim * self.n_vert, "X"),
                                        _stream(stream)), "reassemble_coupling")

    # -- operations ---------------------------------------------------------
    def _fluid_ptrs(self, u, what):
        if len(u) != self.nc:
            raise ValueError(f"{what}: need {self.nc} fluid components")
        arr = (ctypes.c_void_p * 3)()
        for d in range(self.nc):
            arr[d] = _dev(u[d], self.dtype, self.n_fluid[d], f"{what}[{d}]")
        return arr

    def velocity(self, u_f, mass: str = "lumped", rtol: float = 1e-10, maxit: int = 500,
                 out=None, stream=None, with_info: bool = False, noalloc: bool = False):
        """u_s = S^{-1} B u_f, returns (nc, n_vert).  noalloc=True calls
        transfer_velocity_noalloc (no device allocation in the library; pass
        `out` to keep the call itself allocation-free)."""
        import torch
        uf = self._fluid_ptrs(u_f, "u_f")
        n = self.nc * self.n_vert
        if out is None:
            out = torch.empty((self.nc, self.n_vert), dtype=self.dtype, device=u_f[0].device)
        info = _SolveInfo()
        fn = _lib.transfer_velocity_noalloc if noalloc else _lib.transfer_velocity
        st = fn(self.handle, uf, _dev(out, self.dtype, n, "u_s"),
                                    LUMPED if mass == "lumped" else CONSISTENT, float(rtol),
                int(maxit), _stream(stream), ctypes.byref(info) if with_info else None)
        _check(st, "transfer_velocity_noalloc" if noalloc else "transfer_velocity")
        if with_info:
            return out, SolveInfo(tuple(info.iterations)[:self.nc],
                                  tuple(info.rel_residual)[:self.nc])
        return out

    def force(self, f_s, f_f, alpha: float = 1.0, load: bool = False, stream=None):
        """f_f[d] += alpha B^dT f_s[d] (in place), returns f_f."""
        ff = self._fluid_ptrs(f_f, "f_f")
        _check(_lib.transfer_force(self.handle, _dev(f_s, self.dtype, self.nc * self.n_vert, "f_s"), ff,
                                   float(alpha), FORCE_IS_LOAD if load else 0, _stream(stream)),
               "transfer_force")
        return f_f

    def velocity_vjp(self, g_us, u_f=None, u_s=None, mass: str = "lumped", g_uf=None, g_X=None,
                     rtol: float = 1e-12, maxit: int = 500, stream=None):
        """Accumulates g_uf (nc fluid arrays) and g_X ((n_vert, dim) float64)."""
        import torch
        n = self.nc * self.n_vert
        uf = self._fluid_ptrs(u_f, "u_f") if u_f is not None else None
        guf = self._fluid_ptrs(g_uf, "g_uf") if g_uf is not None else None
        _check(_lib.transfer_velocity_vjp(
            self.handle, _dev(g_us, self.dtype, n, "g_us"), uf,
            _dev(u_s, self.dtype, n, "u_s") if u_s is not None else None,
            LUMPED if mass == "lumped" else CONSISTENT, float(rtol), int(maxit), guf,
            _dev(g_X, torch.float64, self.dim * self.n_vert, "g_X") if g_X is not None else None,
            _stream(stream)), "transfer_velocity_vjp")

    def force_vjp(self, g_ff, f_s=None, alpha: float = 1.0, g_fs=None, g_X=None, stream=None):
        import torch
        n = self.nc * self.n_vert
        gff = self._fluid_ptrs(g_ff, "g_ff")
        _check(_lib.transfer_force_vjp(
            self.handle, gff, _dev(f_s, self.dtype, n, "f_s") if f_s is not None else None,
            float(alpha), _dev(g_fs, self.dtype, n, "g_fs") if g_fs is not None else None,
            _dev(g_X, torch.float64, self.dim * self.n_vert, "g_X") if g_X is not None else None,
            _stream(stream)), "transfer_force_vjp")

    def vjp(self, g_us, g_ff, u_f=None, u_s=None, f_s=None, mass: str = "lumped",
            alpha: float = 1.0, g_uf=None, g_fs=None, g_X=None, rtol: float = 1e-12,
            maxit: int = 500, stream=None):
        """velocity_vjp and force_vjp in one call (one pass over the stored
        piece moments for both shape terms when they are kept)."""
        import torch
        n = self.nc * self.n_vert
        uf = self._fluid_ptrs(u_f, "u_f") if u_f is not None else None
        guf = self._fluid_ptrs(g_uf, "g_uf") if g_uf is not None else None
        gff = self._fluid_ptrs(g_ff, "g_ff")
        _check(_lib.transfer_vjp(
            self.handle, _dev(g_us, self.dtype, n, "g_us"), uf,
            _dev(u_s, self.dtype, n, "u_s") if u_s is not None else None,
            LUMPED if mass == "lumped" else CONSISTENT, float(rtol), int(maxit), guf, gff,
            _dev(f_s, self.dtype, n, "f_s") if f_s is not None else None, float(alpha),
            _dev(g_fs, self.dtype, n, "g_fs") if g_fs is not None else None,
            _dev(g_X, torch.float64, self.dim * self.n_vert, "g_X") if g_X is not None else None,
            _stream(stream)), "transfer_vjp")

    def info(self) -> dict:
        i = _Info()
        _check(_lib.coupling_info(self.handle, ctypes.byref(i)), "coupling_info")
        return dict(precision=i.precision, has_consistent_mass=bool(i.has_consistent_mass),
                    n_vert=i.n_vert, n_tet=i.n_tet,
                    lattice=[[i.lattice[d][e] for e in range(3)] for d in range(3)],
                    n_fluid=list(i.n_fluid), pairs=i.pairs, pieces=i.pieces, dropped=i.dropped,
                    zero_tets=i.zero_tets, nnz=list(i.nnz), touched=list(i.touched),
                    nnz_mass=i.nnz_mass, device_bytes=i.device_bytes, assemblies=i.assemblies,
                    subtets=i.subtets, piece_store=bool(i.piece_store),
                    dist_evals=i.dist_evals, cut_points=i.cut_points, dual=bool(i.dual),
                    dim=i.dim, unstructured=bool(i.unstructured), plane_cuts=i.plane_cuts,
                    matrix_free=bool(i.matrix_free))

    def release_scratch(self, stream=None):
        """Return the assembly-only device memory (coupling_release_scratch);
        transfers and the reverse mode keep working, and the next
        reassembly allocates it again."""
        _check(_lib.coupling_release_scratch(self.handle, _stream(stream)),
               "coupling_release_scratch")

    def body_info(self, tet_offsets, stream=None) -> list:
        """Per-body counters (coupling_body_info): body b holds tets
        tet_offsets[b] .. tet_offsets[b+1]-1; a list of dicts."""
        off = np.ascontiguousarray(np.asarray(tet_offsets, dtype=np.int64))
        n = off.size - 1
        if n < 1:
            raise ValueError("tet_offsets needs at least two entries")
        out = (_BodyInfo * n)()
        _check(_lib.coupling_body_info(self.handle, n, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                       out, _stream(stream)), "coupling_body_info")
        return [dict(tets=b.tets, zero_tets=b.zero_tets, pairs=b.pairs, pieces=b.pieces,
                     volume=b.volume) for b in out]

    def export_csr(self, comp: int, transposed: bool = False):
        """(row_ptr, col, val[, row_map]) as numpy arrays (synchronizes)."""
        nr, nz = ctypes.c_int64(), ctypes.c_int64()
        _check(_lib.coupling_export_csr(self.handle, comp, int(transposed), ctypes.byref(nr),
                                        ctypes.byref(nz), None, None, None, None), "export")
        rp = np.empty(nr.value + 1, dtype=np.int32)
        col = np.empty(max(nz.value, 1), dtype=np.int32)
        val = np.empty(max(nz.value, 1), dtype=np.float64)
        rm = np.empty(max(nr.value, 1), dtype=np.int32)
        _check(_lib.coupling_export_csr(self.handle, comp, int(transposed), ctypes.byref(nr),
                                        ctypes.byref(nz), rp.ctypes.data, col.ctypes.data,
                                        val.ctypes.data, rm.ctypes.data if transposed else None),
               "export")
        col, val = col[:nz.value], val[:nz.value]
        if transposed:
            return rp, col, val, rm[:nr.value]
        return rp, col, val
