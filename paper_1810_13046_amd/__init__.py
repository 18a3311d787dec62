"""MI355X-native L2-projection transfer between a staggered rectilinear fluid
grid (Q1 per velocity component) and a P1 tetrahedral solid mesh
(arXiv 1810.13046, Section 2.3).

    from paper_1810_13046_amd import Coupling
    c = Coupling(faces, X, tets, precision="fp64")
    u_s = c.velocity([u0, u1, u2], mass="lumped")
    c.force(f_s, [f0, f1, f2], alpha=1.0)
    report, out = c.fsi_step(X_ref, u_hat0, v_f, solid, fluid, dt=1e-3)   # Section 3

Autograd forms live in paper_1810_13046_amd.autograd.
"""
from .ibvt import (  # noqa: F401
    Coupling, FsiReport, IbvtError, fluid_lumped_volume, lattice_coords, load_library, LIB_PATH,
    EXPORTED, profile_enable, profile_read, use_torch_allocator,
)
