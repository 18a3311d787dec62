"""Dual ("pseudo" L2) multipliers (Section 2.3, eq. biorth) on the HIP path,
through the C ABI, against the FP64 oracle's dual mode: B_ij = ∫ ψ_i N_j
with ψ_i = 5λ_i − 1 per tet, S = diag(m).  Same tolerances as the standard
path (FP64 1e-12, FP32 1e-5 relative Frobenius; gradients 1e-10 / 1e-4),
plus the exact reproduction of affine fields, which holds on the GPU at full
workload size without the oracle."""
import numpy as np
import pytest

import oracle
from tests.gpu_common import (WORKLOADS, fluid_fields, gpu_csr, rel_fro, require_gpu, say,
                              sparse_rel, to_dev, workload)

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}
_cache = {}


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


def ref(name):
    if name not in _cache:
        W = workload(name)
        _cache[name] = (W, oracle.assemble(W.faces, W.X, W.tets, dual=True))
    return _cache[name]


def make(W, prec, dev, store_pieces=True):
    import torch
    from paper_1810_13046_amd import Coupling
    c = Coupling(W.faces, to_dev(W.X, torch.float64, dev), to_dev(W.tets, torch.int32, dev),
                 precision=prec, consistent=False, store_pieces=store_pieces, dual=True)
    torch.cuda.synchronize()
    return c


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(WORKLOADS))
def test_dual_B_matches_oracle(dev, name, prec):
    W, R = ref(name)
    say(f"[gpu] dual assemble {name} {prec}")
    c = make(W, prec, dev)
    assert c.info()["dual"]
    for d in range(3):
        fro, mx = sparse_rel(gpu_csr(c, d, oracle.n_fluid(W.faces, d)), R.B[d])
        say(f"  dual B^{d}: rel fro {fro:.2e} max {mx:.2e}")
        assert fro <= TOL[prec] and (prec == "fp32" or mx <= TOL[prec]), (d, fro, mx)
    c.free()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_dual_transfers_match_oracle(dev, prec):
    import torch
    from paper_1810_13046_amd.ibvt import IbvtError
    W, R = ref("plate4320_grid256s_tilted")
    c = make(W, prec, dev)
    dt = c.dtype
    u_f = fluid_fields(W)
    ud = [to_dev(u, dt, dev) for u in u_f]
    say(f"[gpu] dual velocity {prec}")
    us = c.velocity(ud, mass="lumped").cpu().numpy()
    assert rel_fro(us, oracle.transfer_velocity(R, u_f, "lumped")) <= TOL[prec]
    with pytest.raises(IbvtError):
        c.velocity(ud, mass="consistent")
    f_s = W.f_s()
    for load in (False, True):
        say(f"[gpu] dual force load={load} {prec}")
        f0 = [torch.zeros(u.shape, dtype=dt, device=dev) for u in u_f]
        c.force(to_dev(f_s, dt, dev), f0, alpha=0.6, load=load)
        want = oracle.transfer_force(R, f_s, 0.6, load=load)
        for d in range(3):
            assert rel_fro(f0[d].cpu().numpy().ravel(), want[d]) <= TOL[prec], (load, d)
    c.free()


@pytest.mark.parametrize("store", [True, False])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_dual_vjps_match_oracle(dev, prec, store):
    import torch
    name = "plate4320_grid256s_tilted" if prec == "fp64" else "beam144_grid32"
    W, R = ref(name)
    c = make(W, prec, dev, store_pieces=store)
    dt = c.dtype
    u_f = fluid_fields(W)
    ud = [to_dev(u, dt, dev) for u in u_f]
    us = c.velocity(ud, mass="lumped")
    g_us = us.cpu().numpy().astype(np.float64) - W.u_target()
    g_uf = [torch.zeros_like(u) for u in ud]
    g_X = torch.zeros((W.X.shape[0], 3), dtype=torch.float64, device=dev)
    say(f"[gpu] dual velocity vjp {name} {prec} store={store}")
    c.velocity_vjp(to_dev(g_us, dt, dev), u_f=ud, u_s=us, mass="lumped", g_uf=g_uf, g_X=g_X)
    ref_uf, ref_X = oracle.velocity_vjp(R, u_f, g_us, "lumped")
    tol = 1e-10 if prec == "fp64" else 1e-4
    for d in range(3):
        assert rel_fro(g_uf[d].cpu().numpy().ravel(), ref_uf[d]) <= tol, d
    e = rel_fro(g_X.cpu().numpy(), ref_X)
    say(f"  g_X rel {e:.2e}")
    assert e <= tol
    f_s = W.f_s()
    g_fs = torch.zeros((3, W.X.shape[0]), dtype=dt, device=dev)
    g_X2 = torch.zeros((W.X.shape[0], 3), dtype=torch.float64, device=dev)
    c.force_vjp(ud, f_s=to_dev(f_s, dt, dev), alpha=1.3, g_fs=g_fs, g_X=g_X2)
    rfs, rX = oracle.force_vjp(R, f_s, [u.ravel() for u in u_f], 1.3)
    assert rel_fro(g_fs.cpu().numpy(), rfs) <= (1e-12 if prec == "fp64" else 1e-5)
    assert rel_fro(g_X2.cpu().numpy(), rX) <= tol
    c.free()


def test_dual_reproduces_affine_fields_full_size(dev):
    """Biorthogonality: with S = diag(m), an affine field is reproduced at
    every vertex — on the three-body workload at full size (FP64)."""
    import torch
    import workloads as wl
    from paper_1810_13046_amd import lattice_coords
    W = wl.workload(5)
    say(f"[gpu] dual affine reproduction, full size n_tet={W.tets.shape[0]}")
    c = make(W, "fp64", dev, store_pieces=False)
    co = (0.25, -0.8, 1.1, 0.45)
    u = []
    for d in range(3):
        xs, ys, zs = [torch.as_tensor(a, device=dev) for a in lattice_coords(W.faces, d)]
        Z, Y, Xg = torch.meshgrid(zs, ys, xs, indexing="ij")
        u.append((co[0] + co[1] * Xg + co[2] * Y + co[3] * Z).contiguous())
    us = c.velocity(u, mass="lumped").cpu().numpy()
    want = co[0] + co[1] * W.X[:, 0] + co[2] * W.X[:, 1] + co[3] * W.X[:, 2]
    err = np.max(np.abs(us - want[None, :]))
    say(f"  max abs error {err:.2e}")
    assert err <= 1e-11
    c.free()
