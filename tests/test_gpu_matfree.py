"""The coupling without stored matrices (IBVT_NO_STORE_B) on the HIP path,
through the C ABI: every transfer, adjoint and the shape derivative clip and
integrate the pieces again.  Checked against the FP64 oracle with the
tolerances of the assembled path (FP64 1e-12 relative on the transfers,
1e-10 on the adjoints; FP32-mixed 1e-5 / 1e-4), and against the assembled
coupling on the same inputs (the two differ only in summation order: FP64
1e-12, FP32 1e-5 relative).  Also: the autograd recompute form, the dual
multipliers, the refusals (matrix export; planar couplings) and the device
memory held."""
import numpy as np
import pytest

import oracle
from tests.gpu_common import fluid_fields, rel_fro, rel_max, require_gpu, say, to_dev, workload

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}
ADJ = {"fp64": 1e-10, "fp32": 1e-4}
_cache = {}


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


def ref(name, dual=False):
    k = (name, dual)
    if k not in _cache:
        W = workload(name)
        _cache[k] = (W, oracle.assemble(W.faces, W.X, W.tets, dual=dual))
    return _cache[k]


def make(name, prec, dev, store_B, dual=False):
    import torch
    from paper_1810_13046_amd import Coupling
    W, _ = ref(name, dual)
    say(f"[gpu] assemble {name} {prec} store_B={store_B} dual={dual} n_tet={W.tets.shape[0]}")
    c = Coupling(W.faces, to_dev(W.X, torch.float64, dev), to_dev(W.tets, torch.int32, dev),
                 precision=prec, consistent=not dual, dual=dual, store_B=store_B)
    torch.cuda.synchronize()
    return c


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["beam144_grid32", "plate4320_grid256s_tilted",
                                  "three_bodies12k_grid512x256x256s"])
def test_transfers_without_stored_matrices(dev, name, prec):
    import torch
    from paper_1810_13046_amd import IbvtError
    W, R = ref(name)
    c = make(name, prec, dev, store_B=False)
    s = make(name, prec, dev, store_B=True)
    info = c.info()
    assert info["matrix_free"] and not s.info()["matrix_free"]
    assert info["nnz"] == [0, 0, 0] and not info["piece_store"]
    assert info["pairs"] == s.info()["pairs"] and info["zero_tets"] == s.info()["zero_tets"]
    assert info["device_bytes"] < s.info()["device_bytes"]
    with pytest.raises(IbvtError):
        c.export_csr(0)
    dt = c.dtype
    u_f = fluid_fields(W)
    ud = [to_dev(u, dt, dev) for u in u_f]
    say(f"[gpu] matrix-free velocity {name} {prec}")
    us = c.velocity(ud, mass="lumped").cpu().numpy()
    want = oracle.transfer_velocity(R, u_f, "lumped")
    e = rel_fro(us, want)
    say(f"  lumped rel {e:.2e}")
    assert e <= TOL[prec]
    if prec == "fp64":
        assert rel_max(us, want) <= TOL[prec]
    assert rel_fro(us, s.velocity(ud, mass="lumped").cpu().numpy()) <= TOL[prec]
    rtol = 1e-14 if prec == "fp64" else 1e-7
    us2 = c.velocity(ud, mass="consistent", rtol=rtol, maxit=500).cpu().numpy()
    e2 = rel_fro(us2, oracle.transfer_velocity(R, u_f, "consistent"))
    say(f"  consistent rel {e2:.2e}")
    assert e2 <= (5e-12 if prec == "fp64" else TOL[prec])
    f_s = W.f_s()
    alpha = 0.37
    say(f"[gpu] matrix-free force {name} {prec}")
    f0 = [torch.zeros(u.shape, dtype=dt, device=dev) for u in u_f]
    c.force(to_dev(f_s, dt, dev), f0, alpha=alpha)
    wantf = oracle.transfer_force(R, f_s, alpha)
    for d in range(3):
        e = rel_fro(f0[d].cpu().numpy().ravel(), wantf[d])
        say(f"  force d={d} rel {e:.2e}")
        assert e <= TOL[prec], d
    # accumulation into nonzero arrays: each piece's contribution is added
    # to the running value, so the totals agree with the assembled product
    # to rounding of the totals
    base = [to_dev(np.asarray(u) * 0.5, dt, dev) for u in u_f]
    f1 = [b.clone() for b in base]
    c.force(to_dev(f_s, dt, dev), f1, alpha=alpha)
    f2 = [b.clone() for b in base]
    s.force(to_dev(f_s, dt, dev), f2, alpha=alpha)
    for d in range(3):
        assert rel_fro(f1[d].cpu().numpy(), f2[d].cpu().numpy()) <= TOL[prec], d
    c.free()
    s.free()


@pytest.mark.parametrize("mass", ["lumped", "consistent"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_adjoints_without_stored_matrices(dev, prec, mass):
    import torch
    name = "plate4320_grid256s_tilted" if prec == "fp64" else "beam144_grid32"
    W, R = ref(name)
    c = make(name, prec, dev, store_B=False)
    dt = c.dtype
    rtol = 1e-14 if prec == "fp64" else 1e-7
    u_f = fluid_fields(W)
    ud = [to_dev(u, dt, dev) for u in u_f]
    us = c.velocity(ud, mass=mass, rtol=rtol)
    g_us = us.cpu().numpy().astype(np.float64) - W.u_target()
    g_uf = [torch.zeros_like(u) for u in ud]
    g_X = torch.zeros((W.X.shape[0], 3), dtype=torch.float64, device=dev)
    say(f"[gpu] matrix-free velocity vjp {name} {prec} {mass}")
    c.velocity_vjp(to_dev(g_us, dt, dev), u_f=ud, u_s=us, mass=mass, g_uf=g_uf, g_X=g_X,
                   rtol=rtol)
    ref_uf, ref_X = oracle.velocity_vjp(R, u_f, g_us, mass)
    for d in range(3):
        e = rel_fro(g_uf[d].cpu().numpy().ravel(), ref_uf[d])
        assert e <= ADJ[prec], (d, e)
    e = rel_fro(g_X.cpu().numpy(), ref_X)
    say(f"  g_X rel {e:.2e}")
    assert e <= ADJ[prec]
    # force adjoint, and both adjoints in one call
    f_s = W.f_s()
    alpha = 1.7
    g_ff = [to_dev(u, dt, dev) for u in fluid_fields(W, seed_shift=5)]
    g_fs = torch.zeros((3, W.X.shape[0]), dtype=dt, device=dev)
    g_X2 = torch.zeros_like(g_X)
    c.force_vjp(g_ff, f_s=to_dev(f_s, dt, dev), alpha=alpha, g_fs=g_fs, g_X=g_X2)
    rfs, rX = oracle.force_vjp(R, f_s, [g.cpu().numpy().astype(np.float64).ravel() for g in g_ff],
                               alpha)
    assert rel_fro(g_fs.cpu().numpy(), rfs) <= (TOL[prec] if prec == "fp64" else ADJ[prec])
    assert rel_fro(g_X2.cpu().numpy(), rX) <= ADJ[prec]
    g_uf3 = [torch.zeros_like(u) for u in ud]
    g_fs3 = torch.zeros_like(g_fs)
    g_X3 = torch.zeros_like(g_X)
    c.vjp(to_dev(g_us, dt, dev), g_ff, u_f=ud, u_s=us, f_s=to_dev(f_s, dt, dev), mass=mass,
          alpha=alpha, g_uf=g_uf3, g_fs=g_fs3, g_X=g_X3, rtol=rtol)
    assert rel_fro(g_X3.cpu().numpy(), ref_X + rX) <= ADJ[prec]
    assert rel_fro(g_fs3.cpu().numpy(), rfs) <= ADJ[prec]
    c.free()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_dual_basis_without_stored_matrices(dev, prec):
    import torch
    name = "plate4320_grid256s_tilted"
    W, R = ref(name, dual=True)
    c = make(name, prec, dev, store_B=False, dual=True)
    dt = c.dtype
    u_f = fluid_fields(W)
    ud = [to_dev(u, dt, dev) for u in u_f]
    us = c.velocity(ud, mass="lumped").cpu().numpy()
    e = rel_fro(us, oracle.transfer_velocity(R, u_f, "lumped"))
    say(f"[gpu] matrix-free dual velocity {prec} rel {e:.2e}")
    assert e <= TOL[prec]
    f_s = W.f_s()
    f0 = [torch.zeros(u.shape, dtype=dt, device=dev) for u in u_f]
    c.force(to_dev(f_s, dt, dev), f0, alpha=1.0)
    wantf = oracle.transfer_force(R, f_s, 1.0)
    for d in range(3):
        assert rel_fro(f0[d].cpu().numpy().ravel(), wantf[d]) <= TOL[prec], d
    c.free()


def test_autograd_recompute_holds_no_matrices(dev):
    import torch
    from paper_1810_13046_amd.autograd import transfer_velocity
    name = "plate4320_grid256s_tilted"
    W, R = ref(name)
    u_f = fluid_fields(W)
    grads = {}
    for recompute in (False, True):
        X = to_dev(W.X, torch.float64, dev).requires_grad_(True)
        ud = [to_dev(u, torch.float64, dev).requires_grad_(True) for u in u_f]
        us = transfer_velocity(ud, X, W.faces, to_dev(W.tets, torch.int32, dev), precision="fp64",
                               mass="consistent", rtol=1e-14, recompute_B=recompute)
        loss = 0.5 * ((us - to_dev(W.u_target(), torch.float64, dev)) ** 2).sum()
        loss.backward()
        grads[recompute] = (X.grad.cpu().numpy(), [u.grad.cpu().numpy() for u in ud])
    say("[gpu] autograd recompute_B (matrix-free) against stored")
    assert rel_fro(grads[True][0], grads[False][0]) <= 1e-12
    for d in range(3):
        assert rel_fro(grads[True][1][d], grads[False][1][d]) <= 1e-12


def test_planar_and_unstructured_refuse_the_flag(dev):
    import torch
    from paper_1810_13046_amd import Coupling, IbvtError
    import workloads as wl
    W2 = wl.plane.workload2(1)
    with pytest.raises(IbvtError):
        Coupling(W2.faces, to_dev(W2.X, torch.float64, dev), to_dev(W2.tris, torch.int32, dev),
                 store_B=False)
