"""transfer_vjp — the adjoints of the velocity and the force transfer in one
call — on the HIP path, through the C ABI: against the oracle's two adjoints
summed, and against the two separate calls (with stored moments the two
shape contractions share one pass over them; without, the two calls' paths
run in turn).  Also the dual multipliers, the planar and unstructured
couplings, and a refused call that must leave every output untouched.
Tolerances: g_X against the oracle 1e-10 (FP64) / 1e-4 (FP32) relative, as
for the separate calls; fused against separate 1e-12 (FP64) / 1e-5 (FP32),
since only the order of the sums into g_X differs."""
import numpy as np
import pytest

import oracle
import workloads as wl
from tests.gpu_common import fluid_fields, rel_fro, require_gpu, say, to_dev, workload

pytestmark = pytest.mark.gpu

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


def zeros_like_all(c, dev, ud):
    import torch
    g_uf = [torch.zeros_like(u) for u in ud]
    g_fs = torch.zeros((c.nc, c.n_vert), dtype=c.dtype, device=dev)
    g_X = torch.zeros((c.n_vert, c.dim), dtype=torch.float64, device=dev)
    return g_uf, g_fs, g_X


def both_ways(c, dev, ud, us, g_us, g_ff, f_s, alpha, mass, rtol):
    """(fused outputs, separate outputs) as numpy arrays."""
    out = []
    for fused in (True, False):
        g_uf, g_fs, g_X = zeros_like_all(c, dev, ud)
        if fused:
            c.vjp(g_us, g_ff, u_f=ud, u_s=us, f_s=f_s, mass=mass, alpha=alpha, g_uf=g_uf,
                  g_fs=g_fs, g_X=g_X, rtol=rtol)
        else:
            c.velocity_vjp(g_us, u_f=ud, u_s=us, mass=mass, g_uf=g_uf, g_X=g_X, rtol=rtol)
            c.force_vjp(g_ff, f_s=f_s, alpha=alpha, g_fs=g_fs, g_X=g_X)
        out.append(([g.cpu().numpy() for g in g_uf], g_fs.cpu().numpy(), g_X.cpu().numpy()))
    return out


@pytest.mark.parametrize("store", [True, False])
@pytest.mark.parametrize("mass", ["lumped", "consistent"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_vjp_both_matches_oracle_and_separate_calls(dev, prec, mass, store):
    import torch
    from paper_1810_13046_amd import Coupling
    name = "plate4320_grid256s_tilted" if prec == "fp64" else "beam144_grid32"
    W, R = ref(name)
    say(f"[gpu] vjp both {name} {prec} {mass} store={store}")
    c = Coupling(W.faces, to_dev(W.X, torch.float64, dev), to_dev(W.tets, torch.int32, dev),
                 precision=prec, store_pieces=store)
    dt = c.dtype
    rtol = 1e-14 if prec == "fp64" else 1e-7
    u_f = fluid_fields(W)
    g_ff_np = fluid_fields(W, seed_shift=7)
    ud = [to_dev(u, dt, dev) for u in u_f]
    g_ff = [to_dev(u, dt, dev) for u in g_ff_np]
    us = c.velocity(ud, mass=mass, rtol=rtol)
    g_us_np = us.cpu().numpy().astype(np.float64) - W.u_target()
    g_us = to_dev(g_us_np, dt, dev)
    f_s_np = W.f_s()
    f_s = to_dev(f_s_np, dt, dev)
    alpha = 1.7
    (uf1, fs1, X1), (uf2, fs2, X2) = both_ways(c, dev, ud, us, g_us, g_ff, f_s, alpha, mass, rtol)
    ref_uf, ref_Xv = oracle.velocity_vjp(R, u_f, g_us_np, mass)
    ref_fs, ref_Xf = oracle.force_vjp(R, f_s_np, [u.ravel() for u in g_ff_np], alpha)
    tol = 1e-10 if prec == "fp64" else 1e-4
    e = rel_fro(X1, ref_Xv + ref_Xf)
    say(f"  g_X rel to oracle {e:.2e}, to separate calls {rel_fro(X1, X2):.2e}")
    assert e <= tol
    assert rel_fro(X1, X2) <= (1e-12 if prec == "fp64" else 1e-5)
    assert rel_fro(fs1, ref_fs) <= (1e-12 if prec == "fp64" else 1e-5)
    for d in range(3):
        assert rel_fro(uf1[d].ravel(), ref_uf[d]) <= tol
        np.testing.assert_array_equal(uf1[d], uf2[d])
    np.testing.assert_array_equal(fs1, fs2)
    c.free()


def test_vjp_both_dual(dev):
    import torch
    from paper_1810_13046_amd import Coupling
    name = "beam144_grid32"
    W, R = ref(name, dual=True)
    say("[gpu] vjp both dual")
    c = Coupling(W.faces, to_dev(W.X, torch.float64, dev), to_dev(W.tets, torch.int32, dev),
                 precision="fp64", consistent=False, dual=True)
    u_f = fluid_fields(W)
    ud = [to_dev(u, torch.float64, dev) for u in u_f]
    g_ff = [to_dev(u, torch.float64, dev) for u in fluid_fields(W, seed_shift=3)]
    us = c.velocity(ud, mass="lumped")
    g_us = us - to_dev(W.u_target(), torch.float64, dev)
    f_s = to_dev(W.f_s(), torch.float64, dev)
    (uf1, fs1, X1), (uf2, fs2, X2) = both_ways(c, dev, ud, us, g_us, g_ff, f_s, 0.6, "lumped",
                                              1e-12)
    assert rel_fro(X1, X2) <= 1e-12
    np.testing.assert_array_equal(fs1, fs2)
    c.free()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_vjp_both_planar(dev, prec):
    """Planar couplings take the two calls' paths; the result is theirs."""
    import torch
    from paper_1810_13046_amd import Coupling, lattice_coords
    P2 = wl.plane
    W = P2.workload2(2)
    say(f"[gpu] vjp both planar {prec}")
    c = Coupling(W.faces, to_dev(W.X, torch.float64, dev), to_dev(W.tris, torch.int32, dev),
                 precision=prec)
    dt = c.dtype
    k, phi = P2.fourier_modes2(W.n_modes, W.kmax, 2100 + W.key)
    u = [to_dev(P2.fourier_field2(k[d], phi[d], *lattice_coords(W.faces, d), scale=W.extent),
                dt, dev) for d in range(2)]
    g_ff = [torch.flip(x, dims=[0]).contiguous() for x in u]
    us = c.velocity(u, mass="consistent", rtol=1e-12 if prec == "fp64" else 1e-6)
    g_us = us - to_dev(W.u_target(), dt, dev)
    f_s = to_dev(W.f_s(), dt, dev)
    rtol = 1e-12 if prec == "fp64" else 1e-6
    (uf1, fs1, X1), (uf2, fs2, X2) = both_ways(c, dev, u, us, g_us, g_ff, f_s, 1.3,
                                              "consistent", rtol)
    assert rel_fro(X1, X2) <= (1e-12 if prec == "fp64" else 1e-5)
    np.testing.assert_array_equal(fs1, fs2)
    for d in range(2):
        np.testing.assert_array_equal(uf1[d], uf2[d])
    c.free()


def test_vjp_both_unstructured_and_refusals(dev):
    """The unstructured coupling contracts both adjoints in one pass over its
    per-pair integrals; a non-finite α is refused before any output is
    touched."""
    import torch
    from paper_1810_13046_amd import Coupling, IbvtError
    WU = wl.unstructured
    W = WU.workload_u(1)
    say("[gpu] vjp both: unstructured, and a refused call")
    c = Coupling(None, to_dev(W.X, torch.float64, dev), to_dev(W.tets, torch.int32, dev),
                 fluid_mesh=(to_dev(W.Xf, torch.float64, dev), to_dev(W.tets_f, torch.int32, dev)))
    u = [to_dev(x, torch.float64, dev) for x in W.u_f()]
    us = c.velocity(u, mass="lumped")
    g_us = to_dev(W.f_s(), torch.float64, dev)
    f_s = to_dev(W.f_s()[::-1].copy(), torch.float64, dev)
    g_ff = [torch.flip(x, dims=[0]).contiguous() for x in u]
    (uf1, fs1, X1), (uf2, fs2, X2) = both_ways(c, dev, u, us, g_us, g_ff, f_s, 0.9, "lumped",
                                              1e-12)
    for d in range(3):
        np.testing.assert_array_equal(uf1[d], uf2[d])
    np.testing.assert_array_equal(fs1, fs2)
    assert rel_fro(X1, X2) <= 1e-12
    g_uf, g_fs, g_X = zeros_like_all(c, dev, u)
    with pytest.raises(IbvtError) as e:
        c.vjp(g_us, g_ff, u_f=u, u_s=us, f_s=f_s, alpha=float("nan"), g_uf=g_uf, g_fs=g_fs,
              g_X=g_X)
    assert e.value.name == "IBVT_E_INVALID"
    assert all(int(torch.count_nonzero(g)) == 0 for g in g_uf + [g_fs, g_X])
    c.free()
