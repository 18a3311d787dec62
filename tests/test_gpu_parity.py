"""Parity of the HIP path with the FP64 oracle, through the C ABI.

Tolerances (from the precision policy of the transfer): FP64 path 1e-12
relative (Frobenius and max-entry) on B, B^T and the transferred fields;
FP32-mixed path 1e-5 relative Frobenius.  Sparsity patterns are not
compared (a piece at the drop threshold may be kept on one side only):
differences are taken with missing entries as zeros.
"""
import numpy as np
import pytest

import oracle
from tests.gpu_common import (WORKLOADS, fluid_fields, gpu_csr, rel_fro, rel_max, require_gpu,
                              say, sparse_rel, to_dev, workload)

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


_cache = {}


def ref(name):
    if name not in _cache:
        W = workload(name)
        _cache[name] = (W, oracle.assemble(W.faces, W.X, W.tets))
    return _cache[name]


def make(name, prec, dev, consistent=True, store_pieces=True):
    import torch
    from paper_1810_13046_amd import Coupling
    W, _ = ref(name)
    say(f"[gpu] assemble {name} {prec} n_tet={W.tets.shape[0]} store={store_pieces}")
    c = Coupling(W.faces, to_dev(W.X, torch.float64, dev), to_dev(W.tets, torch.int32, dev),
                 precision=prec, consistent=consistent, store_pieces=store_pieces)
    torch.cuda.synchronize()
    return c


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(WORKLOADS))
def test_B_and_Bt_match_oracle(dev, name, prec):
    W, R = ref(name)
    c = make(name, prec, dev)
    info = c.info()
    for d in range(3):
        nf = oracle.n_fluid(W.faces, d)
        G = gpu_csr(c, d, nf)
        fro, mx = sparse_rel(G, R.B[d])
        say(f"  B^{d}: nnz gpu {G.nnz} oracle {R.B[d].nnz} rel fro {fro:.2e} max {mx:.2e}")
        assert fro <= TOL[prec] and (prec == "fp32" or mx <= TOL[prec]), (d, fro, mx)
        # columns sorted and unique within rows
        rp, col = G.indptr, G.indices
        for i in range(0, G.shape[0], max(1, G.shape[0] // 200)):
            seg = col[rp[i]:rp[i + 1]]
            assert np.all(np.diff(seg) > 0)
        # the transposed copy is exactly the transpose of B
        trp, tcol, tval, rmap = gpu_csr(c, d, nf, transposed=True)
        import scipy.sparse as sp
        T = sp.csr_matrix((tval, tcol, trp), shape=(rmap.size, W.X.shape[0]))
        full = sp.csr_matrix((T.data, T.indices, T.indptr), shape=T.shape)
        Gt = G.T.tocsr()[rmap]
        assert (abs(full - Gt)).max() == 0.0
        assert np.all(np.diff(rmap) > 0)
        assert info["touched"][d] == rmap.size
        assert info["nnz"][d] == G.nnz
    assert abs(info["pieces"] - R.stats["pieces"]) <= max(2, R.stats["pieces"] // 10000)
    assert info["zero_tets"] == 0
    c.free()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["beam144_grid32", "plate4320_grid256s_tilted",
                                  "three_bodies12k_grid512x256x256s"])
def test_transfers_match_oracle(dev, name, prec):
    import torch
    W, R = ref(name)
    c = make(name, prec, dev)
    dt = c.dtype
    u_f = fluid_fields(W)
    ud = [to_dev(u, dt, dev) for u in u_f]
    say(f"[gpu] velocity lumped {name} {prec}")
    us = c.velocity(ud, mass="lumped").cpu().numpy()
    want = oracle.transfer_velocity(R, u_f, "lumped")
    e = rel_fro(us, want)
    say(f"  lumped rel {e:.2e}")
    assert e <= TOL[prec]
    if prec == "fp64":
        assert rel_max(us, want) <= TOL[prec]
    say(f"[gpu] velocity consistent {name} {prec}")
    rtol = 1e-14 if prec == "fp64" else 1e-7
    us2, inf = c.velocity(ud, mass="consistent", rtol=rtol, maxit=500, with_info=True)
    want2 = oracle.transfer_velocity(R, u_f, "consistent")
    e2 = rel_fro(us2.cpu().numpy(), want2)
    say(f"  consistent rel {e2:.2e} iters {inf.iterations} res {inf.rel_residual}")
    assert e2 <= (5e-12 if prec == "fp64" else TOL[prec])
    assert max(inf.rel_residual) <= rtol * 1.0001
    # force into zero arrays, compared with the oracle
    f_s = W.f_s()
    alpha = 0.37
    say(f"[gpu] force {name} {prec}")
    f0 = [torch.zeros(u.shape, dtype=dt, device=dev) for u in u_f]
    c.force(to_dev(f_s, dt, dev), f0, alpha=alpha)
    wantf = oracle.transfer_force(R, f_s, alpha)
    for d in range(3):
        e = rel_fro(f0[d].cpu().numpy().ravel(), wantf[d])
        say(f"  force d={d} rel {e:.2e}")
        assert e <= TOL[prec], d
    # accumulation: f_f += alpha B^T f_s leaves untouched nodes bitwise alone
    base = [to_dev(np.asarray(u) * 0.5, dt, dev) for u in u_f]
    acc = [b.clone() for b in base]
    c.force(to_dev(f_s, dt, dev), acc, alpha=alpha)
    for d in range(3):
        assert torch.equal(acc[d], base[d] + f0[d])
    # force with a load vector (literal transpose of S^{-1} B)
    fd2 = [torch.zeros_like(x) for x in f0]
    c.force(to_dev(f_s, dt, dev), fd2, alpha=alpha, load=True)
    wantl = oracle.transfer_force(R, f_s, alpha, load=True)
    for d in range(3):
        assert rel_fro(fd2[d].cpu().numpy().ravel(), wantl[d]) <= (1e-10 if prec == "fp64" else 1e-4)
    c.free()


@pytest.mark.parametrize("store", [True, False])
@pytest.mark.parametrize("mass", ["lumped", "consistent"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_velocity_vjp_matches_oracle(dev, mass, prec, store):
    import torch
    name = "plate4320_grid256s_tilted" if prec == "fp64" else "beam144_grid32"
    W, R = ref(name)
    c = make(name, prec, dev, store_pieces=store)
    assert c.info()["piece_store"] == store
    dt = c.dtype
    u_f = fluid_fields(W)
    ud = [to_dev(u, dt, dev) for u in u_f]
    us = c.velocity(ud, mass=mass, rtol=1e-14 if prec == "fp64" else 1e-7)
    u_t = W.u_target()
    g_us = us.cpu().numpy().astype(np.float64) - u_t
    g_uf = [torch.zeros_like(u) for u in ud]
    g_X = torch.zeros((W.X.shape[0], 3), dtype=torch.float64, device=dev)
    say(f"[gpu] velocity vjp {name} {prec} {mass}")
    c.velocity_vjp(to_dev(g_us, dt, dev), u_f=ud, u_s=us, mass=mass, g_uf=g_uf, g_X=g_X,
                   rtol=1e-14 if prec == "fp64" else 1e-7)
    ref_uf, ref_X = oracle.velocity_vjp(R, u_f, g_us, mass)
    tol = 1e-10 if prec == "fp64" else 1e-4
    for d in range(3):
        e = rel_fro(g_uf[d].cpu().numpy().ravel(), ref_uf[d])
        assert e <= tol, (d, e)
    e = rel_fro(g_X.cpu().numpy(), ref_X)
    say(f"  g_X rel {e:.2e}")
    assert e <= tol
    c.free()


def test_force_vjp_matches_oracle(dev):
    import torch
    name = "plate4320_grid256s_tilted"
    W, R = ref(name)
    c = make(name, "fp64", dev)
    u_f = fluid_fields(W)
    g_ff = [to_dev(u, torch.float64, dev) for u in u_f]
    f_s = W.f_s()
    alpha = 1.7
    g_fs = torch.zeros((3, W.X.shape[0]), dtype=torch.float64, device=dev)
    g_X = torch.zeros((W.X.shape[0], 3), dtype=torch.float64, device=dev)
    say("[gpu] force vjp")
    c.force_vjp(g_ff, f_s=to_dev(f_s, torch.float64, dev), alpha=alpha, g_fs=g_fs, g_X=g_X)
    rfs, rX = oracle.force_vjp(R, f_s, [u.ravel() for u in u_f], alpha)
    assert rel_fro(g_fs.cpu().numpy(), rfs) <= 1e-12
    assert rel_fro(g_X.cpu().numpy(), rX) <= 1e-10
    c.free()


def test_assembly_is_bitwise_deterministic_and_reassembly_matches(dev):
    import torch
    name = "three_bodies12k_grid512x256x256s"
    W, _ = ref(name)
    c1 = make(name, "fp64", dev)
    c2 = make(name, "fp64", dev)
    for d in range(3):
        a = c1.export_csr(d)
        b = c2.export_csr(d)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
    # move the mesh, reassemble c1 in place, compare with a fresh assembly at X1
    X1 = W.X + 1e-3 * np.sin(7.0 * W.X[:, [1, 2, 0]])
    say("[gpu] reassemble")
    c1.reassemble(to_dev(X1, torch.float64, dev))
    R1 = oracle.assemble(W.faces, X1, W.tets)
    for d in range(3):
        G = gpu_csr(c1, d, oracle.n_fluid(W.faces, d))
        fro, mx = sparse_rel(G, R1.B[d])
        assert fro <= 1e-12 and mx <= 1e-12
    assert c1.info()["assemblies"] == 2
    c1.free()
    c2.free()


def test_edge_cases(dev):
    import torch
    from paper_1810_13046_amd import Coupling, IbvtError
    faces = [np.linspace(0, 1, 9)] * 3
    X = np.array([[0.4, 0.4, 0.4], [0.6, 0.41, 0.42], [0.45, 0.6, 0.43], [0.44, 0.45, 0.6],
                  [0.5, 0.5, 0.5]], dtype=np.float64)
    # empty mesh: no tets, every transfer is zero
    say("[gpu] edge: empty mesh")
    c = Coupling(faces, to_dev(X, torch.float64, dev), torch.zeros((0, 4), dtype=torch.int32, device=dev))
    u = [torch.ones(n, dtype=torch.float64, device=dev) for n in c.n_fluid]
    assert float(c.velocity(u).abs().sum()) == 0.0
    assert c.info()["nnz"] == [0, 0, 0]
    c.free()
    # a zero-volume tet next to a valid one: counted, contributes nothing
    say("[gpu] edge: zero-volume tet")
    T = np.array([[0, 1, 2, 3], [0, 1, 4, 2]], dtype=np.int32)
    # vertices 0, 1, 2, 4 all lie in the plane z = 3/8 (exact in binary), so
    # tet (0, 1, 4, 2) has a determinant of exactly zero
    Xz = np.array([[0.375, 0.375, 0.375], [0.625, 0.375, 0.375], [0.375, 0.625, 0.375],
                   [0.4, 0.45, 0.6], [0.5, 0.5, 0.375]], dtype=np.float64)
    c = Coupling(faces, to_dev(Xz, torch.float64, dev), to_dev(T, torch.int32, dev))
    R = oracle.assemble(faces, Xz, T)
    assert c.info()["zero_tets"] == 1
    for d in range(3):
        G = gpu_csr(c, d, oracle.n_fluid(faces, d))
        assert sparse_rel(G, R.B[d])[0] <= 1e-12
    c.free()
    # solid leaving the lattice hull
    say("[gpu] edge: out of grid")
    Xo = X.copy()
    Xo[0] = [0.01, 0.4, 0.4]   # below the first cell-centre node (1/16)
    with pytest.raises(IbvtError) as e:
        Coupling(faces, to_dev(Xo, torch.float64, dev), to_dev(T[:1], torch.int32, dev))
    assert e.value.name == "IBVT_E_OUT_OF_GRID"
    # non-finite coordinate
    say("[gpu] edge: NaN")
    Xn = X.copy()
    Xn[1, 2] = np.nan
    with pytest.raises(IbvtError) as e:
        Coupling(faces, to_dev(Xn, torch.float64, dev), to_dev(T[:1], torch.int32, dev))
    assert e.value.name == "IBVT_E_INVALID"
    # bad vertex index
    say("[gpu] edge: bad index")
    with pytest.raises(IbvtError) as e:
        Coupling(faces, to_dev(X, torch.float64, dev),
                 to_dev(np.array([[0, 1, 2, 9]], dtype=np.int32), torch.int32, dev))
    assert e.value.name == "IBVT_E_INVALID"
    # a mass solve that cannot converge in one iteration
    say("[gpu] edge: mass solve maxit")
    W, _ = ref("beam144_grid32")
    c = make("beam144_grid32", "fp64", dev)
    ud = [to_dev(u, torch.float64, dev) for u in fluid_fields(W)]
    with pytest.raises(IbvtError) as e:
        c.velocity(ud, mass="consistent", rtol=1e-15, maxit=1)
    assert e.value.name == "IBVT_E_NOT_CONVERGED"
    # a loose tolerance: one iteration, and the reported residual meets it
    say("[gpu] edge: mass solve with a loose tolerance")
    _, info = c.velocity(ud, mass="consistent", rtol=20.0, maxit=5, with_info=True)
    assert info.iterations[0] == 1 and max(info.rel_residual) <= 20.0
    c.free()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_failed_reassembly_refuses_transfers_until_reassembled(dev, prec):
    """A reassembly that fails (a vertex leaves the lattice hull) leaves the
    handle unusable: transfers, reverse-mode calls and the export are
    refused on the host; a later successful reassembly makes it usable again
    with the right matrices."""
    import torch
    from paper_1810_13046_amd import IbvtError
    W, R = ref("beam144_grid32")
    c = make("beam144_grid32", prec, dev)
    dt = c.dtype
    ud = [to_dev(u, dt, dev) for u in fluid_fields(W)]
    Xo = W.X.copy()
    Xo[0] = [0.001, 0.5, 0.5]
    say(f"[gpu] failed reassembly {prec}")
    with pytest.raises(IbvtError) as e:
        c.reassemble(to_dev(Xo, torch.float64, dev))
    assert e.value.name == "IBVT_E_OUT_OF_GRID"
    us = torch.zeros((3, W.X.shape[0]), dtype=dt, device=dev)
    for call in (lambda: c.velocity(ud, out=us),
                 lambda: c.velocity(ud, mass="consistent", out=us),
                 lambda: c.force(us, [torch.zeros_like(u) for u in ud]),
                 lambda: c.velocity_vjp(us, u_f=ud, u_s=us,
                                        g_X=torch.zeros((W.X.shape[0], 3), dtype=torch.float64,
                                                        device=dev)),
                 lambda: c.force_vjp(ud, f_s=us, g_fs=torch.zeros_like(us)),
                 lambda: c.vjp(us, ud, u_f=ud, u_s=us, f_s=us,
                               g_X=torch.zeros((W.X.shape[0], 3), dtype=torch.float64,
                                               device=dev)),
                 lambda: c.export_csr(0)):
        with pytest.raises(IbvtError) as e:
            call()
        assert e.value.name == "IBVT_E_INVALID"
    assert float(us.abs().sum()) == 0.0  # nothing was written
    c.reassemble(to_dev(W.X, torch.float64, dev))
    for d in range(3):
        fro, mx = sparse_rel(gpu_csr(c, d, oracle.n_fluid(W.faces, d)), R.B[d])
        assert fro <= TOL[prec]
    c.free()
