"""The planar coupling (Q1 quadrilateral lattice x P1 triangles, the setting
of the paper's 2D experiments) on the HIP path, through the C ABI, against
the 2D FP64 oracle (oracle/plane.py): B^d and B^dT element by element,
transfers (lumped, consistent, load), dual multipliers ψ = 4λ − 1, the
reverse mode with the shape derivative, autograd, reassembly, the Picard
driver of Section 3 and edge cases.
Tolerances as in three dimensions: FP64 1e-12, FP32 1e-5 relative Frobenius
for B and the transfers; gradients 1e-10 / 1e-4.

The Turek–Hron-like workloads run at every refinement of the paper's table
up to the reference mesh (43,824 triangles in a 4608 x 762 grid, the size
bench.py times), all compared entry by entry: the 2D oracle finishes them in
seconds."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as wl
from tests.gpu_common import rel_fro, require_gpu, say, sparse_rel, to_dev

pytestmark = pytest.mark.gpu

P2 = wl.plane
TOL = {"fp64": 1e-12, "fp32": 1e-5}
GTOL = {"fp64": 1e-10, "fp32": 1e-4}
_cache = {}


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


@pytest.fixture(scope="module")
def pl():
    from oracle import plane
    plane.build(force=False)
    return plane


def ref(pl, key, dual=False):
    k = (key, dual)
    if k not in _cache:
        W = P2.workload2(key)
        _cache[k] = (W, pl.assemble(W.faces, W.X, W.tris, dual=dual))
    return _cache[k]


def fields(pl, W, shift=0):
    k, phi = P2.fourier_modes2(W.n_modes, W.kmax, 2100 + W.key + shift)
    return [P2.fourier_field2(k[d], phi[d], *pl.lattice(W.faces, d), scale=W.extent)
            for d in range(2)]


def make(W, prec, dev, consistent=True, dual=False, X=None):
    import torch
    from paper_1810_13046_amd import Coupling
    X = W.X if X is None else X
    c = Coupling(W.faces, to_dev(X, torch.float64, dev), to_dev(W.tris, torch.int32, dev),
                 precision=prec, consistent=consistent, dual=dual)
    torch.cuda.synchronize()
    return c


def col_of(c, d):
    return c.export_csr(d)[1]


def gpu_B(c, pl, faces, d):
    rp, col, val = c.export_csr(d)
    return sp.csr_matrix((val, col, rp), shape=(c.n_vert, pl.n_fluid(faces, d)))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("key", [1, 2, 3, 4, 5, 6])
def test_planar_B_and_Bt_match_oracle(dev, pl, key, prec):
    W, R = ref(pl, key)
    say(f"[gpu] planar assemble {W.name} {prec} n_tri={W.tris.shape[0]}")
    c = make(W, prec, dev)
    info = c.info()
    assert info["dim"] == 2 and info["n_tet"] == W.tris.shape[0]
    assert info["pairs"] == R.stats["pairs"]
    # keep decisions at the 1e-14 |T| threshold may differ by rounding
    assert abs(info["pieces"] - R.stats["pieces"]) <= 4
    assert info["zero_tets"] == 0 and info["nnz"][2] == 0
    for d in range(2):
        G = gpu_B(c, pl, W.faces, d)
        fro, mx = sparse_rel(G, R.B[d])
        say(f"  B^{d}: nnz {G.nnz} (oracle {R.B[d].nnz}) rel fro {fro:.2e} max {mx:.2e}")
        assert fro <= TOL[prec] and (prec == "fp32" or mx <= TOL[prec]), (d, fro, mx)
        assert abs(G.nnz - R.B[d].nnz) <= 8
        rp, col, val, rm = c.export_csr(d, transposed=True)
        Bt = sp.csr_matrix((val, col, rp), shape=(rm.size, c.n_vert))
        ref_t = R.B[d].T.tocsr()[rm]
        assert sparse_rel(Bt, ref_t)[0] <= TOL[prec]
        # B^T rows are the touched fluid nodes
        assert np.array_equal(np.sort(rm), np.unique(col_of(c, d)))
    c.free()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("key", [1, 5])
def test_planar_transfers_match_oracle(dev, pl, key, prec):
    import torch
    W, R = ref(pl, key)
    c = make(W, prec, dev)
    dt = c.dtype
    u_f = fields(pl, W)
    ud = [to_dev(u, dt, dev) for u in u_f]
    for mass in ("lumped", "consistent"):
        say(f"[gpu] planar velocity {W.name} {prec} {mass}")
        us, info = c.velocity(ud, mass=mass, rtol=1e-13 if prec == "fp64" else 1e-6,
                              with_info=True)
        assert us.shape == (2, W.X.shape[0])
        want = pl.transfer_velocity(R, u_f, mass)
        e = rel_fro(us.cpu().numpy(), want)
        say(f"  rel {e:.2e} info {info}")
        assert e <= (TOL[prec] if mass == "lumped" else (1e-11 if prec == "fp64" else 1e-5))
    f_s = W.f_s()
    for load in (False, True):
        say(f"[gpu] planar force load={load} {prec}")
        base = [np.random.default_rng(7 + d).standard_normal(u.shape) for d, u in enumerate(u_f)]
        ff = [to_dev(b, dt, dev) for b in base]
        c.force(to_dev(f_s, dt, dev), ff, alpha=0.7, load=load)
        want = pl.transfer_force(R, f_s, 0.7, load=load, base=base)
        for d in range(2):
            e = rel_fro(ff[d].cpu().numpy().ravel(), want[d])
            assert e <= (TOL[prec] if not load else (1e-10 if prec == "fp64" else 1e-5)), (d, e)
    c.free()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_planar_dual_matches_oracle(dev, pl, prec):
    import torch
    from paper_1810_13046_amd import IbvtError
    W, R = ref(pl, 3, dual=True)
    say(f"[gpu] planar dual {W.name} {prec}")
    c = make(W, prec, dev, consistent=False, dual=True)
    assert c.info()["dual"]
    for d in range(2):
        fro, mx = sparse_rel(gpu_B(c, pl, W.faces, d), R.B[d])
        assert fro <= TOL[prec], (d, fro)
    u_f = fields(pl, W)
    ud = [to_dev(u, c.dtype, dev) for u in u_f]
    us = c.velocity(ud, mass="lumped").cpu().numpy()
    assert rel_fro(us, pl.transfer_velocity(R, u_f, "lumped")) <= TOL[prec]
    with pytest.raises(IbvtError):
        c.velocity(ud, mass="consistent")
    f_s = W.f_s()
    ff = [torch.zeros(u.shape, dtype=c.dtype, device=dev) for u in u_f]
    c.force(to_dev(f_s, c.dtype, dev), ff, alpha=1.0, load=True)
    want = pl.transfer_force(R, f_s, 1.0, load=True)
    for d in range(2):
        assert rel_fro(ff[d].cpu().numpy().ravel(), want[d]) <= TOL[prec]
    c.free()


def test_planar_dual_reproduces_affine_fields(dev, pl):
    """ψ_i = 4λ_i − 1 with S = diag(m) reproduces affine fields at every
    vertex, on the reference mesh."""
    import torch
    W = P2.workload2(5)
    c = make(W, "fp64", dev, consistent=False, dual=True)
    co = (0.3, -1.2, 2.1)
    u = []
    for d in range(2):
        xs, ys = pl.lattice(W.faces, d)
        Y, Xg = np.meshgrid(ys, xs, indexing="ij")
        u.append(to_dev(co[0] + co[1] * Xg + co[2] * Y, torch.float64, dev))
    us = c.velocity(u, mass="lumped").cpu().numpy()
    want = co[0] + co[1] * W.X[:, 0] + co[2] * W.X[:, 1]
    err = np.max(np.abs(us - want[None, :]))
    say(f"[gpu] planar dual affine reproduction: max abs error {err:.2e}")
    assert err <= 1e-11
    c.free()


@pytest.mark.parametrize("mass,dual", [("lumped", False), ("consistent", False),
                                       ("lumped", True)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_planar_vjps_match_oracle(dev, pl, prec, mass, dual):
    import torch
    W, R = ref(pl, 2, dual=dual)
    c = make(W, prec, dev, consistent=(mass == "consistent"), dual=dual)
    dt = c.dtype
    u_f = fields(pl, W)
    ud = [to_dev(u, dt, dev) for u in u_f]
    us = c.velocity(ud, mass=mass, rtol=1e-13 if prec == "fp64" else 1e-6)
    g_us = us.cpu().numpy().astype(np.float64) - W.u_target()
    g_uf = [torch.zeros_like(u) for u in ud]
    g_X = torch.zeros((W.X.shape[0], 2), dtype=torch.float64, device=dev)
    say(f"[gpu] planar velocity vjp {prec} {mass} dual={dual}")
    c.velocity_vjp(to_dev(g_us, dt, dev), u_f=ud, u_s=us, mass=mass, g_uf=g_uf, g_X=g_X,
                   rtol=1e-13 if prec == "fp64" else 1e-6)
    ref_uf, ref_X = pl.velocity_vjp(R, u_f, g_us, mass)
    for d in range(2):
        assert rel_fro(g_uf[d].cpu().numpy().ravel(), ref_uf[d]) <= GTOL[prec], d
    e = rel_fro(g_X.cpu().numpy(), ref_X)
    say(f"  g_X rel {e:.2e}")
    assert e <= GTOL[prec]
    f_s = W.f_s()
    g_fs = torch.zeros((2, W.X.shape[0]), dtype=dt, device=dev)
    g_X2 = torch.zeros((W.X.shape[0], 2), dtype=torch.float64, device=dev)
    c.force_vjp(ud, f_s=to_dev(f_s, dt, dev), alpha=1.3, g_fs=g_fs, g_X=g_X2)
    rfs, rX = pl.force_vjp(R, f_s, [u.ravel() for u in u_f], 1.3)
    assert rel_fro(g_fs.cpu().numpy(), rfs) <= TOL[prec]
    assert rel_fro(g_X2.cpu().numpy(), rX) <= GTOL[prec]
    c.free()


def test_planar_autograd_and_reassembly(dev, pl):
    """torch.autograd through the planar transfers, then a moved mesh
    reassembled in place against a fresh oracle assembly."""
    import torch
    from paper_1810_13046_amd import Coupling
    from paper_1810_13046_amd.autograd import transfer_force, transfer_velocity
    W, R = ref(pl, 1)
    u_f = fields(pl, W)
    X = to_dev(W.X, torch.float64, dev).requires_grad_(True)
    tris = to_dev(W.tris, torch.int32, dev)
    ud = [to_dev(u, torch.float64, dev).requires_grad_(True) for u in u_f]
    tgt = to_dev(W.u_target(), torch.float64, dev)
    say("[gpu] planar autograd velocity")
    us = transfer_velocity(ud, X, W.faces, tris, mass="consistent")
    loss = 0.5 * ((us - tgt) ** 2).sum()
    loss.backward()
    g_us = us.detach().cpu().numpy() - W.u_target()
    ref_uf, ref_X = pl.velocity_vjp(R, u_f, g_us, "consistent")
    assert rel_fro(X.grad.cpu().numpy(), ref_X) <= 1e-10
    for d in range(2):
        assert rel_fro(ud[d].grad.cpu().numpy().ravel(), ref_uf[d]) <= 1e-10
    say("[gpu] planar autograd force")
    X.grad = None
    f_s = to_dev(W.f_s(), torch.float64, dev).requires_grad_(True)
    ff = transfer_force(f_s, X, W.faces, tris, alpha=0.9)
    assert len(ff) == 2
    g = [torch.as_tensor(np.random.default_rng(30 + d).standard_normal(tuple(f.shape)),
                         device=dev) for d, f in enumerate(ff)]
    sum((f * gg).sum() for f, gg in zip(ff, g)).backward()
    rfs, rX = pl.force_vjp(R, W.f_s(), [gg.cpu().numpy().ravel() for gg in g], 0.9)
    assert rel_fro(f_s.grad.cpu().numpy(), rfs) <= 1e-12
    assert rel_fro(X.grad.cpu().numpy(), rX) <= 1e-10
    say("[gpu] planar reassembly")
    c = Coupling(W.faces, to_dev(W.X, torch.float64, dev), tris, precision="fp64")
    X1 = W.X + 2e-3 * np.sin(9.0 * W.X[:, [1, 0]])
    c.reassemble(to_dev(X1, torch.float64, dev))
    R1 = pl.assemble(W.faces, X1, W.tris)
    for d in range(2):
        fro, mx = sparse_rel(gpu_B(c, pl, W.faces, d), R1.B[d])
        assert fro <= 1e-12 and mx <= 1e-12
    assert c.info()["assemblies"] == 2
    c.free()


def test_planar_edge_cases(dev, pl):
    import torch
    from paper_1810_13046_amd import Coupling, IbvtError
    faces = [np.linspace(0, 1, 11), np.linspace(0, 1, 9)]
    fx, fy = faces
    mx = 0.5 * (fx[5] + fx[6])          # a vertical line of component 1's lattice
    my = 0.5 * (fy[2] + fy[3])          # a horizontal line of component 0's lattice
    # vertices on grid lines and nodes, edges on cell lines (either side),
    # a zero-area triangle and a triangle inside one cell
    X = np.array([
        [fx[3], 0.25], [fx[3], 0.55], [0.52, my],    # vertical edge on a face line, triangle right of it
        [mx, fy[2]], [mx, fy[5]], [0.41, 0.45],      # vertical edge on a centre line, triangle left of it
        [0.22, fy[3]], [0.71, fy[3]], [fx[5], 0.66], # horizontal edge on a face line
        [0.42, 0.42], [0.44, 0.43], [0.43, 0.46],    # inside one cell
        [0.25, 0.3], [0.35, 0.3], [0.45, 0.3],       # collinear: zero area
    ], dtype=np.float64)
    T = np.arange(15, dtype=np.int32).reshape(5, 3)
    T[1] = T[1, [0, 2, 1]]                          # clockwise
    say("[gpu] planar edge: ties and a zero-area triangle")
    for prec in ("fp64", "fp32"):
        c = Coupling(faces, to_dev(X, torch.float64, dev), to_dev(T, torch.int32, dev),
                     precision=prec)
        R = pl.assemble(faces, X, T)
        assert c.info()["zero_tets"] == 1 == R.stats["zero_tris"]
        for d in range(2):
            fro, mx = sparse_rel(gpu_B(c, pl, faces, d), R.B[d])
            assert fro <= TOL[prec], (prec, d, fro)
        c.free()
    # empty mesh
    say("[gpu] planar edge: empty mesh")
    c = Coupling(faces, to_dev(X, torch.float64, dev), torch.zeros((0, 3), dtype=torch.int32,
                                                                    device=dev))
    u = [torch.ones(n, dtype=torch.float64, device=dev) for n in c.n_fluid]
    assert float(c.velocity(u).abs().sum()) == 0.0
    assert c.info()["nnz"] == [0, 0, 0]
    c.free()
    # out of the lattice hull (below the first cell-centre node 1/16)
    say("[gpu] planar edge: out of grid")
    Xo = X.copy()
    Xo[0] = [0.3, 0.01]
    with pytest.raises(IbvtError) as e:
        Coupling(faces, to_dev(Xo, torch.float64, dev), to_dev(T[:1], torch.int32, dev))
    assert e.value.name == "IBVT_E_OUT_OF_GRID"
    say("[gpu] planar edge: NaN and bad index")
    Xn = X.copy()
    Xn[1, 1] = np.nan
    with pytest.raises(IbvtError) as e:
        Coupling(faces, to_dev(Xn, torch.float64, dev), to_dev(T[:1], torch.int32, dev))
    assert e.value.name == "IBVT_E_INVALID"
    with pytest.raises(IbvtError) as e:
        Coupling(faces, to_dev(X, torch.float64, dev),
                 to_dev(np.array([[0, 1, 99]], dtype=np.int32), torch.int32, dev))
    assert e.value.name == "IBVT_E_INVALID"
    # the Picard driver takes two fluid arrays for a planar coupling
    say("[gpu] planar edge: fsi_step with three fluid arrays refused")
    c = Coupling(faces, to_dev(X, torch.float64, dev), to_dev(T[:1], torch.int32, dev))
    v3 = [torch.zeros(n, dtype=torch.float64, device=dev) for n in c.n_fluid[:2]] * 2
    with pytest.raises(IbvtError) as e:
        c.fsi_step(to_dev(X, torch.float64, dev),
                   torch.zeros((2, X.shape[0]), dtype=torch.float64, device=dev), v3[:3],
                   None, None, dt=1.0)
    assert e.value.name == "IBVT_E_INVALID"
    c.free()


@pytest.mark.parametrize("density", [False, True])
@pytest.mark.parametrize("mode", ["lumped", "consistent", "dual"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fsi_step_matches_oracle(dev, pl, prec, mode, density):
    """The Picard driver (Section 3, Steps 1-6) on a planar coupling, with a
    linear spring for the solid and a fluid responding linearly to the
    force, against the 2D oracle's loop: FP64 the same iteration count
    (within one) and fields within 1e-10; FP32-mixed within 1e-4 of the FP64
    oracle."""
    import torch
    from paper_1810_13046_amd import Coupling
    W = P2.workload2(1)
    n = W.X.shape[0]
    dual = mode == "dual"
    mass = "consistent" if mode == "consistent" else "lumped"
    rng = np.random.default_rng(17)
    u_rest = 1e-3 * rng.standard_normal((2, n))
    v_base = [rng.standard_normal(pl.n_fluid(W.faces, d)) for d in range(2)]
    k_s, beta = 10.0, 0.5
    if density:  # force densities are loads over node areas ~ h^2: keep the map contractive
        beta *= min(pl.fluid_lumped_volume(W.faces, d).min() for d in range(2))
    u0 = 1e-3 * np.random.default_rng(4).standard_normal((2, n))
    dt, alpha = 0.05, 0.8
    eps_abs = 1e-13 if prec == "fp64" else 0.0
    eps_rel = 0.0 if prec == "fp64" else 1e-4
    say(f"[gpu] planar fsi_step {W.name} {prec} {mode} density={density}")
    ref_ = pl.fsi_step(W.faces, W.X, W.tris, u0, [np.zeros_like(v) for v in v_base],
                       lambda u: -k_s * (u - u_rest),
                       lambda ft: [v_base[d] + beta * ft[d] for d in range(2)],
                       dt, alpha, eps_abs=1e-13, eps_rel=0.0, max_iter=200, mass=mass,
                       force_density=density, dual=dual)
    assert ref_["converged"]
    c = Coupling(W.faces, to_dev(W.X, torch.float64, dev), to_dev(W.tris, torch.int32, dev),
                 precision=prec, consistent=(mass == "consistent"), dual=dual)
    dt_ = c.dtype
    ur = to_dev(u_rest, dt_, dev)
    vb = [to_dev(v.reshape(tuple(reversed(pl.lattice_shape(W.faces, d)))), dt_, dev)
          for d, v in enumerate(v_base)]
    vf = [torch.zeros_like(v) for v in vb]

    def solid(u_hat, f_fsi):
        torch.mul(u_hat - ur, -k_s, out=f_fsi)

    def fluid(f_tilde, v):
        for d in range(2):
            torch.add(vb[d], f_tilde[d], alpha=beta, out=v[d])

    rep, out = c.fsi_step(to_dev(W.X, torch.float64, dev), to_dev(u0, dt_, dev), vf, solid, fluid,
                          dt=dt, alpha=alpha, eps_abs=eps_abs, eps_rel=eps_rel, max_iter=200,
                          mass=mass, force_density=density,
                          cg_rtol=1e-14 if prec == "fp64" else 1e-7)
    say(f"  iterations gpu {rep.iterations} oracle {ref_['iterations']} res {rep.res_abs:.2e}")
    assert rep.converged
    tol = GTOL[prec]
    if prec == "fp64":
        assert abs(rep.iterations - ref_["iterations"]) <= 1
    assert rel_fro(out["f_fsi"].cpu().numpy(), ref_["f_fsi"]) <= tol
    assert rel_fro(out["u_hat"].cpu().numpy(), ref_["u_hat"]) <= tol
    assert rel_fro(out["w_s"].cpu().numpy(), ref_["w_s"]) <= tol
    for d in range(2):
        assert out["f_tilde"][d].shape == vb[d].shape
        assert rel_fro(out["f_tilde"][d].cpu().numpy().ravel(), ref_["f_tilde"][d]) <= tol, d
        assert rel_fro(vf[d].cpu().numpy().ravel(), ref_["v_f"][d]) <= tol, d
    c.free()


def test_fluid_lumped_area_matches_oracle(dev, pl):
    """ibvt_fluid_lumped_volume_2d against the planar oracle's lumped areas
    (products of exact 1D hat integrals), on the clustered reference grid."""
    from paper_1810_13046_amd import fluid_lumped_volume
    W = P2.workload2(5)
    say("[gpu] planar lumped areas")
    for d in range(2):
        got = fluid_lumped_volume(W.faces, d, device=dev).cpu().numpy()
        want = pl.fluid_lumped_volume(W.faces, d)
        assert got.shape == want.shape
        assert np.max(np.abs(got - want)) <= 1e-15 * want.max()
