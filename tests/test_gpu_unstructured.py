"""The coupling with an unstructured background (P1 tetrahedral fluid mesh x
P1 solid tets) on the HIP path, through the C ABI, against the oracle
(oracle/unstructured.py): B and B^T entry by entry, the candidate count of
the tree search against the exact box test, transfers (lumped, consistent,
load), the reverse mode with the shape derivative, dual multipliers,
determinism and reassembly, the full-size case by sampled rows and exact
affine reproduction, and error paths.  Tolerances:
FP64 1e-12, FP32 1e-5 relative Frobenius."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as wl
from tests.gpu_common import rel_fro, require_gpu, say, sparse_rel, to_dev

pytestmark = pytest.mark.gpu

WU = wl.unstructured
TOL = {"fp64": 1e-12, "fp32": 1e-5}
_cache = {}


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


@pytest.fixture(scope="module")
def un():
    from oracle import unstructured
    unstructured.build(force=False)
    return unstructured


def ref(un, key, dual=False):
    k = (key, dual)
    if k not in _cache:
        W = WU.workload_u(key)
        _cache[k] = (W, un.assemble(W.Xf, W.tets_f, W.X, W.tets, dual=dual))
    return _cache[k]


def make(W, prec, dev, consistent=True, dual=False, X=None):
    import torch
    from paper_1810_13046_amd import Coupling
    X = W.X if X is None else X
    c = Coupling(None, to_dev(X, torch.float64, dev), to_dev(W.tets, torch.int32, dev),
                 precision=prec, consistent=consistent, dual=dual,
                 fluid_mesh=(to_dev(W.Xf, torch.float64, dev),
                             to_dev(W.tets_f, torch.int32, dev)))
    torch.cuda.synchronize()
    return c


def gpu_B(c):
    rp, col, val = c.export_csr(0)
    return sp.csr_matrix((val, col, rp), shape=(c.n_vert, c.n_fluid[0]))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("key", [1, 2])
def test_unstructured_B_matches_oracle(dev, un, key, prec):
    W, R = ref(un, key)
    say(f"[gpu] unstructured assemble {W.name} {prec}")
    c = make(W, prec, dev)
    info = c.info()
    assert info["unstructured"] and info["n_fluid"] == [W.Xf.shape[0]] * 3
    # the tree search returns exactly the pairs whose closed boxes meet
    assert info["pairs"] == R.stats["pairs"]
    assert abs(info["pieces"] - R.stats["pieces"]) <= 4
    G = gpu_B(c)
    fro, mx = sparse_rel(G, R.B)
    say(f"  B: nnz {G.nnz} (oracle {R.B.nnz}) rel fro {fro:.2e} max {mx:.2e}")
    assert fro <= TOL[prec] and (prec == "fp32" or mx <= TOL[prec])
    for d in range(3):   # the components share B
        rp, col, val = c.export_csr(d)
        assert val.size == G.nnz
    rp, col, val, rm = c.export_csr(0, transposed=True)
    Bt = sp.csr_matrix((val, col, rp), shape=(rm.size, c.n_vert))
    assert sparse_rel(Bt, R.B.T.tocsr()[rm])[0] <= TOL[prec]
    c.free()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_unstructured_transfers_match_oracle(dev, un, prec):
    import torch
    W, R = ref(un, 2)
    c = make(W, prec, dev)
    dt = c.dtype
    u_f = W.u_f()
    ud = [to_dev(u, dt, dev) for u in u_f]
    for mass in ("lumped", "consistent"):
        say(f"[gpu] unstructured velocity {prec} {mass}")
        us = c.velocity(ud, mass=mass, rtol=1e-13 if prec == "fp64" else 1e-6).cpu().numpy()
        want = un.transfer_velocity(R, u_f, mass)
        e = rel_fro(us, want)
        say(f"  rel {e:.2e}")
        assert e <= (TOL[prec] if mass == "lumped" else (1e-11 if prec == "fp64" else 1e-5))
    f_s = W.f_s()
    for load in (False, True):
        say(f"[gpu] unstructured force load={load} {prec}")
        base = np.random.default_rng(5).standard_normal(u_f.shape)
        ff = [to_dev(b, dt, dev) for b in base]
        c.force(to_dev(f_s, dt, dev), ff, alpha=0.8, load=load)
        want = un.transfer_force(R, f_s, 0.8, load=load, base=base)
        for d in range(3):
            e = rel_fro(ff[d].cpu().numpy(), want[d])
            assert e <= (TOL[prec] if not load else (1e-10 if prec == "fp64" else 1e-5)), (d, e)
    # reverse mode: fluid cotangents and the shape derivative, both adjoints
    g_tol = 1e-10 if prec == "fp64" else 1e-4
    g_us_np = np.random.default_rng(8).standard_normal((3, W.X.shape[0]))
    g_us = to_dev(g_us_np, dt, dev)
    for mass in ("lumped", "consistent"):
        say(f"[gpu] unstructured velocity vjp {prec} {mass}")
        rt = 1e-14 if prec == "fp64" else 1e-7
        us = c.velocity(ud, mass=mass, rtol=rt)
        g_uf = [torch.zeros_like(u) for u in ud]
        g_X = torch.zeros((W.X.shape[0], 3), dtype=torch.float64, device=dev)
        c.velocity_vjp(g_us, u_f=ud, u_s=us, mass=mass, g_uf=g_uf, g_X=g_X, rtol=rt)
        want_uf, want_X = un.velocity_vjp(R, u_f, g_us_np, mass)
        e = rel_fro(g_X.cpu().numpy(), want_X)
        say(f"  g_X rel {e:.2e}")
        assert e <= g_tol
        for d in range(3):
            assert rel_fro(g_uf[d].cpu().numpy(), want_uf[d]) <= g_tol
    say(f"[gpu] unstructured force vjp {prec}")
    g_ff_np = np.random.default_rng(9).standard_normal((3, W.Xf.shape[0]))
    g_fs = torch.zeros((3, W.X.shape[0]), dtype=dt, device=dev)
    g_X = torch.zeros((W.X.shape[0], 3), dtype=torch.float64, device=dev)
    c.force_vjp([to_dev(g, dt, dev) for g in g_ff_np], f_s=to_dev(f_s, dt, dev), alpha=1.3,
                g_fs=g_fs, g_X=g_X)
    want_fs, want_X = un.force_vjp(R, f_s, g_ff_np, 1.3)
    e = rel_fro(g_X.cpu().numpy(), want_X)
    say(f"  g_X rel {e:.2e}")
    assert e <= g_tol
    assert rel_fro(g_fs.cpu().numpy(), want_fs) <= TOL[prec]
    c.free()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_unstructured_dual(dev, un, prec):
    W, R = ref(un, 1, dual=True)
    c = make(W, prec, dev, consistent=False, dual=True)
    say(f"[gpu] unstructured dual {prec}")
    assert sparse_rel(gpu_B(c), R.B)[0] <= TOL[prec]
    co = (0.2, -0.7, 1.3, 0.5)
    u = WU.linear_fields(W.Xf, co)
    us = c.velocity([to_dev(u, c.dtype, dev)] * 3, mass="lumped").cpu().numpy()
    assert np.max(np.abs(us - WU.linear_fields(W.X, co)[None, :])) <= (
        1e-11 if prec == "fp64" else 1e-5)
    # the shape derivative with the dual weights
    import torch
    u_f = W.u_f()
    ud = [to_dev(x, c.dtype, dev) for x in u_f]
    usd = c.velocity(ud, mass="lumped")
    g_us_np = np.random.default_rng(10).standard_normal((3, W.X.shape[0]))
    g_X = torch.zeros((W.X.shape[0], 3), dtype=torch.float64, device=dev)
    c.velocity_vjp(to_dev(g_us_np, c.dtype, dev), u_f=ud, u_s=usd, mass="lumped", g_X=g_X)
    _, want_X = un.velocity_vjp(R, u_f, g_us_np, "lumped")
    assert rel_fro(g_X.cpu().numpy(), want_X) <= (1e-10 if prec == "fp64" else 1e-4)
    c.free()


def test_unstructured_determinism_and_reassembly(dev, un):
    import torch
    W, _ = ref(un, 1)
    c1 = make(W, "fp64", dev)
    c2 = make(W, "fp64", dev)
    for a, b in zip(c1.export_csr(0), c2.export_csr(0)):
        assert np.array_equal(a, b)
    X1 = W.X + 4e-3 * np.sin(5.0 * W.X[:, [2, 0, 1]])
    say("[gpu] unstructured reassemble")
    c1.reassemble(to_dev(X1, torch.float64, dev))
    R1 = un.assemble(W.Xf, W.tets_f, X1, W.tets)
    fro, mx = sparse_rel(gpu_B(c1), R1.B)
    assert fro <= 1e-12 and mx <= 1e-12
    assert c1.info()["assemblies"] == 2
    c1.free()
    c2.free()


def test_unstructured_wide_rows_fall_back_to_sort(dev, un):
    """Rows are gathered one wavefront per solid vertex in LDS; a vertex
    whose tets meet more fluid vertices than that holds sends the assembly
    through the sort-based path.  Both sum every entry in pair order, so the
    rows of the beam's vertices come out bit-identical either way."""
    import torch
    from paper_1810_13046_amd import profile_enable, profile_read
    W, R = ref(un, 1)
    big = np.array([[0.1, 0.1, 0.1], [0.9, 0.1, 0.1], [0.1, 0.9, 0.1], [0.1, 0.1, 0.9]])
    X2 = np.concatenate([W.X, big])
    n0 = W.X.shape[0]
    T2 = np.concatenate([W.tets, np.arange(n0, n0 + 4, dtype=np.int32)[None, :]])
    runs = {}
    for name, X, T in (("beam", W.X, W.tets), ("beam+big", X2, T2)):
        say(f"[gpu] unstructured rows: {name}")
        torch.cuda.synchronize()
        profile_read()
        profile_enable(True)
        c = make(W, "fp64", dev, X=X) if name == "beam" else Coupling_for(W, X, T, dev)
        prof = profile_read()
        profile_enable(False)
        runs[name] = (c, prof)
    assert "rows_sort" not in runs["beam"][1] and "rows_compact" in runs["beam"][1]
    assert "rows_sort" in runs["beam+big"][1]
    Rb = un.assemble(W.Xf, W.tets_f, X2, T2)
    G2 = gpu_B(runs["beam+big"][0])
    fro, mx = sparse_rel(G2, Rb.B)
    say(f"  sort path rel fro {fro:.2e} max {mx:.2e}; big-tet row nnz {G2[n0:].getnnz(axis=1)}")
    assert fro <= 1e-12 and mx <= 1e-12
    assert G2[n0:].getnnz(axis=1).max() > 256
    rp1, col1, val1 = runs["beam"][0].export_csr(0)
    rp2, col2, val2 = runs["beam+big"][0].export_csr(0)
    assert np.array_equal(rp1, rp2[:n0 + 1])
    assert np.array_equal(col1, col2[:rp1[-1]])
    assert np.array_equal(val1, val2[:rp1[-1]])
    for c, _ in runs.values():
        c.free()


def Coupling_for(W, X, T, dev):
    import torch
    from paper_1810_13046_amd import Coupling
    c = Coupling(None, to_dev(X, torch.float64, dev), to_dev(T, torch.int32, dev),
                 fluid_mesh=(to_dev(W.Xf, torch.float64, dev), to_dev(W.tets_f, torch.int32, dev)))
    torch.cuda.synchronize()
    return c


def test_unstructured_full_size(dev, un):
    """The 5.3M-tet warped fluid mesh with the 200k-tet beam: sampled rows of
    B against the oracle (the rows' full vertex stars), and exact
    reproduction of an affine field by the consistent transfer."""
    import torch
    W = WU.workload_u(3)
    say(f"[gpu] unstructured full size: fluid {W.tets_f.shape[0]} tets, solid {W.tets.shape[0]}")
    c = make(W, "fp64", dev)
    G = gpu_B(c)
    rng = np.random.default_rng(12)
    verts = np.sort(rng.choice(W.X.shape[0], 24, replace=False))
    star = np.nonzero(np.isin(W.tets, verts).any(axis=1))[0]
    Rs = un.assemble(W.Xf, W.tets_f, W.X, W.tets[star])
    fro, mx = sparse_rel(G[verts], Rs.B[verts])
    say(f"  sampled rows rel fro {fro:.2e} max {mx:.2e}")
    assert fro <= 1e-12 and mx <= 1e-12
    co = (0.3, 1.1, -0.4, 0.9)
    u = to_dev(WU.linear_fields(W.Xf, co), torch.float64, dev)
    us, info = c.velocity([u, u, u], mass="consistent", rtol=1e-13, with_info=True)
    err = np.max(np.abs(us.cpu().numpy() - WU.linear_fields(W.X, co)[None, :]))
    say(f"  affine reproduction max error {err:.2e} ({info})")
    assert err <= 1e-10
    c.free()


def test_unstructured_edge_cases(dev, un):
    import torch
    from paper_1810_13046_amd import Coupling, IbvtError
    W, _ = ref(un, 1)
    Xf = to_dev(W.Xf, torch.float64, dev)
    Tf = to_dev(W.tets_f, torch.int32, dev)
    # a solid tet partly outside the fluid mesh: only the inside part counts
    say("[gpu] unstructured edge: solid leaving the fluid mesh")
    S = np.array([[0.8, 0.5, 0.5], [1.2, 0.5, 0.5], [0.9, 0.8, 0.5], [0.9, 0.55, 0.8]])
    T = np.array([[0, 1, 2, 3]], dtype=np.int32)
    c = Coupling(None, to_dev(S, torch.float64, dev), to_dev(T, torch.int32, dev),
                 fluid_mesh=(Xf, Tf))
    R = un.assemble(W.Xf, W.tets_f, S, T)
    assert sparse_rel(gpu_B(c), R.B)[0] <= 1e-12
    assert 0 < gpu_B(c).sum() < abs(np.linalg.det(S[1:] - S[0])) / 6
    c.free()
    say("[gpu] unstructured edge: empty solid mesh")
    c = Coupling(None, to_dev(S, torch.float64, dev), torch.zeros((0, 4), dtype=torch.int32,
                                                                  device=dev),
                 fluid_mesh=(Xf, Tf))
    assert c.info()["nnz"] == [0, 0, 0]
    c.free()
    say("[gpu] unstructured edge: bad indices and NaN")
    bad = W.tets_f.copy()
    bad[3, 2] = W.Xf.shape[0] + 5
    with pytest.raises(IbvtError) as e:
        Coupling(None, to_dev(W.X, torch.float64, dev), to_dev(W.tets, torch.int32, dev),
                 fluid_mesh=(Xf, to_dev(bad, torch.int32, dev)))
    assert e.value.name == "IBVT_E_INVALID"
    Xn = W.Xf.copy()
    Xn[7, 1] = np.nan
    with pytest.raises(IbvtError) as e:
        Coupling(None, to_dev(W.X, torch.float64, dev), to_dev(W.tets, torch.int32, dev),
                 fluid_mesh=(to_dev(Xn, torch.float64, dev), Tf))
    assert e.value.name == "IBVT_E_INVALID"
    say("[gpu] unstructured edge: fsi_step with two fluid arrays refused")
    c = make(W, "fp64", dev)
    v = [torch.zeros(c.n_fluid[0], dtype=torch.float64, device=dev) for _ in range(2)]
    with pytest.raises(IbvtError) as e:
        c.fsi_step(to_dev(W.X, torch.float64, dev),
                   torch.zeros((3, W.X.shape[0]), dtype=torch.float64, device=dev), v,
                   lambda u, f: f.zero_(), lambda ft, vv: None, dt=1.0)
    assert e.value.name == "IBVT_E_INVALID"
    c.free()


@pytest.mark.parametrize("mode,density", [("lumped", False), ("consistent", False),
                                          ("dual", False), ("lumped", True)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_unstructured_fsi_step_matches_oracle(dev, un, prec, mode, density):
    """The Picard driver (Section 3, Steps 1-6) over the unstructured
    coupling, with a linear spring for the solid and a fluid whose nodal
    velocity responds linearly to the force, against the oracle's loop: FP64
    the same iteration count (within one) and fields within 1e-10; FP32-mixed
    within 1e-4 of the FP64 oracle."""
    import torch
    W = WU.workload_u(2)
    n, nf = W.X.shape[0], W.Xf.shape[0]
    dual = mode == "dual"
    mass = "consistent" if mode == "consistent" else "lumped"
    rng = np.random.default_rng(17)
    u_rest = 1e-3 * rng.standard_normal((3, n))
    v_base = [rng.standard_normal(nf) for _ in range(3)]
    k_s, beta = 10.0, 0.5
    if density:  # force densities are loads over node volumes: keep the map contractive
        from oracle import lumped_mass
        beta *= lumped_mass(W.Xf, W.tets_f).min()
    u0 = 1e-3 * np.random.default_rng(4).standard_normal((3, n))
    dt, alpha = 0.05, 0.8
    say(f"[gpu] unstructured fsi_step {prec} {mode} density={density}")
    ref_ = un.fsi_step(W.Xf, W.tets_f, W.X, W.tets, u0, [np.zeros(nf)] * 3,
                       lambda u: -k_s * (u - u_rest),
                       lambda ft: [v_base[d] + beta * ft[d] for d in range(3)],
                       dt, alpha, eps_abs=1e-13, eps_rel=0.0, max_iter=200, mass=mass,
                       force_density=density, dual=dual)
    assert ref_["converged"]
    c = make(W, prec, dev, consistent=(mass == "consistent"), dual=dual)
    dt_ = c.dtype
    ur = to_dev(u_rest, dt_, dev)
    vb = [to_dev(v, dt_, dev) for v in v_base]
    vf = [torch.zeros_like(v) for v in vb]

    def solid(u_hat, f_fsi):
        torch.mul(u_hat - ur, -k_s, out=f_fsi)

    def fluid(f_tilde, v):
        for d in range(3):
            torch.add(vb[d], f_tilde[d], alpha=beta, out=v[d])

    rep, out = c.fsi_step(to_dev(W.X, torch.float64, dev), to_dev(u0, dt_, dev), vf, solid, fluid,
                          dt=dt, alpha=alpha, eps_abs=1e-13 if prec == "fp64" else 0.0,
                          eps_rel=0.0 if prec == "fp64" else 1e-4, max_iter=200, mass=mass,
                          force_density=density, cg_rtol=1e-14 if prec == "fp64" else 1e-7)
    say(f"  iterations gpu {rep.iterations} oracle {ref_['iterations']} res {rep.res_abs:.2e}")
    assert rep.converged
    tol = 1e-10 if prec == "fp64" else 1e-4
    if prec == "fp64":
        assert abs(rep.iterations - ref_["iterations"]) <= 1
    assert rel_fro(out["f_fsi"].cpu().numpy(), ref_["f_fsi"]) <= tol
    assert rel_fro(out["u_hat"].cpu().numpy(), ref_["u_hat"]) <= tol
    assert rel_fro(out["w_s"].cpu().numpy(), ref_["w_s"]) <= tol
    for d in range(3):
        assert rel_fro(out["f_tilde"][d].cpu().numpy(), ref_["f_tilde"][d]) <= tol, d
        assert rel_fro(vf[d].cpu().numpy(), ref_["v_f"][d]) <= tol, d
    c.free()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_unstructured_fsi_density_with_an_orphan_fluid_vertex(dev, un, prec):
    """A fluid vertex no fluid tet uses (zero lumped volume): the driver's
    force density there is zero, every value is finite, and the rest matches
    the oracle's loop."""
    import torch
    W = WU.workload_u(2)
    n, nf = W.X.shape[0], W.Xf.shape[0]
    Xf2 = np.vstack([W.Xf, W.Xf[:1] + 0.01])
    rng = np.random.default_rng(9)
    u0 = 1e-3 * rng.standard_normal((3, n))
    vb = [np.concatenate([rng.standard_normal(nf), [0.0]]) for _ in range(3)]
    say(f"[gpu] unstructured fsi_step with an orphan fluid vertex {prec}")
    ref_ = un.fsi_step(Xf2, W.tets_f, W.X, W.tets, u0, [np.zeros(nf + 1)] * 3,
                       lambda u: -10.0 * u, lambda ft: [vb[d] + 1e-6 * ft[d] for d in range(3)],
                       0.05, 0.8, eps_abs=0.0, eps_rel=0.0, max_iter=2, force_density=True)
    from paper_1810_13046_amd import Coupling
    c = Coupling(None, to_dev(W.X, torch.float64, dev), to_dev(W.tets, torch.int32, dev),
                 precision=prec, consistent=False,
                 fluid_mesh=(to_dev(Xf2, torch.float64, dev), to_dev(W.tets_f, torch.int32, dev)))
    dt_ = c.dtype
    vbd = [to_dev(v, dt_, dev) for v in vb]
    vf = [torch.zeros_like(v) for v in vbd]

    def fluid(f_tilde, v):
        for d in range(3):
            torch.add(vbd[d], f_tilde[d], alpha=1e-6, out=v[d])

    rep, out = c.fsi_step(to_dev(W.X, torch.float64, dev), to_dev(u0, dt_, dev), vf,
                          lambda u, f: torch.mul(u, -10.0, out=f), fluid, dt=0.05, alpha=0.8,
                          eps_abs=0.0, eps_rel=0.0, max_iter=2, force_density=True,
                          raise_not_converged=False)
    tol = 1e-10 if prec == "fp64" else 1e-4
    for d in range(3):
        ft = out["f_tilde"][d].cpu().numpy().astype(np.float64)
        assert np.all(np.isfinite(ft)) and ft[nf] == 0.0
        assert rel_fro(ft, ref_["f_tilde"][d]) <= tol, d
    c.free()
