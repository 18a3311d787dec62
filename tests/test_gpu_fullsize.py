"""Full-size parity in the configuration bench.py times (three bodies,
4.5M tets, 512x256x256 stretched grid; mixed precision and FP64): sampled
rows of B and B^T and the transferred values there are recomputed one by one
by the oracle from the tets that touch them; the stored B^T of one component
is checked to be exactly the transpose of B; the consistent solve is checked
by its residual against the oracle's mass matrix."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workloads as wl
from tests.gpu_common import rel_fro, require_gpu, say, to_dev

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}


@pytest.fixture(scope="module")
def big():
    require_gpu()
    W = wl.workload(5)
    k, phi = wl.fourier_modes(W.n_modes, W.kmax, 2000 + W.cfg)
    u = []
    import torch
    for d in range(3):
        xs, ys, zs = oracle.lattice(W.faces, d)
        u.append(wl.fourier_field(k[d], phi[d], xs, ys, zs, device="cuda:0").cpu().numpy())
    return W, u


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_sampled_rows_full_size(big, prec):
    import torch
    from paper_1810_13046_amd import Coupling
    W, u_f = big
    dev = torch.device("cuda:0")
    say(f"[gpu] full-size assembly {prec} n_tet={W.tets.shape[0]}")
    c = Coupling(W.faces, to_dev(W.X, torch.float64, dev), to_dev(W.tets, torch.int32, dev),
                 precision=prec, consistent=True)
    dt = c.dtype
    ud = [to_dev(a, dt, dev) for a in u_f]
    us = c.velocity(ud, mass="lumped").cpu().numpy().astype(np.float64)
    f_s = W.f_s()
    ff = [torch.zeros(a.shape, dtype=dt, device=dev) for a in u_f]
    c.force(to_dev(f_s, dt, dev), ff, alpha=1.0)
    ff = [a.cpu().numpy().astype(np.float64).ravel() for a in ff]
    usc, info = c.velocity(ud, mass="consistent", rtol=1e-10, maxit=500, with_info=True)
    usc = usc.cpu().numpy().astype(np.float64)
    bounds = oracle.tet_bounds(W.X, W.tets)
    rng = np.random.default_rng(77)
    verts = np.sort(rng.choice(W.X.shape[0], 48, replace=False))
    star = oracle.vertex_star(W.tets, verts)
    R = oracle.assemble(W.faces, W.X, W.tets, subset=star)
    m = oracle.lumped_mass(W.X, W.tets[star], n_vert=W.X.shape[0])
    for d in range(3):
        rp, col, val = c.export_csr(d)
        G = sp.csr_matrix((val, col, rp), shape=(W.X.shape[0], oracle.n_fluid(W.faces, d)))
        Gs, Rs = G[verts], R.B[d][verts]
        e = sp.linalg.norm(Gs - Rs) / sp.linalg.norm(Rs)
        say(f"  B^{d} sampled rows rel {e:.2e}")
        assert e <= TOL[prec]
        want = (Rs @ u_f[d].ravel()) / m[verts]
        assert rel_fro(us[d][verts], want) <= TOL[prec]
        # sampled fluid rows of B^T: nodes touched by the sampled rows
        cols = np.unique(Rs.indices)
        pick = np.sort(rng.choice(cols, min(24, cols.size), replace=False))
        nx, ny, _ = oracle.lattice_shape(W.faces, d)
        sub = np.unique(np.concatenate([
            oracle.tets_touching_node(W.faces, W.X, W.tets, d,
                                      (j % nx, (j // nx) % ny, j // (nx * ny)), bounds)
            for j in pick]))
        Rc = oracle.assemble(W.faces, W.X, W.tets, subset=sub).B[d].tocsc()[:, pick]
        Gc = G.tocsc()[:, pick]
        e = sp.linalg.norm(Gc - Rc) / sp.linalg.norm(Rc)
        say(f"  B^{d}T sampled columns rel {e:.2e}")
        assert e <= TOL[prec]
        assert rel_fro(ff[d][pick], Rc.T @ f_s[d]) <= TOL[prec]
        if d == 0:
            # the stored B^T (the radix-sort path at this size) is exactly the
            # transpose of B, each row's vertices ascending
            trp, tcol, tval, rmap = c.export_csr(d, transposed=True)
            Tt = sp.csr_matrix((tval, tcol, trp), shape=(rmap.size, W.X.shape[0]))
            assert np.all(np.diff(rmap) > 0) and rmap.size == np.unique(G.indices).size
            assert abs(Tt - G.T.tocsr()[rmap]).max() == 0.0
            starts = trp[:-1]
            inner = np.ones(tcol.size, dtype=bool)
            inner[starts] = False
            assert np.all(np.diff(tcol)[inner[1:]] > 0)
            say(f"  B^{d}T: exact transpose of {G.nnz} nonzeros")
        # consistent solve: M u_s = B u_f with the oracle's M and the GPU's B
        if d == 0:
            M = oracle.consistent_mass(W.X, W.tets)
        b = G @ u_f[d].ravel()
        res = np.linalg.norm(b - M @ usc[d]) / np.linalg.norm(b)
        say(f"  consistent residual d={d}: {res:.2e} (reported {info.rel_residual[d]:.2e})")
        assert res <= (1e-9 if prec == "fp64" else 1e-5)
    c.free()
