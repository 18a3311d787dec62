"""Helpers for the GPU parity tests (inputs come from the seeded generators
and the oracle's lattices; nothing here computes the transfer)."""
from __future__ import annotations

import sys

import numpy as np
import scipy.sparse as sp

import oracle
import workloads as wl


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a HIP device (run with -m 'not gpu' on CPU)")
    from paper_1810_13046_amd import ibvt
    ibvt.load_library()
    return torch.device("cuda:0")


def fluid_fields(W, faces=None, seed_shift=0):
    """u_f per component on the oracle's lattices (numpy, shape (nz,ny,nx))."""
    faces = W.faces if faces is None else faces
    k, phi = wl.fourier_modes(W.n_modes, W.kmax, 2000 + W.cfg + seed_shift)
    out = []
    for d in range(3):
        xs, ys, zs = oracle.lattice(faces, d)
        out.append(wl.fourier_field(k[d], phi[d], xs, ys, zs).numpy())
    return out


def to_dev(a, dtype, dev):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=dev, dtype=dtype).contiguous()


def gpu_csr(cpl, d, n_fluid, transposed=False):
    if transposed:
        rp, col, val, rm = cpl.export_csr(d, True)
        return rp, col, val, rm
    rp, col, val = cpl.export_csr(d)
    return sp.csr_matrix((val, col, rp), shape=(cpl.n_vert, n_fluid))


def rel_fro(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def rel_max(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    m = np.max(np.abs(b)) if b.size else 0.0
    return (np.max(np.abs(a - b)) / (m if m > 0 else 1.0)) if a.size else 0.0


def sparse_rel(A, B):
    """Relative Frobenius and max-abs difference of two sparse matrices
    (missing entries are zeros: sparsity patterns need not agree)."""
    D = (A - B).tocoo()
    nb = sp.linalg.norm(B) if B.nnz else 1.0
    mb = np.max(np.abs(B.data)) if B.nnz else 1.0
    dmax = np.max(np.abs(D.data)) if D.nnz else 0.0
    dfro = np.sqrt(np.sum(D.data ** 2)) if D.nnz else 0.0
    return dfro / nb, dmax / mb


WORKLOADS = {
    "beam144_grid32": (1, False),
    "beam1920_grid128": (2, True),
    "plate4320_grid256s_tilted": (3, True),
    "beam3600_grid192": (4, True),
    "three_bodies12k_grid512x256x256s": (5, True),
}


def workload(name):
    cfg, small = WORKLOADS[name]
    return wl.workload(cfg, small=small)


def sampled_rows_check(c, faces, X, tets, u_f, f_s, n_rows, seed, us=None, ff=None):
    """Sampled rows of B^d and columns of B^dT of a GPU coupling against the
    oracle, which integrates only the tets that touch them; with us (lumped
    velocity, (3, n_v)) and ff (force, 3 flat arrays) also the transferred
    values there.  Returns the largest relative Frobenius error of each
    kind."""
    import scipy.sparse as sp_
    bounds = oracle.tet_bounds(X, tets)
    rng = np.random.default_rng(seed)
    verts = np.sort(rng.choice(X.shape[0], n_rows, replace=False))
    star = oracle.vertex_star(tets, verts)
    R = oracle.assemble(faces, X, tets, subset=star)
    m = oracle.lumped_mass(X, tets[star], n_vert=X.shape[0])
    err = dict(rows=0.0, cols=0.0, velocity=0.0, force=0.0)
    for d in range(3):
        rp, col, val = c.export_csr(d)
        G = sp_.csr_matrix((val, col, rp), shape=(X.shape[0], oracle.n_fluid(faces, d)))
        Gs, Rs = G[verts], R.B[d][verts]
        err["rows"] = max(err["rows"], sp_.linalg.norm(Gs - Rs) / sp_.linalg.norm(Rs))
        if us is not None:
            want = (Rs @ np.asarray(u_f[d]).ravel()) / m[verts]
            err["velocity"] = max(err["velocity"], rel_fro(us[d][verts], want))
        cols = np.unique(Rs.indices)
        pick = np.sort(rng.choice(cols, min(16, cols.size), replace=False))
        nx, ny, _ = oracle.lattice_shape(faces, d)
        sub = np.unique(np.concatenate([
            oracle.tets_touching_node(faces, X, tets, d, (j % nx, (j // nx) % ny, j // (nx * ny)),
                                      bounds) for j in pick]))
        Rc = oracle.assemble(faces, X, tets, subset=sub).B[d].tocsc()[:, pick]
        Gc = G.tocsc()[:, pick]
        err["cols"] = max(err["cols"], sp_.linalg.norm(Gc - Rc) / sp_.linalg.norm(Rc))
        if ff is not None:
            err["force"] = max(err["force"], rel_fro(ff[d][pick], Rc.T @ f_s[d]))
    return err
