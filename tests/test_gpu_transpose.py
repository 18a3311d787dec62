"""B^dT through the bucket transpose, through the C ABI.

Large operators are transposed through buckets of 32 consecutive lattice
nodes (per-bucket counting sort in LDS); small ones through a counting sort
over the whole lattice.  IBVT_BUCKET_NNZ=1 puts every operator through the
bucket path: B^dT (row pointers, vertices, values, row map) must equal the
counting path's bit for bit and the exact transpose of the exported B^d,
and the force transfer must give the same bits.  A fine solid in a 4^3 grid
makes buckets beyond the LDS capacity (4096 records) and rows longer than
it, which take the bucket kernel's grouped, chunked ranking."""
import os

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as wl
from tests.gpu_common import require_gpu, say, to_dev, workload

pytestmark = pytest.mark.gpu

SORT_CAP = 4096
BUCKET_NODES = 32


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


def dense_case():
    """A 32^3-hexahedron box (196,608 tets, 35,937 vertices) in a 4^3 grid,
    inside the hull [0.125, 0.875] of the cell-midpoint lattice nodes."""
    rng = np.random.default_rng(11)
    b = wl.box_body("dense", (0.7, 0.7, 0.7), (0.5, 0.5, 0.5), (32, 32, 32), 0.2, rng)
    faces = [wl.uniform_faces(4) for _ in range(3)]
    return faces, b.X, b.tets


def both_paths(faces, X, T, prec, dev):
    import torch
    from paper_1810_13046_amd import Coupling
    Xd = to_dev(X, torch.float64, dev)
    Td = to_dev(T, torch.int32, dev)
    assert "IBVT_BUCKET_NNZ" not in os.environ
    counting = Coupling(faces, Xd, Td, precision=prec)
    os.environ["IBVT_BUCKET_NNZ"] = "1"
    try:
        buckets = Coupling(faces, Xd, Td, precision=prec)
        torch.cuda.synchronize()
    finally:
        del os.environ["IBVT_BUCKET_NNZ"]
    return counting, buckets


def check_equal(counting, buckets, n_vert, dev, seed):
    import torch
    stats = []
    for d in range(3):
        a = counting.export_csr(d, transposed=True)
        b = buckets.export_csr(d, transposed=True)
        for x, y, what in zip(a, b, ("rowptr", "col", "val", "rowmap")):
            assert np.array_equal(x, y), (d, what)
        rp, col, val, rm = b
        # exact transpose of the exported B^d, restricted to its nonzero columns
        brp, bcol, bval = buckets.export_csr(d)
        Bd = sp.csr_matrix((bval, bcol, brp), shape=(n_vert, buckets.n_fluid[d]))
        BT = Bd.T.tocsr()
        touched = np.flatnonzero(np.diff(BT.indptr))
        assert np.array_equal(rm, touched), d
        BTs = BT[touched]
        BTs.sort_indices()
        assert np.array_equal(rp, BTs.indptr) and np.array_equal(col, BTs.indices), d
        assert np.array_equal(val, BTs.data), d
        lens = np.diff(rp)
        per_bucket = np.bincount(rm // BUCKET_NODES, weights=lens)
        stats.append((int(lens.max()), int(per_bucket.max())))
    rng = np.random.default_rng(seed)
    f_s = rng.standard_normal((3, n_vert))
    out = []
    for c in (counting, buckets):
        dt = c.dtype
        ff = [torch.zeros(n, dtype=dt, device=dev) for n in c.n_fluid]
        c.force(to_dev(f_s, dt, dev), ff, alpha=0.75)
        torch.cuda.synchronize()
        out.append(ff)
    for x, y in zip(*out):
        assert torch.equal(x, y)
    return stats


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["beam1920_grid128", "plate4320_grid256s_tilted",
                                  "three_bodies12k_grid512x256x256s"])
def test_bucket_transpose_equals_counting_sort(dev, name, prec):
    W = workload(name)
    say(f"[gpu] transpose paths {name} {prec}")
    counting, buckets = both_paths(W.faces, W.X, W.tets, prec, dev)
    check_equal(counting, buckets, W.X.shape[0], dev, 5)
    counting.free()
    buckets.free()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_bucket_transpose_beyond_lds(dev, prec):
    faces, X, T = dense_case()
    say(f"[gpu] transpose paths, dense buckets {prec} n_tet={T.shape[0]}")
    counting, buckets = both_paths(faces, X, T, prec, dev)
    stats = check_equal(counting, buckets, X.shape[0], dev, 6)
    say(f"  (longest row, largest bucket) per component: {stats}")
    # the fixture reaches both cases of the kernel's large-bucket branch
    assert max(s[1] for s in stats) > SORT_CAP
    assert max(s[0] for s in stats) > SORT_CAP
    counting.free()
    buckets.free()
