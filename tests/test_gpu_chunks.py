"""The chunked assembly on small meshes, through the C ABI: with
IBVT_CHUNK_ITEMS set so that the pairs are clipped, integrated and gathered
in 8 chunks (rows whose pairs lie in several chunks carry their partial
sums between chunks), B^d and B^dT, the transfers and the shape derivative
must equal those of the one-chunk assembly bit for bit (the same additions
in the same order), and B^d must match the FP64 oracle (1e-12 relative,
FP32-mixed 1e-5)."""
import os

import numpy as np
import pytest

import oracle
from tests.gpu_common import (fluid_fields, gpu_csr, require_gpu, say, sparse_rel, to_dev,
                              workload)

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


def split_rows(T, n_chunks):
    """(vertex, component) rows whose incident tets lie in more than one
    chunk of the (component, tet) items (every tet of these meshes lies
    inside the grid, so every tet has pairs)."""
    n_t = T.shape[0]
    n_tc = 3 * n_t
    at = np.array([n_tc * k // n_chunks for k in range(n_chunks + 1)])
    n = 0
    for d in range(3):
        ch = np.searchsorted(at, d * n_t + np.arange(n_t), side="right") - 1
        lo = np.full(T.max() + 1, 99)
        hi = np.full(T.max() + 1, -1)
        np.minimum.at(lo, T.ravel(), np.repeat(ch, 4))
        np.maximum.at(hi, T.ravel(), np.repeat(ch, 4))
        n += int(np.count_nonzero((hi >= 0) & (lo != hi)))
    return n


def run(c, W, dev, dt):
    import torch
    ud = [to_dev(u, dt, dev) for u in fluid_fields(W)]
    us = c.velocity(ud, mass="lumped")
    ff = [torch.zeros_like(u) for u in ud]
    c.force(to_dev(W.f_s(), dt, dev), ff, alpha=0.5)
    g_uf = [torch.zeros_like(u) for u in ud]
    g_fs = torch.zeros((3, W.X.shape[0]), dtype=dt, device=dev)
    g_X = torch.zeros((W.X.shape[0], 3), dtype=torch.float64, device=dev)
    c.vjp(us - 1.0, ud, u_f=ud, u_s=us, f_s=to_dev(W.f_s(), dt, dev), mass="lumped", alpha=0.5,
          g_uf=g_uf, g_fs=g_fs, g_X=g_X)
    torch.cuda.synchronize()
    return [us] + ff + g_uf + [g_fs, g_X]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["plate4320_grid256s_tilted", "three_bodies12k_grid512x256x256s"])
def test_eight_chunks_equal_one(dev, name, prec):
    import torch
    from paper_1810_13046_amd import Coupling
    W = workload(name)
    n_tc = 3 * W.tets.shape[0]
    assert split_rows(W.tets, 8) > 0
    X = to_dev(W.X, torch.float64, dev)
    T = to_dev(W.tets, torch.int32, dev)
    assert "IBVT_CHUNK_ITEMS" not in os.environ
    one = Coupling(W.faces, X, T, precision=prec)
    dt = one.dtype
    say(f"[gpu] {name} {prec}: one chunk, then 8 chunks of {n_tc // 8} items")
    os.environ["IBVT_CHUNK_ITEMS"] = str(n_tc // 8)
    try:
        eight = Coupling(W.faces, X, T, precision=prec)
        torch.cuda.synchronize()
        assert eight.info()["pairs"] == one.info()["pairs"]
        for d in range(3):
            for tr in (False, True):
                a, b = one.export_csr(d, transposed=tr), eight.export_csr(d, transposed=tr)
                for x, y in zip(a, b):
                    assert np.array_equal(x, y), (d, tr)
        for x, y in zip(run(one, W, dev, dt), run(eight, W, dev, dt)):
            assert torch.equal(x, y)
        # reassembly keeps the chunked matrices
        eight.reassemble(X)
        for d in range(3):
            assert all(np.array_equal(x, y) for x, y in zip(one.export_csr(d), eight.export_csr(d)))
    finally:
        del os.environ["IBVT_CHUNK_ITEMS"]
    R = oracle.assemble(W.faces, W.X, W.tets)
    for d in range(3):
        fro, mx = sparse_rel(gpu_csr(eight, d, oracle.n_fluid(W.faces, d)), R.B[d])
        say(f"  B^{d} rel fro {fro:.2e} max {mx:.2e}")
        assert fro <= TOL[prec] and (prec == "fp32" or mx <= TOL[prec]), (d, fro, mx)
    one.free()
    eight.free()
