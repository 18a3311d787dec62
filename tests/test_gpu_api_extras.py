"""Interface extras on the HIP path, through the C ABI: the per-body
counters (coupling_body_info), a caller-supplied device allocator
(ibvt_set_allocator, here PyTorch's caching allocator) and the release of
the assembly's scratch (coupling_release_scratch).

Per-body counters are checked against what the mesh fixes by itself
(each body's tet count, zero-volume tets and volume from the vertex
coordinates, in numpy) and against coupling_info's totals; the transfers of
a coupling whose buffers come from the caller's allocator against the FP64
oracle (1e-12 relative)."""
import gc

import numpy as np
import pytest

import oracle
from tests.gpu_common import fluid_fields, rel_fro, require_gpu, say, to_dev, workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


def tet_volumes(X, T):
    P = X[T]
    e = P[:, 1:, :] - P[:, :1, :]
    return np.abs(np.einsum("ij,ij->i", e[:, 0], np.cross(e[:, 1], e[:, 2]))) / 6.0


@pytest.mark.parametrize("store_B", [True, False])
def test_body_counters(dev, store_B):
    import torch
    from paper_1810_13046_amd import Coupling, IbvtError
    W = workload("three_bodies12k_grid512x256x256s")
    off = np.asarray(W.body_tet_offsets, dtype=np.int64)
    assert off.size >= 3 and off[0] == 0 and off[-1] == W.tets.shape[0]
    say(f"[gpu] body counters store_B={store_B}: {off.size - 1} bodies")
    c = Coupling(W.faces, to_dev(W.X, torch.float64, dev), to_dev(W.tets, torch.int32, dev),
                 precision="fp64", store_B=store_B)
    bodies = c.body_info(off)
    info = c.info()
    vol = tet_volumes(W.X, W.tets)
    for b, r in enumerate(bodies):
        v = vol[off[b]:off[b + 1]]
        assert r["tets"] == off[b + 1] - off[b]
        assert r["zero_tets"] == int(np.count_nonzero(v == 0.0))
        assert abs(r["volume"] - v.sum()) <= 1e-12 * v.sum()
        assert r["pairs"] > 0
        assert r["pieces"] == (-1 if not store_B else r["pieces"])
    assert sum(r["pairs"] for r in bodies) == info["pairs"]
    assert sum(r["zero_tets"] for r in bodies) == info["zero_tets"]
    if store_B:
        assert sum(r["pieces"] for r in bodies) == info["pieces"]
        assert all(0 < r["pieces"] <= r["pairs"] for r in bodies)
    # one body holding everything equals the totals; bad offsets are refused
    whole = c.body_info([0, W.tets.shape[0]])[0]
    assert whole["pairs"] == info["pairs"]
    for bad in ([1, W.tets.shape[0]], [0, W.tets.shape[0] - 1], [0, 10, 5, W.tets.shape[0]]):
        with pytest.raises(IbvtError):
            c.body_info(bad)
    c.free()


def test_caller_allocator(dev):
    import torch
    from paper_1810_13046_amd import Coupling, use_torch_allocator
    W = workload("plate4320_grid256s_tilted")
    R = oracle.assemble(W.faces, W.X, W.tets)
    X = to_dev(W.X, torch.float64, dev)
    T = to_dev(W.tets, torch.int32, dev)
    u_f = fluid_fields(W)
    ud = [to_dev(u, torch.float64, dev) for u in u_f]
    # tensors of earlier tests still waiting for the cycle collector would
    # otherwise be freed while this test counts torch's allocations
    gc.collect()
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated(dev)
    use_torch_allocator(True)
    try:
        say("[gpu] coupling on torch's caching allocator")
        c = Coupling(W.faces, X, T, precision="fp64", consistent=True)
        torch.cuda.synchronize()
        held = torch.cuda.memory_allocated(dev) - before
        nbytes = c.info()["device_bytes"]
        say(f"  device_bytes {nbytes}, torch allocated {held}")
        assert nbytes > 0 and held >= nbytes
        us = c.velocity(ud, mass="consistent", rtol=1e-14).cpu().numpy()
        assert rel_fro(us, oracle.transfer_velocity(R, u_f, "consistent")) <= 5e-12
        c.reassemble(X)
        us = c.velocity(ud, mass="lumped").cpu().numpy()
        assert rel_fro(us, oracle.transfer_velocity(R, u_f, "lumped")) <= 1e-12
        c.free()
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated(dev) == before
    finally:
        use_torch_allocator(False)
    # the default allocator again: torch's count does not move
    c = Coupling(W.faces, X, T, precision="fp64", consistent=True)
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated(dev) == before
    c.free()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_release_scratch_keeps_transfers_and_adjoints(dev, prec):
    """After coupling_release_scratch the coupling holds less device memory
    and gives bit-identical transfers and adjoints; a reassembly afterwards
    gives bit-identical matrices again."""
    import torch
    from paper_1810_13046_amd import Coupling
    W = workload("plate4320_grid256s_tilted")
    X = to_dev(W.X, torch.float64, dev)
    c = Coupling(W.faces, X, to_dev(W.tets, torch.int32, dev), precision=prec, consistent=True)
    dt = c.dtype
    ud = [to_dev(u, dt, dev) for u in fluid_fields(W)]
    f_s = to_dev(W.f_s(), dt, dev)

    def run():
        us = c.velocity(ud, mass="consistent", rtol=1e-12 if prec == "fp64" else 1e-7)
        ff = [torch.zeros_like(u) for u in ud]
        c.force(f_s, ff, alpha=0.5)
        g_uf = [torch.zeros_like(u) for u in ud]
        g_X = torch.zeros((W.X.shape[0], 3), dtype=torch.float64, device=dev)
        c.velocity_vjp(us - 1.0, u_f=ud, u_s=us, mass="consistent", g_uf=g_uf, g_X=g_X,
                       rtol=1e-12 if prec == "fp64" else 1e-7)
        torch.cuda.synchronize()
        return [us] + ff + g_uf + [g_X]

    before = run()
    csr = [c.export_csr(d) for d in range(3)]
    held = c.info()["device_bytes"]
    c.release_scratch()
    torch.cuda.synchronize()
    after_bytes = c.info()["device_bytes"]
    say(f"[gpu] release scratch {prec}: {held} -> {after_bytes} bytes")
    assert after_bytes < held
    for a, b in zip(before, run()):
        assert torch.equal(a, b)
    c.reassemble(X)
    for d in range(3):
        rp, col, val = c.export_csr(d)
        assert np.array_equal(rp, csr[d][0]) and np.array_equal(col, csr[d][1])
        assert np.array_equal(val, csr[d][2])
    for a, b in zip(before, run()):
        assert torch.equal(a, b)
    c.free()
