"""transfer_velocity_noalloc (the allocation-free velocity transfer) against
transfer_velocity through the C ABI: two calls in a row on two couplings,
the second smaller, in both precisions and with both masses; the results
are those of the allocating call (same kernels, same order), which match
the FP64 oracle to the transfer's tolerances; a coupling too large for the
library's per-GPU scratch is refused before any work."""
import numpy as np
import pytest

import oracle
import workloads as wl
from tests.gpu_common import fluid_fields, rel_fro, require_gpu, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_velocity_matches_allocating_call(dev, prec):
    import torch
    from paper_1810_13046_amd import Coupling
    tol = 1e-12 if prec == "fp64" else 1e-5
    # the larger input first, then a smaller one: the shared scratch keeps
    # the first call's contents
    for W in (wl.workload(3, small=True), wl.workload(1)):
        say(f"[gpu] noalloc {W.name} {prec}: {W.tets.shape[0]} tets")
        c = Coupling(W.faces, to_dev(W.X, torch.float64, dev), to_dev(W.tets, torch.int32, dev),
                     precision=prec, consistent=True)
        u_f = fluid_fields(W)
        ud = [to_dev(a, c.dtype, dev) for a in u_f]
        R = oracle.assemble(W.faces, W.X, W.tets)
        for mass in ("consistent", "lumped"):
            rtol = 1e-14 if prec == "fp64" else 1e-7
            want, iw = c.velocity(ud, mass=mass, rtol=rtol, maxit=500, with_info=True)
            out = torch.full_like(want, float("nan"))
            got, ig = c.velocity(ud, mass=mass, rtol=rtol, maxit=500, out=out, with_info=True,
                                 noalloc=True)
            torch.cuda.synchronize()
            assert got.data_ptr() == out.data_ptr()
            assert torch.equal(got, want), mass
            assert ig.iterations == iw.iterations and ig.rel_residual == iw.rel_residual
            ref = oracle.transfer_velocity(R, u_f, mass)
            e = rel_fro(got.cpu().numpy(), ref)
            say(f"  {mass}: identical to transfer_velocity; vs oracle {e:.2e}")
            assert e <= (tol if mass == "lumped" else max(tol, 5 * rtol))
        c.free()


def test_noalloc_refuses_a_coupling_beyond_its_scratch(dev):
    """2.5M solid vertices (most unused) with consistent mass need more than
    the 256 MiB the library holds per GPU: IBVT_E_CAPACITY, nothing
    written; the lumped transfer needs no scratch and runs."""
    import torch
    from paper_1810_13046_amd import Coupling, IbvtError
    faces = [np.linspace(0.0, 1.0, 9)] * 3
    n = 2_500_000
    X = np.full((n, 3), 0.5)
    X[:4] = [[0.4, 0.4, 0.4], [0.6, 0.41, 0.42], [0.45, 0.6, 0.43], [0.44, 0.45, 0.6]]
    T = np.array([[0, 1, 2, 3]], dtype=np.int32)
    c = Coupling(faces, to_dev(X, torch.float64, dev), to_dev(T, torch.int32, dev),
                 precision="fp32", consistent=True)
    u = [torch.ones(m, dtype=torch.float32, device=dev) for m in c.n_fluid]
    out = torch.full((3, n), 7.0, dtype=torch.float32, device=dev)
    say("[gpu] noalloc refusal beyond the scratch")
    with pytest.raises(IbvtError) as e:
        c.velocity(u, mass="consistent", out=out, noalloc=True)
    assert e.value.name == "IBVT_E_CAPACITY"
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
    got = c.velocity(u, mass="lumped", out=out, noalloc=True)
    assert abs(float(got[:, :4].mean()) - 1.0) <= 1e-6  # constants are reproduced
    c.free()
