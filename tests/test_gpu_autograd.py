"""autograd forms: hand-written backward against the oracle's adjoint and
against central finite differences of the GPU forward (FP64)."""
import numpy as np
import pytest

import oracle
import workloads as wl
from tests.gpu_common import fluid_fields, rel_fro, require_gpu, say, to_dev, workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


@pytest.fixture(scope="module")
def plate():
    W = workload("plate4320_grid256s_tilted")
    return W, oracle.assemble(W.faces, W.X, W.tets)


@pytest.mark.parametrize("recompute", [False, True])
@pytest.mark.parametrize("mass", ["lumped", "consistent"])
def test_velocity_autograd_matches_oracle(dev, plate, mass, recompute):
    import torch
    from paper_1810_13046_amd.autograd import transfer_velocity
    W, R = plate
    u_f = fluid_fields(W)
    u = [to_dev(a, torch.float64, dev).requires_grad_(True) for a in u_f]
    X = to_dev(W.X, torch.float64, dev).requires_grad_(True)
    T = to_dev(W.tets, torch.int32, dev)
    u_t = W.u_target()
    say(f"[gpu] autograd velocity {mass} recompute={recompute}")
    us = transfer_velocity(u, X, W.faces, T, "fp64", mass, 1e-14, 500, None, recompute)
    L = 0.5 * ((us - to_dev(u_t, torch.float64, dev)) ** 2).sum()
    L.backward()
    g_us = us.detach().cpu().numpy() - u_t
    ref_uf, ref_X = oracle.velocity_vjp(R, u_f, g_us, mass)
    for d in range(3):
        assert rel_fro(u[d].grad.cpu().numpy().ravel(), ref_uf[d]) <= 1e-10
    e = rel_fro(X.grad.cpu().numpy(), ref_X)
    say(f"  g_X rel {e:.2e}")
    assert e <= 1e-10


def test_velocity_gradient_central_fd(dev):
    """dL/dX along seeded directions vs central differences of the GPU
    forward pass (h = 1e-6), lumped and consistent."""
    import torch
    from paper_1810_13046_amd.autograd import transfer_velocity
    W = workload("plate4320_grid256s_tilted")
    u_f = fluid_fields(W)
    u = [to_dev(a, torch.float64, dev) for a in u_f]
    T = to_dev(W.tets, torch.int32, dev)
    u_t = to_dev(W.u_target(), torch.float64, dev)
    dirs = wl.fd_directions(W.X.shape[0], 16, 5003)
    h = 1e-6
    for mass in ("lumped", "consistent"):
        X = to_dev(W.X, torch.float64, dev).requires_grad_(True)
        us = transfer_velocity(u, X, W.faces, T, "fp64", mass, 1e-14, 500)
        L = 0.5 * ((us - u_t) ** 2).sum()
        (gX,) = torch.autograd.grad(L, X)
        gX = gX.cpu().numpy()

        def loss(Xn):
            with torch.no_grad():
                v = transfer_velocity(u, to_dev(Xn, torch.float64, dev), W.faces, T, "fp64",
                                      mass, 1e-14, 500)
                return 0.5 * float(((v - u_t) ** 2).sum())

        worst = 0.0
        for D in dirs:
            fd = (loss(W.X + h * D) - loss(W.X - h * D)) / (2 * h)
            an = float(np.sum(gX * D))
            worst = max(worst, abs(fd - an) / max(1e-3, abs(an)))
        say(f"[gpu] FD {mass}: worst rel {worst:.2e}")
        assert worst <= 1e-5


def test_force_autograd_matches_oracle(dev, plate):
    import torch
    from paper_1810_13046_amd.autograd import transfer_force
    W, R = plate
    f_s = W.f_s()
    fs = to_dev(f_s, torch.float64, dev).requires_grad_(True)
    X = to_dev(W.X, torch.float64, dev).requires_grad_(True)
    T = to_dev(W.tets, torch.int32, dev)
    gff = fluid_fields(W)
    say("[gpu] autograd force")
    ff = transfer_force(fs, X, W.faces, T, "fp64", 0.8)
    L = sum((ff[d] * to_dev(gff[d], torch.float64, dev)).sum() for d in range(3))
    L.backward()
    rfs, rX = oracle.force_vjp(R, f_s, [g.ravel() for g in gff], 0.8)
    assert rel_fro(fs.grad.cpu().numpy(), rfs) <= 1e-12
    assert rel_fro(X.grad.cpu().numpy(), rX) <= 1e-10


def test_time_series_reassembly_and_recompute_backward(dev):
    """A bending beam over 32 steps: B rebuilt every step in place
    (reassemble_coupling); the last step's B matches the oracle; the loss
    over the last 8 steps is differentiated with recompute-B and compared
    with the oracle's adjoint summed over the same steps."""
    import torch
    from paper_1810_13046_amd import Coupling
    from paper_1810_13046_amd.autograd import transfer_velocity
    from tests.gpu_common import gpu_csr, sparse_rel
    W = wl.workload(4, small=True)
    T = to_dev(W.tets, torch.int32, dev)
    u_f = fluid_fields(W)
    u = [to_dev(a, torch.float64, dev) for a in u_f]
    c = Coupling(W.faces, to_dev(W.X, torch.float64, dev), T, precision="fp64")
    for n in range(32):
        Xn = W.X + wl.bending_displacement(W.X, n, 6000 + W.cfg, x0=W.X[:, 0].min(),
                                           length=np.ptp(W.X[:, 0]), amplitude=0.01)
        c.reassemble(to_dev(Xn, torch.float64, dev))
    say("[gpu] series: last step vs oracle")
    R = oracle.assemble(W.faces, Xn, W.tets)
    for d in range(3):
        fro, mx = sparse_rel(gpu_csr(c, d, oracle.n_fluid(W.faces, d)), R.B[d])
        assert fro <= 1e-12 and mx <= 1e-12
    assert c.info()["assemblies"] == 33
    c.free()
    # recompute-B backward over the last 8 steps
    ut = wl.gaussian_nodal(W.X.shape[0], 4000 + W.cfg)
    uu = [a.clone().requires_grad_(True) for a in u]
    X0 = to_dev(W.X, torch.float64, dev).requires_grad_(True)
    L = 0.0
    ref_uf = [np.zeros(a.size) for a in u_f]
    ref_X = np.zeros_like(W.X)
    for n in range(24, 32):
        disp = wl.bending_displacement(W.X, n, 6000 + W.cfg, x0=W.X[:, 0].min(),
                                       length=np.ptp(W.X[:, 0]), amplitude=0.01)
        Xn = X0 + to_dev(disp, torch.float64, dev)
        us = transfer_velocity(uu, Xn, W.faces, T, "fp64", "lumped", 1e-12, 500, None, True)
        L = L + 0.5 * ((us - to_dev(ut, torch.float64, dev)) ** 2).sum()
        Rn = oracle.assemble(W.faces, W.X + disp, W.tets)
        usn = oracle.transfer_velocity(Rn, u_f, "lumped")
        guf, gX = oracle.velocity_vjp(Rn, u_f, usn - ut, "lumped")
        for d in range(3):
            ref_uf[d] += guf[d]
        ref_X += gX
    L.backward()
    for d in range(3):
        assert rel_fro(uu[d].grad.cpu().numpy().ravel(), ref_uf[d]) <= 1e-10
    assert rel_fro(X0.grad.cpu().numpy(), ref_X) <= 1e-10


def test_unstructured_coupling_autograd_matches_oracle(dev):
    """An unstructured coupling passed to the autograd forms: the gradients
    of L = 1/2 ||u_s − u_t||^2 + <g, f_f> with respect to the fluid nodal
    fields, the solid forces and the solid vertices, against the oracle's
    two adjoints."""
    import torch
    from oracle import unstructured as un
    from paper_1810_13046_amd import Coupling
    from paper_1810_13046_amd.autograd import transfer_force, transfer_velocity
    un.build(force=False)
    W = wl.unstructured.workload_u(1)
    R = un.assemble(W.Xf, W.tets_f, W.X, W.tets)
    X = to_dev(W.X, torch.float64, dev).requires_grad_(True)
    T = to_dev(W.tets, torch.int32, dev)
    c = Coupling(None, X.detach(), T, fluid_mesh=(to_dev(W.Xf, torch.float64, dev),
                                                  to_dev(W.tets_f, torch.int32, dev)))
    u_f = W.u_f()
    u = [to_dev(a, torch.float64, dev).requires_grad_(True) for a in u_f]
    f_s_np = W.f_s()
    f_s = to_dev(f_s_np, torch.float64, dev).requires_grad_(True)
    g_np = np.random.default_rng(17).standard_normal((3, W.Xf.shape[0]))
    u_t = np.random.default_rng(18).standard_normal((3, W.X.shape[0]))
    say("[gpu] autograd with an unstructured coupling")
    us = transfer_velocity(u, X, None, T, "fp64", "consistent", 1e-14, 500, c)
    ff = transfer_force(f_s, X, None, T, "fp64", 0.6, c)
    L = 0.5 * ((us - to_dev(u_t, torch.float64, dev)) ** 2).sum() + sum(
        (ff[d] * to_dev(g_np[d], torch.float64, dev)).sum() for d in range(3))
    L.backward()
    g_us = us.detach().cpu().numpy() - u_t
    ref_uf, ref_Xv = un.velocity_vjp(R, u_f, g_us, "consistent")
    ref_fs, ref_Xf = un.force_vjp(R, f_s_np, g_np, 0.6)
    e = rel_fro(X.grad.cpu().numpy(), ref_Xv + ref_Xf)
    say(f"  g_X rel {e:.2e}")
    assert e <= 1e-10
    for d in range(3):
        assert rel_fro(u[d].grad.cpu().numpy(), ref_uf[d] + 0.0) <= 1e-10
    assert rel_fro(f_s.grad.cpu().numpy(), ref_fs) <= 1e-12
    c.free()
