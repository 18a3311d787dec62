"""Picard coupling (Section 3, Steps 1-6) through the C driver fsi_step,
against the oracle's loop with the same linear stub solvers, and the fluid
lattice's lumped volume.  FP64: same iteration count (within one), fields
within 1e-10 relative; FP32-mixed: fields within 1e-4 of the FP64 oracle;
with stored matrices and without (IBVT_NO_STORE_B)."""
import numpy as np
import pytest

import oracle
from tests.gpu_common import rel_fro, require_gpu, say, to_dev, workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


def test_fluid_lumped_volume_matches_oracle(dev):
    from paper_1810_13046_amd import fluid_lumped_volume
    W = workload("plate4320_grid256s_tilted")
    for d in range(3):
        got = fluid_lumped_volume(W.faces, d, device=dev).cpu().numpy()
        want = oracle.fluid_lumped_volume(W.faces, d)
        assert got.shape == want.shape
        assert np.max(np.abs(got - want)) <= 1e-15 * want.max()


def _stubs(W, seed, density):
    rng = np.random.default_rng(seed)
    n = W.X.shape[0]
    u_rest = 1e-3 * rng.standard_normal((3, n))
    v_base = [rng.standard_normal(oracle.n_fluid(W.faces, d)) for d in range(3)]
    beta = 0.5
    if density:  # force densities are loads over node volumes ~ h^3: keep the map contractive
        beta *= min(oracle.fluid_lumped_volume(W.faces, d).min() for d in range(3))
    return u_rest, 10.0, v_base, beta


@pytest.mark.parametrize("store_B", [True, False])
@pytest.mark.parametrize("density", [False, True])
@pytest.mark.parametrize("mode", ["lumped", "consistent", "dual"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fsi_step_matches_oracle(dev, prec, mode, density, store_B):
    import torch
    from paper_1810_13046_amd import Coupling
    name = "beam144_grid32" if prec == "fp32" else "plate4320_grid256s_tilted"
    W = workload(name)
    n = W.X.shape[0]
    dual = mode == "dual"
    mass = "consistent" if mode == "consistent" else "lumped"
    u_rest, k_s, v_base, beta = _stubs(W, 17, density)
    rng = np.random.default_rng(4)
    u0 = 1e-3 * rng.standard_normal((3, n))
    dt, alpha = 0.05, 0.8
    eps_abs = 1e-13 if prec == "fp64" else 0.0
    # FP32: the transferred velocity's rounding (about 1e-7 of |w|, times dt k)
    # sets a floor near 5e-6 on the force residual relative to the force
    eps_rel = 0.0 if prec == "fp64" else 1e-4
    say(f"[gpu] fsi_step {name} {prec} {mode} density={density} store_B={store_B}")
    ref = oracle.fsi_step(W.faces, W.X, W.tets, u0, [np.zeros_like(v) for v in v_base],
                          lambda u: -k_s * (u - u_rest),
                          lambda ft: [v_base[d] + beta * ft[d] for d in range(3)],
                          dt, alpha, eps_abs=1e-13, eps_rel=0.0, max_iter=200, mass=mass,
                          force_density=density, dual=dual)
    assert ref["converged"]
    c = Coupling(W.faces, to_dev(W.X, torch.float64, dev), to_dev(W.tets, torch.int32, dev),
                 precision=prec, consistent=(mass == "consistent"), dual=dual, store_B=store_B)
    dt_ = c.dtype
    ur = to_dev(u_rest, dt_, dev)
    vb = [to_dev(v.reshape(tuple(reversed(oracle.lattice_shape(W.faces, d)))), dt_, dev)
          for d, v in enumerate(v_base)]
    vf = [torch.zeros_like(v) for v in vb]

    def solid(u_hat, f_fsi):
        torch.mul(u_hat - ur, -k_s, out=f_fsi)

    def fluid(f_tilde, v):
        for d in range(3):
            torch.add(vb[d], f_tilde[d], alpha=beta, out=v[d])

    rep, out = c.fsi_step(to_dev(W.X, torch.float64, dev), to_dev(u0, dt_, dev), vf, solid, fluid,
                          dt=dt, alpha=alpha, eps_abs=eps_abs, eps_rel=eps_rel, max_iter=200,
                          mass=mass, force_density=density, cg_rtol=1e-14 if prec == "fp64" else 1e-7)
    say(f"  iterations gpu {rep.iterations} oracle {ref['iterations']} res {rep.res_abs:.2e}")
    assert rep.converged
    tol = 1e-10 if prec == "fp64" else 1e-4
    if prec == "fp64":
        assert abs(rep.iterations - ref["iterations"]) <= 1
    assert rel_fro(out["f_fsi"].cpu().numpy(), ref["f_fsi"]) <= tol
    assert rel_fro(out["u_hat"].cpu().numpy(), ref["u_hat"]) <= tol
    assert rel_fro(out["w_s"].cpu().numpy(), ref["w_s"]) <= tol
    for d in range(3):
        assert rel_fro(out["f_tilde"][d].cpu().numpy().ravel(), ref["f_tilde"][d]) <= tol, d
        assert rel_fro(vf[d].cpu().numpy().ravel(), ref["v_f"][d]) <= tol, d
    c.free()


def test_fsi_step_errors(dev):
    import torch
    from paper_1810_13046_amd import Coupling
    from paper_1810_13046_amd.ibvt import IbvtError
    W = workload("beam144_grid32")
    n = W.X.shape[0]
    c = Coupling(W.faces, to_dev(W.X, torch.float64, dev), to_dev(W.tets, torch.int32, dev),
                 precision="fp64", consistent=False)
    vf = [torch.zeros(tuple(reversed(oracle.lattice_shape(W.faces, d))), dtype=torch.float64,
                      device=dev) for d in range(3)]
    X = to_dev(W.X, torch.float64, dev)
    u0 = torch.zeros((3, n), dtype=torch.float64, device=dev)

    def solid(u, f):
        f.copy_(-u)

    def fluid(ft, v):
        for d in range(3):
            v[d].add_(ft[d], alpha=0.5)

    # not converged within two iterations: status, report and fields of the last iteration
    rep, out = c.fsi_step(X, u0 + 1e-3, vf, solid, fluid, dt=0.1, eps_abs=1e-30, eps_rel=0.0,
                          max_iter=2, raise_not_converged=False)
    assert rep.iterations == 2 and not rep.converged
    with pytest.raises(IbvtError):
        c.fsi_step(X, u0 + 1e-3, vf, solid, fluid, dt=0.1, eps_abs=1e-30, eps_rel=0.0, max_iter=2)
    # consistent mass not built
    with pytest.raises(IbvtError):
        c.fsi_step(X, u0, vf, solid, fluid, dt=0.1, mass="consistent")

    # a failing callback stops the step and its exception is raised
    def bad(u, f):
        raise RuntimeError("solid solver failed")

    with pytest.raises(RuntimeError, match="solid solver failed"):
        c.fsi_step(X, u0, vf, bad, fluid, dt=0.1)
    c.free()
