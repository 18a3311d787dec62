"""Pins of the FP64 oracle of the coupling with an unstructured (P1
tetrahedral) fluid background (no GPU): closed forms, an independent Gauss
rule, tilings, the symmetry of exchanging the two meshes, exact
reproduction of affine fields, partition of unity, Monte Carlo brute force,
and central finite differences of the reverse mode's shape derivative."""
import numpy as np
import pytest

import workloads as wl
from tests.refquad import ref_simplex_monomial, tet_integral

WU = wl.unstructured
REF = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=np.float64)


@pytest.fixture(scope="module")
def un(oracle_mod):
    from oracle import unstructured
    unstructured.build(force=False)
    return unstructured


@pytest.fixture(scope="module")
def w1(un):
    W = WU.workload_u(1)
    return W, un.assemble(W.Xf, W.tets_f, W.X, W.tets)


def test_int2_reference_simplex_monomials(un):
    coord = [REF[:, 0], REF[:, 1], REF[:, 2]]
    one = np.ones(4)
    for a in range(3):
        for b in range(3):
            f = coord[a] if a < 3 else one
            g = coord[b]
            al = [0, 0, 0]
            al[a] += 1
            al[b] += 1
            want = float(ref_simplex_monomial(*al))
            assert un.int2(REF, f, g) == pytest.approx(want, rel=1e-14)
    assert un.int2(REF, one, one) == pytest.approx(1 / 6, rel=1e-15)


def test_int2_matches_gauss_rule(un):
    rng = np.random.default_rng(3)
    for _ in range(20):
        Y = rng.uniform(-1, 2, size=(4, 3))
        c = rng.standard_normal((2, 4))
        f, g = (c[m, 0] + Y @ c[m, 1:] for m in range(2))
        want = tet_integral(Y, lambda p: (c[0, 0] + p @ c[0, 1:]) * (c[1, 0] + p @ c[1, 1:]))
        assert un.int2(Y, f, g) == pytest.approx(want, rel=1e-12, abs=1e-14)


def test_clip_volume_closed_forms(un):
    assert un.clip_volume(REF, REF) == pytest.approx(1 / 6, rel=1e-14)
    assert un.clip_volume(REF, REF + 2.0) == 0.0
    # a scaled copy inside
    inner = 0.1 + 0.5 * REF   # largest coordinate sum 0.8: inside the simplex
    assert un.clip_volume(inner, REF) == pytest.approx(0.125 / 6, rel=1e-14)
    assert un.clip_volume(REF, inner) == pytest.approx(0.125 / 6, rel=1e-14)
    # the simplex and its translate along x: {x >= a} ∩ S, volume (1 - a)^3/6
    for a in (0.1, 0.35, 0.7):
        assert un.clip_volume(REF, REF + [a, 0, 0]) == pytest.approx((1 - a) ** 3 / 6, rel=1e-13)
    # sharing a face only
    mirror = REF * [-1, 1, 1]
    assert un.clip_volume(REF, mirror) == pytest.approx(0.0, abs=1e-16)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_clip_pieces_tile_the_tet(un, seed):
    """A tet inside a tetrahedral mesh of a box: the pieces over all the
    mesh's tets add up to its volume."""
    rng = np.random.default_rng(seed)
    box = WU.warped_box("b", 3, 0.2, 0.5, rng)
    T = rng.uniform(0.1, 0.9, size=(4, 3))
    vol = abs(np.linalg.det(T[1:] - T[0])) / 6
    tot = sum(un.clip_volume(T, box.X[t]) for t in box.tets)
    assert tot == pytest.approx(vol, rel=1e-12)


def test_row_sums_are_lumped_mass_and_total_volume(un, w1):
    """Σ_j μ_j = 1 inside the fluid mesh: row sums = ∫ λ_i; total = exact
    beam volume."""
    W, R = w1
    m = un.lumped_mass(W.X, W.tets)
    np.testing.assert_allclose(np.asarray(R.B.sum(axis=1)).ravel(), m, rtol=1e-12)
    assert R.B.sum() == pytest.approx(0.4 * 0.1 * 0.1, rel=1e-13)


def test_exchange_symmetry(un):
    """B with the roles of the two meshes exchanged is the transpose."""
    rng = np.random.default_rng(8)
    A = WU.warped_box("a", 3, 0.2, 0.4, rng)
    C = WU.warped_box("c", 4, 0.2, 0.4, rng)
    R1 = un.assemble(A.X, A.tets, C.X, C.tets)
    R2 = un.assemble(C.X, C.tets, A.X, A.tets)
    D = (R1.B - R2.B.T).tocoo()
    assert (np.abs(D.data).max() if D.nnz else 0.0) <= 1e-13 * np.abs(R1.B.data).max()
    # column sums when the solid fills the fluid mesh's box: ∫ μ_j, the
    # fluid mesh's lumped mass
    mf = un.lumped_mass(C.X, C.tets)
    np.testing.assert_allclose(np.asarray(R2.B.sum(axis=0)).ravel(), mf, rtol=1e-12)


def test_affine_reproduction(un, w1):
    """P1 fluid fields reproduce affine functions and ∫ λ_i u = Σ_l M_il u_l:
    the consistent transfer returns u at the solid vertices."""
    W, R = w1
    co = (0.4, -1.1, 0.7, 2.3)
    u = WU.linear_fields(W.Xf, co)
    us = un.transfer_velocity(R, [u, 2 * u, -u], "consistent")
    want = WU.linear_fields(W.X, co)
    np.testing.assert_allclose(us[0], want, atol=1e-12)
    np.testing.assert_allclose(us[1], 2 * want, atol=1e-12)


def test_monte_carlo_entries(un):
    """Entries of B for one solid tet against a small fluid mesh, by Monte
    Carlo with a 5-sigma bound."""
    rng = np.random.default_rng(21)
    F = WU.warped_box("f", 2, 0.2, 0.3, rng)
    S = np.array([[0.15, 0.2, 0.25], [0.8, 0.3, 0.2], [0.3, 0.85, 0.35], [0.35, 0.3, 0.9]])
    R = un.assemble(F.X, F.tets, S, np.array([[0, 1, 2, 3]], dtype=np.int32))
    B = R.B.toarray()
    n = 400000
    w = rng.dirichlet(np.ones(4), size=n)
    pts = w @ S
    vol = abs(np.linalg.det(S[1:] - S[0])) / 6
    # fluid hats at the points: locate the containing fluid tet
    acc = np.zeros((4, F.X.shape[0]))
    sq = np.zeros((4, F.X.shape[0]))
    found = np.zeros(n, dtype=bool)
    for t in F.tets:
        A = np.ones((4, 4))
        A[:, 1:] = F.X[t]
        coef = np.linalg.inv(A)
        mu = np.column_stack([np.ones(n), pts]) @ coef
        inside = np.all(mu >= -1e-14, axis=1) & ~found
        found |= inside
        for j in range(4):
            contrib = w[inside] * mu[inside, j][:, None]
            acc[:, t[j]] += contrib.sum(axis=0)
            sq[:, t[j]] += (contrib ** 2).sum(axis=0)
    assert found.all()
    est = vol * acc / n
    sd = vol * np.sqrt(np.maximum(sq / n - (acc / n) ** 2, 0) / n)
    big = B > 1e-4          # entries the samples resolve: a 5-sigma bound
    assert big.sum() > 20
    assert np.all(np.abs(est - B)[big] <= 5 * sd[big])
    # entries of tiny pieces (few or no samples): an absolute bound
    assert np.all(np.abs(est - B)[~big] <= 3e-5)


def test_dual_row_sums_and_reproduction(un, w1):
    W, _ = w1
    R = un.assemble(W.Xf, W.tets_f, W.X, W.tets, dual=True)
    m = un.lumped_mass(W.X, W.tets)
    np.testing.assert_allclose(np.asarray(R.B.sum(axis=1)).ravel(), m, rtol=1e-12)
    co = (-0.3, 0.9, 1.4, -0.6)
    us = un.transfer_velocity(R, [WU.linear_fields(W.Xf, co)], "lumped")
    np.testing.assert_allclose(us[0], WU.linear_fields(W.X, co), atol=1e-11)


def _fd(f, X, D, h=1e-6):
    return (f(X + h * D) - f(X - h * D)) / (2 * h)


@pytest.mark.parametrize("mass,dual", [("lumped", False), ("consistent", False), ("lumped", True)])
def test_velocity_shape_derivative_matches_finite_differences(un, w1, mass, dual):
    """g_X of L = 1/2 ||S^{-1} B(X) u_f − u_t||^2 against central differences
    of the assembled transfer along random directions."""
    W, _ = w1
    R = un.assemble(W.Xf, W.tets_f, W.X, W.tets, dual=dual)
    u_f = W.u_f()
    u_t = np.random.default_rng(41).standard_normal((3, W.X.shape[0]))
    r = un.transfer_velocity(R, u_f, mass) - u_t
    _, gX = un.velocity_vjp(R, u_f, r, mass)
    rng = np.random.default_rng(42)
    for _ in range(3):
        D = rng.standard_normal(W.X.shape)
        fd = _fd(lambda Y: un.velocity_loss(W.Xf, W.tets_f, Y, W.tets, u_f, u_t, mass, dual), W.X, D)
        an = float(np.sum(gX * D))
        assert abs(an - fd) <= 1e-6 * abs(fd) + 1e-10, (an, fd)


def test_force_shape_derivative_matches_finite_differences(un, w1):
    """g_X of φ = α Σ_d f_s,d^T B(X) g_ff,d against central differences."""
    W, R = w1
    f_s = W.f_s()
    g_ff = np.random.default_rng(43).standard_normal((3, W.Xf.shape[0]))
    alpha = 0.7
    _, gX = un.force_vjp(R, f_s, g_ff, alpha)

    def phi(Y):
        C = un.assemble(W.Xf, W.tets_f, Y, W.tets)
        return alpha * float(sum(f_s[d] @ (C.B @ g_ff[d]) for d in range(3)))

    rng = np.random.default_rng(44)
    for _ in range(3):
        D = rng.standard_normal(W.X.shape)
        fd = _fd(phi, W.X, D)
        an = float(np.sum(gX * D))
        assert abs(an - fd) <= 1e-6 * abs(fd) + 1e-10, (an, fd)


def test_shape_derivative_of_rigid_translation_is_zero_for_affine_fields(un, w1):
    """Translating the solid inside the fluid mesh leaves ∫ λ_i U unchanged
    when U is affine (the P1 fluid interpolant reproduces it exactly and
    the integral only sees U on the solid), so the velocity-force pairing's
    derivative along a uniform translation vanishes."""
    W, R = w1
    co = (0.2, -0.5, 0.8, 1.1)
    U = WU.linear_fields(W.Xf, co)
    f_s = W.f_s()
    _, gX = un.force_vjp(R, f_s, [U, U, U], 1.0)
    # d/dε Σ_i f_i ∫ λ_i U(x + ε e_k) = Σ_i f_i ∫ λ_i ∂_k U = ∂_k U Σ_i f_i m_i
    m = un.lumped_mass(W.X, W.tets)
    for k in range(3):
        want = co[1 + k] * float(sum(f_s[d] @ m for d in range(3)))
        assert abs(gX[:, k].sum() - want) <= 1e-10 * (1 + abs(want))


@pytest.mark.parametrize("mode,density", [("lumped", False), ("consistent", False),
                                          ("dual", False), ("lumped", True)])
def test_fsi_picard_reaches_the_fixed_point(un, w1, mode, density):
    """With a linear spring for the solid and a fluid whose nodal velocity
    responds linearly to the force, the fixed point of Steps 1-5 solves
    (I + k dt beta alpha T D⁻¹ Tᵀ) f = −k (û0 − û_rest + dt T v_base) per
    component, T = S⁻¹B and D the fluid nodes' lumped volumes ∫ μ_j (the
    identity without the density option): the Picard loop must land on the
    direct solution of that dense system."""
    from oracle import consistent_mass, lumped_mass
    W, _ = w1
    n = W.X.shape[0]
    nf = W.Xf.shape[0]
    dual = mode == "dual"
    mass = "consistent" if mode == "consistent" else "lumped"
    rng = np.random.default_rng(21)
    u_rest = 1e-3 * rng.standard_normal((3, n))
    v_base = [rng.standard_normal(nf) for _ in range(3)]
    k_s, beta = 10.0, 0.5
    if density:
        beta *= lumped_mass(W.Xf, W.tets_f).min()

    def solid(u_hat):
        return -k_s * (u_hat - u_rest)

    def fluid(f_tilde):
        return [v_base[d] + beta * f_tilde[d] for d in range(3)]

    u0 = 1e-3 * np.random.default_rng(5).standard_normal((3, n))
    dt, alpha = 0.05, 0.8
    r = un.fsi_step(W.Xf, W.tets_f, W.X, W.tets, u0, [np.zeros(nf)] * 3, solid, fluid, dt, alpha,
                    eps_abs=1e-14, eps_rel=0.0, max_iter=200, mass=mass, force_density=density,
                    dual=dual)
    assert r["converged"]
    c = un.assemble(W.Xf, W.tets_f, W.X + u0.T, W.tets, dual=dual)
    Sm = (np.diag(lumped_mass(c.X, W.tets)) if mass == "lumped"
          else consistent_mass(c.X, W.tets).toarray())
    T = np.linalg.solve(Sm, c.B.toarray())
    Dinv = 1.0 / lumped_mass(W.Xf, W.tets_f) if density else np.ones(nf)
    A = np.eye(n) + k_s * dt * beta * alpha * (T * Dinv[None, :]) @ T.T
    for d in range(3):
        rhs = -k_s * (u0[d] - u_rest[d] + dt * T @ v_base[d])
        f_star = np.linalg.solve(A, rhs)
        assert np.max(np.abs(r["f_fsi"][d] - f_star)) <= 1e-11 * max(1.0, np.max(np.abs(f_star)))


def test_fsi_density_of_an_orphan_fluid_vertex_is_zero(un, w1):
    """A fluid vertex that no fluid tet uses has no lumped volume and
    receives no load; with the force-density option its density is zero
    (not 0/0), and every other node is what it is without that vertex."""
    W, _ = w1
    n, nf = W.X.shape[0], W.Xf.shape[0]
    Xf2 = np.vstack([W.Xf, W.Xf[:1] + 0.01])
    rng = np.random.default_rng(8)
    u0 = 1e-3 * rng.standard_normal((3, n))
    v0 = [rng.standard_normal(nf) for _ in range(3)]

    def run(Xf, extra):
        v = [np.concatenate([a, np.zeros(extra)]) for a in v0]
        return un.fsi_step(Xf, W.tets_f, W.X, W.tets, u0, v, lambda u: -10.0 * u,
                           lambda ft: [a + 1e-6 * f for a, f in zip(v, ft)], 0.05, 0.8,
                           eps_abs=0.0, eps_rel=0.0, max_iter=2, force_density=True)

    a, b = run(W.Xf, 0), run(Xf2, 1)
    for d in range(3):
        assert np.all(np.isfinite(b["f_tilde"][d]))
        assert b["f_tilde"][d][nf] == 0.0
        assert np.max(np.abs(b["f_tilde"][d][:nf] - a["f_tilde"][d])) <= 1e-12 * max(
            1.0, np.max(np.abs(a["f_tilde"][d])))
