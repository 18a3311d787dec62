"""Pins of the 2D FP64 oracle (Q1 quadrilateral lattice x P1 triangles)
against what the mathematics fixes (no GPU).

Each test checks the oracle against something other than itself: textbook
closed forms on the reference triangle, an independent conical-product Gauss
rule (tests/refquad.py), exact 1D hat integrals, brute force by sub-sampling,
exact reproduction properties of the L2 projection (Section 2.3), and finite
differences for the gradients.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as wl
from tests.refquad import hat_integral_exact, ref_triangle_monomial, tri_integral

P2 = wl.plane
REF = np.array([[0, 0], [1, 0], [0, 1]], dtype=np.float64)


@pytest.fixture(scope="module")
def pl(oracle_mod):
    from oracle import plane
    plane.build(force=False)
    return plane


@pytest.fixture(scope="module")
def th1(pl):
    W = P2.workload2(1)
    return W, pl.assemble(W.faces, W.X, W.tris)


@pytest.fixture(scope="module")
def th1_dual(pl, th1):
    W, _ = th1
    return W, pl.assemble(W.faces, W.X, W.tris, dual=True)


def _field(faces, d, fn, pl):
    xs, ys = pl.lattice(faces, d)
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    return fn(X, Y)


# ---------------------------------------------------------------------------
# closed-form integration of three affine factors
# ---------------------------------------------------------------------------

def test_int3_reference_triangle_monomials(pl):
    """x^a y^b (a+b<=3) on the reference triangle: a! b!/(a+b+2)!."""
    coord = {0: REF[:, 0], 1: REF[:, 1]}
    one = np.ones(3)
    for a in range(4):
        for b in range(4 - a):
            fs = [coord[0]] * a + [coord[1]] * b
            fs += [one] * (3 - len(fs))
            got = pl.int3(REF, *fs)
            assert got == pytest.approx(float(ref_triangle_monomial(a, b)), rel=1e-14, abs=1e-16)


def test_int3_matches_gauss_rule_on_random_triangles(pl):
    rng = np.random.default_rng(5)
    for _ in range(20):
        Y = rng.uniform(-1, 2, size=(3, 2))
        c = rng.standard_normal((3, 3))           # three affine functions
        f = [c[m, 0] + Y @ c[m, 1:] for m in range(3)]
        got = pl.int3(Y, *f)
        want = tri_integral(Y, lambda p: np.prod([c[m, 0] + p @ c[m, 1:] for m in range(3)],
                                                 axis=0))
        assert got == pytest.approx(want, rel=1e-12, abs=1e-14)


# ---------------------------------------------------------------------------
# clipping
# ---------------------------------------------------------------------------

def test_clip_area_closed_forms(pl):
    T = REF
    # inside / containing / corner cut / empty / edge on a cell line
    assert pl.clip_area(T, [-1, -1], [2, 2]) == pytest.approx(0.5, rel=1e-15)
    assert pl.clip_area(T, [0, 0], [0.5, 0.5]) == pytest.approx(0.25, rel=1e-15)
    assert pl.clip_area(T, [0.25, 0], [1, 1]) == pytest.approx(0.75 ** 2 / 2, rel=1e-14)
    assert pl.clip_area(T, [0.5, 0.5], [1, 1]) == 0.0
    assert pl.clip_area(T, [-1, -1], [0, 1]) == 0.0       # shares the edge x = 0 only
    # band 0.2 <= y <= 0.6: trapezoid between heights, width 1 - y
    assert pl.clip_area(T, [-1, 0.2], [2, 0.6]) == pytest.approx(
        0.5 * (0.8 + 0.4) * 0.4, rel=1e-14)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_clip_pieces_tile_the_triangle(pl, seed):
    """Pieces over every cell of a grid add up to the triangle's area, also
    when vertices sit exactly on grid lines."""
    rng = np.random.default_rng(seed)
    fx = np.sort(np.concatenate([[-0.1, 1.1], rng.uniform(0, 1, 7)]))
    fy = np.sort(np.concatenate([[-0.1, 1.1], rng.uniform(0, 1, 6)]))
    T = rng.uniform(0, 1, size=(3, 2))
    if seed == 2:           # vertices on grid lines
        T[0] = [fx[3], fy[2]]
        T[1, 0] = fx[5]
    area = 0.5 * abs((T[1, 0] - T[0, 0]) * (T[2, 1] - T[0, 1]) -
                     (T[1, 1] - T[0, 1]) * (T[2, 0] - T[0, 0]))
    tot = sum(pl.clip_area(T, [fx[i], fy[j]], [fx[i + 1], fy[j + 1]])
              for i in range(fx.size - 1) for j in range(fy.size - 1))
    assert tot == pytest.approx(area, rel=1e-13)


# ---------------------------------------------------------------------------
# the coupling matrices
# ---------------------------------------------------------------------------

def test_row_sums_are_lumped_mass(pl, th1):
    """Σ_j N_j = 1 on the lattice hull, so Σ_j B_ij = ∫ λ_i = Σ_{T∋i} |T|/3."""
    W, R = th1
    m = pl.lumped_mass(W.X, W.tris)
    for d in range(2):
        rs = np.asarray(R.B[d].sum(axis=1)).ravel()
        np.testing.assert_allclose(rs, m, rtol=1e-13, atol=0)


def test_total_is_exact_rectangle_area(pl):
    """Σ_ij B_ij over the tail alone is its exact (rectangle) area."""
    W = P2.workload2(2)
    tail = W.bodies[1]
    R = pl.assemble(W.faces, tail.X, tail.tris)
    for d in range(2):
        assert R.B[d].sum() == pytest.approx(tail.exact_area, rel=1e-13)


def test_column_sums_rectangle_closed_form(pl):
    """Σ_i B_ij = ∫_rect N_j = product of exact 1D hat integrals."""
    W = P2.workload2(1)
    tail = W.bodies[1]
    (x0, y0), (x1, y1) = tail.box
    R = pl.assemble(W.faces, tail.X, tail.tris)
    for d in range(2):
        lx, ly = pl.lattice(W.faces, d)
        cs = np.asarray(R.B[d].sum(axis=0)).ravel()
        nz = np.nonzero(cs)[0]
        assert nz.size > 10
        for j in nz[:: max(1, nz.size // 40)]:
            ix, iy = j % lx.size, j // lx.size
            want = hat_integral_exact(lx, ix, x0, x1) * hat_integral_exact(ly, iy, y0, y1)
            assert cs[j] == pytest.approx(want, rel=1e-12, abs=1e-18)


def test_affine_reproduction(pl, th1):
    """Q1 interpolates affine fields exactly and ∫ λ_i u = Σ_l M_il u(X_l):
    the consistent transfer returns u at the vertices."""
    W, R = th1
    for d in range(2):
        u = [_field(W.faces, e, lambda X, Y: 0.3 + 1.7 * X - 2.1 * Y, pl) for e in range(2)]
        us = pl.transfer_velocity(R, u, "consistent")
        want = 0.3 + 1.7 * W.X[:, 0] - 2.1 * W.X[:, 1]
        np.testing.assert_allclose(us[d], want, rtol=0, atol=1e-12)


def test_bilinear_action_exact(pl, th1):
    """For u = x y (in Q1), (B u)_i = ∫ λ_i x y: per triangle by an
    independent Gauss rule."""
    W, R = th1
    A = np.zeros(W.X.shape[0])
    for t in range(W.tris.shape[0]):
        Y = W.X[W.tris[t]]
        inv = np.linalg.inv(np.column_stack([np.ones(3), Y]))
        vals = tri_integral(Y, lambda p: (np.column_stack([np.ones(len(p)), p]) @ inv)
                            * (p[:, 0] * p[:, 1])[:, None])
        np.add.at(A, W.tris[t], vals)
    for d in range(2):
        u = _field(W.faces, d, lambda X, Y: X * Y, pl).ravel()
        np.testing.assert_allclose(R.B[d] @ u, A, rtol=1e-12, atol=1e-16)


def test_single_triangle_brute_force(pl):
    """Entries of B for one triangle spanning several cells, against a
    brute-force sum over a fine sub-triangulation with a Gauss rule on each
    sub-triangle (N_j is only piecewise bilinear, so the sum converges as
    the refinement grows; tolerance from the observed O(h^2) rate)."""
    faces = [np.array([0.0, 0.1, 0.25, 0.4, 0.6, 0.7]), np.array([0.0, 0.15, 0.3, 0.5, 0.65])]
    X = np.array([[0.13, 0.21], [0.52, 0.11], [0.31, 0.47]])
    tris = np.array([[0, 1, 2]], dtype=np.int32)
    R = pl.assemble(faces, X, tris)
    inv = np.linalg.inv(np.column_stack([np.ones(3), X]))
    k = 64                                  # 4^6 sub-triangles
    for d in range(2):
        lx, ly = pl.lattice(faces, d)
        B = R.B[d].toarray()
        # barycentric sub-grid
        pts, tri = [], []
        idx = {}
        for i in range(k + 1):
            for j in range(k + 1 - i):
                idx[(i, j)] = len(pts)
                a, b = i / k, j / k
                pts.append(X[0] + a * (X[1] - X[0]) + b * (X[2] - X[0]))
        for i in range(k):
            for j in range(k - i):
                tri.append((idx[(i, j)], idx[(i + 1, j)], idx[(i, j + 1)]))
                if j + i + 1 < k:
                    tri.append((idx[(i + 1, j)], idx[(i + 1, j + 1)], idx[(i, j + 1)]))
        pts = np.array(pts)
        acc = np.zeros((3, lx.size * ly.size))

        def hats(nodes, x):
            H = np.zeros((x.size, nodes.size))
            c = np.clip(np.searchsorted(nodes, x, side="right") - 1, 0, nodes.size - 2)
            w = (x - nodes[c]) / (nodes[c + 1] - nodes[c])
            H[np.arange(x.size), c] = 1 - w
            H[np.arange(x.size), c + 1] = w
            return H

        for t in tri:
            Y = pts[list(t)]

            def f(p):
                lam = np.column_stack([np.ones(len(p)), p]) @ inv          # (m, 3)
                N = np.einsum("mi,mj->mij", hats(ly, p[:, 1]), hats(lx, p[:, 0]))
                N = N.reshape(len(p), -1)
                return np.einsum("mi,mj->mij", lam, N)

            acc += tri_integral(Y, f, n=3)
        err = np.abs(acc - B).max() / np.abs(B).max()
        assert err < 2e-4, err


def test_translation_by_one_cell_shifts_columns(pl):
    faces = [np.linspace(0, 1, 33), np.linspace(0, 1, 29)]
    W = P2.workload2(1)
    body = W.bodies[1]
    X = body.X - body.X.mean(0) + 0.5
    R0 = pl.assemble(faces, X, body.tris)
    R1 = pl.assemble(faces, X + np.array([1 / 32, 0.0]), body.tris)
    for d in range(2):
        A0, A1 = R0.B[d].tocoo(), R1.B[d].tocoo()
        m0 = sp.csr_matrix((A0.data, (A0.row, A0.col + 1)), shape=A1.shape)
        assert abs(m0 - R1.B[d]).max() <= 1e-13 * abs(R1.B[d]).max()


def test_permutation_invariance(pl, th1):
    """Reordering a triangle's vertices (flipping its orientation) leaves B unchanged."""
    W, R = th1
    t2 = W.tris[:, [0, 2, 1]].copy()
    R2 = pl.assemble(W.faces, W.X, t2)
    for d in range(2):
        assert abs(R.B[d] - R2.B[d]).max() <= 1e-13 * abs(R.B[d]).max()   # rounding order


def test_force_conservation_and_adjoint(pl, th1):
    """Σ_j (B^T f)_j = Σ_i m_i f_i (partition of unity), and <B u, f> = <u, B^T f>."""
    W, R = th1
    f = W.f_s()
    m = pl.lumped_mass(W.X, W.tris)
    ff = pl.transfer_force(R, f)
    for d in range(2):
        assert ff[d].sum() == pytest.approx(float(m @ f[d]), rel=1e-12)
        u = np.random.default_rng(d).standard_normal(R.B[d].shape[1])
        assert float((R.B[d] @ u) @ f[d]) == pytest.approx(float(u @ ff[d]), rel=1e-12)


def test_mass_matrix_against_gauss_rule(pl, th1):
    W, _ = th1
    ref = np.zeros((W.X.shape[0], W.X.shape[0]))
    for t in W.tris[:40]:
        Y = W.X[t]
        inv = np.linalg.inv(np.column_stack([np.ones(3), Y]))
        loc = tri_integral(Y, lambda p: np.einsum(
            "mi,mj->mij", np.column_stack([np.ones(len(p)), p]) @ inv,
            np.column_stack([np.ones(len(p)), p]) @ inv))
        ref[np.ix_(t, t)] += loc
    M40 = pl.consistent_mass(W.X, W.tris[:40]).toarray()
    np.testing.assert_allclose(M40, ref, rtol=1e-12, atol=1e-20)


# ---------------------------------------------------------------------------
# dual multipliers
# ---------------------------------------------------------------------------

def test_dual_biorthogonality_closed_form(pl):
    """ψ_i = 4λ_i − 1: ∫ ψ_i λ_j = δ_ij |T|/3 on a triangle (Gauss rule)."""
    Y = np.array([[0.1, 0.2], [0.9, 0.35], [0.3, 0.8]])
    inv = np.linalg.inv(np.column_stack([np.ones(3), Y]))
    G = tri_integral(Y, lambda p: np.einsum(
        "mi,mj->mij", 4 * (np.column_stack([np.ones(len(p)), p]) @ inv) - 1,
        np.column_stack([np.ones(len(p)), p]) @ inv))
    area = 0.5 * abs(np.linalg.det(np.column_stack([Y[1] - Y[0], Y[2] - Y[0]])))
    np.testing.assert_allclose(G, np.eye(3) * area / 3, atol=1e-15)


def test_dual_affine_reproduction(pl, th1_dual):
    W, R = th1_dual
    u = [_field(W.faces, e, lambda X, Y: -0.4 + 0.6 * X + 1.3 * Y, pl) for e in range(2)]
    us = pl.transfer_velocity(R, u, "lumped")
    want = -0.4 + 0.6 * W.X[:, 0] + 1.3 * W.X[:, 1]
    for d in range(2):
        np.testing.assert_allclose(us[d], want, rtol=0, atol=1e-11)


def test_dual_row_sums_are_lumped_mass(pl, th1_dual):
    W, R = th1_dual
    m = pl.lumped_mass(W.X, W.tris)
    for d in range(2):
        np.testing.assert_allclose(np.asarray(R.B[d].sum(axis=1)).ravel(), m, rtol=1e-12)


# ---------------------------------------------------------------------------
# gradients
# ---------------------------------------------------------------------------

def _small_case():
    faces = [np.linspace(0.0, 1.0, 17), np.linspace(0.0, 1.0, 13)]
    rng = np.random.default_rng(11)
    b = P2.rect_body("r", (0.31, 0.27), (0.69, 0.58), 5, 4, 0.2, rng)
    return faces, b.X, b.tris


@pytest.mark.parametrize("mass,dual", [("lumped", False), ("consistent", False),
                                       ("lumped", True)])
def test_velocity_gradient_fd(pl, mass, dual):
    faces, X, tris = _small_case()
    k, phi = P2.fourier_modes2(6, 3, 77)
    u = [P2.fourier_field2(k[d], phi[d], *pl.lattice(faces, d)) for d in range(2)]
    tgt = P2.gaussian_nodal2(X.shape[0], 78)
    R = pl.assemble(faces, X, tris, dual=dual)
    us = pl.transfer_velocity(R, u, mass)
    _, gX = pl.velocity_vjp(R, u, us - tgt, mass)
    dirs = P2.fd_directions2(X.shape[0], 3, 79)
    h = 1e-6
    for D in dirs:
        lp = pl.velocity_loss(faces, X + h * D, tris, u, tgt, mass, dual)
        lm = pl.velocity_loss(faces, X - h * D, tris, u, tgt, mass, dual)
        fd = (lp - lm) / (2 * h)
        an = float(np.sum(gX * D))
        assert an == pytest.approx(fd, rel=2e-6, abs=1e-9)


def test_force_gradient_fd(pl):
    faces, X, tris = _small_case()
    f = P2.gaussian_nodal2(X.shape[0], 81)
    g = [np.random.default_rng(82 + d).standard_normal(pl.n_fluid(faces, d)) for d in range(2)]
    R = pl.assemble(faces, X, tris)
    _, gX = pl.force_vjp(R, f, g, alpha=1.3)

    def L(Xp):
        ff = pl.transfer_force(pl.assemble(faces, Xp, tris), f, alpha=1.3)
        return sum(float(ff[d] @ g[d]) for d in range(2))

    h = 1e-6
    for D in P2.fd_directions2(X.shape[0], 3, 83):
        fd = (L(X + h * D) - L(X - h * D)) / (2 * h)
        assert float(np.sum(gX * D)) == pytest.approx(fd, rel=2e-6, abs=1e-9)


# ---------------------------------------------------------------------------
# Picard coupling (Section 3) in the plane
# ---------------------------------------------------------------------------

def test_fluid_lumped_area(pl):
    """∫ N_j over the lattice hull, against a two-point Gauss rule per cell
    (exact for the bilinear hat) with the hat read off a piecewise-linear
    interpolant of a unit vector; the areas tile the hull."""
    faces = [np.concatenate([[0.0], np.cumsum(np.random.default_rng(3).uniform(0.5, 2.0, 9))]),
             np.linspace(-0.2, 0.3, 7)]
    g = np.array([-1.0, 1.0]) / np.sqrt(3.0)
    for d in range(2):
        lat = pl.lattice(faces, d)
        A = pl.fluid_lumped_volume(faces, d)
        assert A.shape == (lat[1].size, lat[0].size)
        q = []
        for L in lat:
            h = np.diff(L)
            xs = (0.5 * (L[:-1] + L[1:])[:, None] + 0.5 * h[:, None] * g[None, :]).ravel()
            ws = np.repeat(0.5 * h, 2)
            q.append((xs, ws))
        for j in range(lat[1].size):
            for i in range(lat[0].size):
                ex = np.zeros(lat[0].size)
                ex[i] = 1.0
                ey = np.zeros(lat[1].size)
                ey[j] = 1.0
                hx = np.interp(q[0][0], lat[0], ex)
                hy = np.interp(q[1][0], lat[1], ey)
                ref = float(hx @ q[0][1]) * float(hy @ q[1][1])
                assert abs(A[j, i] - ref) <= 1e-15 * max(1.0, ref)
        hull = (lat[0][-1] - lat[0][0]) * (lat[1][-1] - lat[1][0])
        assert abs(A.sum() - hull) <= 1e-13 * hull


@pytest.mark.parametrize("mode,density", [("lumped", False), ("consistent", False),
                                          ("dual", False), ("lumped", True)])
def test_fsi_picard_reaches_the_fixed_point(pl, mode, density):
    """With a linear spring for the solid and a fluid whose velocity responds
    linearly to the force, the fixed point of Steps 1-5 solves
    (I + k dt beta alpha T D⁻¹ Tᵀ) f = −k (û0 − û_rest + dt T v_base) per
    component, T = S⁻¹B and D the fluid nodes' lumped areas (identity
    without the density option): the Picard loop must land on the direct
    solution of that dense system."""
    faces, X, tris = _small_case()
    n = X.shape[0]
    dual = mode == "dual"
    mass = "consistent" if mode == "consistent" else "lumped"
    rng = np.random.default_rng(21)
    u_rest = 1e-3 * rng.standard_normal((2, n))
    v_base = [rng.standard_normal(pl.n_fluid(faces, d)) for d in range(2)]
    k_s, beta = 10.0, 0.5 if not density else 0.5 / 400.0

    def solid(u_hat):
        return -k_s * (u_hat - u_rest)

    def fluid(f_tilde):
        return [v_base[d] + beta * f_tilde[d] for d in range(2)]

    u0 = 1e-3 * np.random.default_rng(5).standard_normal((2, n))
    v0 = [np.zeros(pl.n_fluid(faces, d)) for d in range(2)]
    dt, alpha = 0.05, 0.8
    r = pl.fsi_step(faces, X, tris, u0, v0, solid, fluid, dt, alpha, eps_abs=1e-14, eps_rel=0.0,
                    max_iter=200, mass=mass, force_density=density, dual=dual)
    assert r["converged"]
    c = pl.assemble(faces, X + u0.T, tris, dual=dual)
    Sm = (np.diag(pl.lumped_mass(c.X, tris)) if mass == "lumped"
          else pl.consistent_mass(c.X, tris).toarray())
    for d in range(2):
        Td = np.linalg.solve(Sm, c.B[d].toarray())
        Dinv = (1.0 / pl.fluid_lumped_volume(faces, d).ravel() if density
                else np.ones(Td.shape[1]))
        A = np.eye(n) + k_s * dt * beta * alpha * (Td * Dinv[None, :]) @ Td.T
        rhs = -k_s * (u0[d] - u_rest[d] + dt * Td @ v_base[d])
        f_star = np.linalg.solve(A, rhs)
        assert np.max(np.abs(r["f_fsi"][d] - f_star)) <= 1e-11 * max(1.0, np.max(np.abs(f_star)))


def test_jacobi_scaled_mass_spectrum_bounds(pl):
    """The eigenvalues of D⁻¹M for the consistent planar P1 mass lie in
    [1/2, 2]: each triangle's D_e⁻¹M_e = (I + 11ᵀ)/2 has eigenvalues 1/2
    (twice) and 2, and the assembled Rayleigh quotient is a ratio of sums of
    the elements' quotients.  A jittered graded mesh, and one triangle's
    extremes exactly."""
    _, X, tris = _small_case()
    X = X * np.array([1.0, 4.0]) + 1e-3 * np.random.default_rng(9).standard_normal(X.shape)
    M = pl.consistent_mass(X, tris).toarray()
    d = np.diag(M)
    lam = np.linalg.eigvalsh(M / np.sqrt(np.outer(d, d)))
    assert lam.min() >= 0.5 - 1e-12 and lam.max() <= 2.0 + 1e-12
    T1 = np.array([[0, 0], [1, 0], [0.3, 1e-3]], dtype=np.float64)
    M1 = pl.consistent_mass(T1, np.array([[0, 1, 2]])).toarray()
    d1 = np.diag(M1)
    lam1 = np.linalg.eigvalsh(M1 / np.sqrt(np.outer(d1, d1)))
    np.testing.assert_allclose(lam1, [0.5, 0.5, 2.0], atol=1e-12)
