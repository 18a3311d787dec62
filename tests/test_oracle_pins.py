"""Pins of the FP64 oracle against what the mathematics fixes (no GPU).

Each test checks the oracle against something other than itself: textbook
closed forms, an independent Gauss rule (tests/refquad.py), exact 1D hat
integrals, Monte Carlo brute force, exact reproduction properties of the
L2 projection (Section 2.3), and finite differences for the gradients.
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import workloads as wl
from tests.refquad import hat_integral_exact, ref_simplex_monomial, stroud_rule, tet_integral


# ---------------------------------------------------------------------------
# closed-form integration of four affine factors
# ---------------------------------------------------------------------------

REF = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=np.float64)


def test_int4_reference_simplex_monomials(oracle_mod):
    """x^a y^b z^c (a+b+c<=4) on the reference simplex: a!b!c!/(a+b+c+3)!."""
    coord = {0: REF[:, 0], 1: REF[:, 1], 2: REF[:, 2]}
    one = np.ones(4)
    for a in range(5):
        for b in range(5 - a):
            for c in range(5 - a - b):
                facs = [coord[0]] * a + [coord[1]] * b + [coord[2]] * c
                facs += [one] * (4 - len(facs))
                got = oracle_mod.int4(REF, *facs)
                want = float(ref_simplex_monomial(a, b, c))
                assert abs(got - want) <= 1e-15 * want, (a, b, c, got, want)


def _poly_cube_exact(affs):
    """∫_[0,1]^3 Π (c0 + c1 x + c2 y + c3 z) with Fraction arithmetic."""
    poly = {(0, 0, 0): Fraction(1)}
    for c in affs:
        new = {}
        for (p, q, r), v in poly.items():
            for k, e in enumerate([(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]):
                key = (p + e[0], q + e[1], r + e[2])
                new[key] = new.get(key, 0) + v * Fraction(int(c[k]))
        poly = new
    return sum(v / ((p + 1) * (q + 1) * (r + 1)) for (p, q, r), v in poly.items())


def test_int4_unit_cube_kuhn(oracle_mod):
    """Six diagonal tets tile the unit cube: the sum of their closed forms must
    equal the exact cube integral of random integer affine products."""
    tets = wl.kuhn_tets((1, 1, 1))
    X = wl.hex_block((1, 1, 1)).astype(np.float64)
    rng = np.random.default_rng(7)
    for _ in range(20):
        affs = rng.integers(-5, 6, size=(4, 4))
        want = float(_poly_cube_exact(affs))
        got = 0.0
        for t in tets:
            Y = X[t]
            vals = [c[0] + Y @ c[1:] for c in affs]
            got += oracle_mod.int4(Y, *vals)
        assert abs(got - want) <= 1e-13 * max(1.0, abs(want))


def test_int4_matches_stroud_on_random_tets(oracle_mod):
    rng = np.random.default_rng(11)
    for _ in range(20):
        Y = rng.uniform(-1, 1, size=(4, 3))
        affs = rng.standard_normal((4, 4))
        vals = [c[0] + Y @ c[1:] for c in affs]
        got = oracle_mod.int4(Y, *vals)
        want = tet_integral(Y, lambda p: np.prod([c[0] + p @ c[1:] for c in affs], axis=0), n=4)
        assert abs(got - want) <= 1e-13 * max(1e-3, abs(want))


# ---------------------------------------------------------------------------
# clipping
# ---------------------------------------------------------------------------

def test_clip_volume_closed_form(oracle_mod):
    # reference simplex ∩ [0, 1/2]^3: the three corners beyond 1/2 are cut off
    got = oracle_mod.clip_volume(REF, np.zeros(3), np.full(3, 0.5))
    assert abs(got - 5.0 / 48.0) <= 1e-16
    # a box that contains the tet
    assert abs(oracle_mod.clip_volume(REF, -np.ones(3), np.ones(3) * 2) - 1 / 6) <= 1e-16
    # disjoint box
    assert oracle_mod.clip_volume(REF, np.full(3, 2.0), np.full(3, 3.0)) == 0.0
    # slab 1/4 <= x <= 1/2: ((3/4)^3 - (1/2)^3)/6
    got = oracle_mod.clip_volume(REF, np.array([0.25, -1, -1]), np.array([0.5, 2, 2]))
    assert abs(got - ((0.75 ** 3 - 0.5 ** 3) / 6.0)) <= 1e-16


@pytest.mark.parametrize("case", ["random", "on_planes", "coplanar_face"])
def test_clip_pieces_tile_the_tet(oracle_mod, case):
    """Σ over cells of |T ∩ C| = |T|, including vertices exactly on planes and
    faces lying in a cell plane."""
    rng = np.random.default_rng({"random": 1, "on_planes": 2, "coplanar_face": 3}[case])
    grid = np.linspace(0.0, 1.0, 9)
    for _ in range(25):
        if case == "random":
            P = rng.uniform(0.05, 0.95, size=(4, 3))
        elif case == "on_planes":
            P = grid[rng.integers(1, 8, size=(4, 3))]
            P[:, 0] += rng.uniform(-0.06, 0.06, 4) * (rng.random(4) < 0.5)
        else:
            P = rng.uniform(0.1, 0.9, size=(4, 3))
            P[:3, 2] = grid[4]
        vol = abs(np.linalg.det(P[1:] - P[0])) / 6.0
        if vol < 1e-6:
            continue
        tot = 0.0
        for i, j, k in itertools.product(range(8), repeat=3):
            tot += oracle_mod.clip_volume(P, np.array([grid[i], grid[j], grid[k]]),
                                          np.array([grid[i + 1], grid[j + 1], grid[k + 1]]))
        assert abs(tot - vol) <= 1e-13 * vol, (tot, vol)


# ---------------------------------------------------------------------------
# coupling matrix B on workloads
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def cfg1(oracle_mod):
    W = wl.workload(1)
    return W, oracle_mod.assemble(W.faces, W.X, W.tets)


@pytest.fixture(scope="module")
def cfg3s(oracle_mod):
    W = wl.workload(3, small=True)
    return W, oracle_mod.assemble(W.faces, W.X, W.tets)


def test_row_sums_are_lumped_mass(oracle_mod, cfg1, cfg3s):
    """Partition of unity of the Q1 hats: Σ_j B_ij = ∫ λ_i = m_i."""
    for W, c in (cfg1, cfg3s):
        m = oracle_mod.lumped_mass(W.X, W.tets)
        for d in range(3):
            rs = np.asarray(c.B[d].sum(axis=1)).ravel()
            assert np.max(np.abs(rs - m)) <= 1e-13 * m.max()


def test_total_is_exact_box_volume(oracle_mod, cfg1):
    W, c = cfg1
    for d in range(3):
        assert abs(c.B[d].sum() - W.bodies[0].exact_volume) <= 1e-15


def test_column_sums_box_closed_form(oracle_mod, cfg1):
    """For an axis-aligned box solid, Σ_i B_ij = ∫_box N_j, a product of three
    exact 1D hat integrals — for every fluid node of every component."""
    W, c = cfg1
    lo, hi = W.bodies[0].box
    for d in range(3):
        lat = oracle_mod.lattice(W.faces, d)
        I = [np.array([hat_integral_exact(lat[e], k, lo[e], hi[e]) for k in range(lat[e].size)])
             for e in range(3)]
        ref = np.einsum("k,j,i->kji", I[2], I[1], I[0]).ravel()
        cs = np.asarray(c.B[d].sum(axis=0)).ravel()
        assert np.max(np.abs(cs - ref)) <= 1e-13 * ref.max()


def _lattice_field(oracle_mod, faces, d, fn):
    xs, ys, zs = oracle_mod.lattice(faces, d)
    Z, Y, Xc = np.meshgrid(zs, ys, xs, indexing="ij")
    return fn(Xc, Y, Z)


def test_trilinear_action_exact(oracle_mod, cfg1, cfg3s):
    """A global trilinear p is reproduced exactly by the Q1 interpolant, so
    (B p)_i = ∫ λ_i p over whole tets (independent Gauss rule, no clipping)."""
    rng = np.random.default_rng(5)
    for W, c in (cfg1, cfg3s):
        co = rng.uniform(-1, 1, size=6)
        p = lambda x, y, z: (co[0] + co[1] * x) * (co[2] + co[3] * y) * (co[4] + co[5] * z)
        bary, wt = stroud_rule(4)
        ref = np.zeros(W.X.shape[0])
        vol = oracle_mod.tet_volumes(W.X, W.tets)
        for k in range(4):
            P = W.X[W.tets]                                    # (n_t, 4, 3)
            pts = np.einsum("qv,tve->tqe", bary, P)
            vals = p(pts[..., 0], pts[..., 1], pts[..., 2]) * bary[None, :, k]
            np.add.at(ref, W.tets[:, k], vol * (vals @ wt))
        for d in range(3):
            u = _lattice_field(oracle_mod, W.faces, d, p).ravel()
            got = c.B[d] @ u
            assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_affine_reproduction(oracle_mod, cfg1, cfg3s):
    """Consistent L2 projection reproduces affine fields at the nodes; the
    lumped one gives p at the mass-weighted point x̄_i."""
    for W, c in (cfg1, cfg3s):
        co = np.array([0.3, -1.2, 0.7, 2.1])
        p = lambda x, y, z: co[0] + co[1] * x + co[2] * y + co[3] * z
        u_f = [_lattice_field(oracle_mod, W.faces, d, p) for d in range(3)]
        us = oracle_mod.transfer_velocity(c, u_f, "consistent")
        want = p(W.X[:, 0], W.X[:, 1], W.X[:, 2])
        assert np.max(np.abs(us - want[None, :])) <= 1e-11
        ul = oracle_mod.transfer_velocity(c, u_f, "lumped")
        vol = oracle_mod.tet_volumes(W.X, W.tets)
        m = oracle_mod.lumped_mass(W.X, W.tets)
        xbar = np.zeros_like(W.X)
        s = W.X[W.tets].sum(axis=1)
        for k in range(4):
            np.add.at(xbar, W.tets[:, k], (vol / 20.0)[:, None] * (W.X[W.tets[:, k]] + s))
        xbar /= m[:, None]
        assert np.max(np.abs(ul - p(xbar[:, 0], xbar[:, 1], xbar[:, 2])[None, :])) <= 1e-11


def test_whole_tet_inside_one_cell(oracle_mod):
    """A tet strictly inside one cell: B entries are whole-tet integrals."""
    faces = [np.linspace(0, 1, 5)] * 3
    rng = np.random.default_rng(3)
    # [.375, .5] lies inside one cell of both the face lattice ([.25, .5]) and
    # the centre lattice ([.375, .625]) along every axis
    X = 0.375 + 0.125 * rng.uniform(0.1, 0.9, size=(4, 3))
    tets = np.array([[0, 1, 2, 3]], dtype=np.int32)
    c = oracle_mod.assemble(faces, X, tets)
    for d in range(3):
        lat = oracle_mod.lattice(faces, d)
        shape = (lat[2].size, lat[1].size, lat[0].size)
        B = c.B[d].toarray()
        for j in np.nonzero(np.abs(B).sum(0))[0]:
            kz, ky, kx = np.unravel_index(j, shape)

            def f(p, kx=kx, ky=ky, kz=kz):
                hx = oracle_mod.hat_1d(lat[0], p[:, 0])[:, kx]
                hy = oracle_mod.hat_1d(lat[1], p[:, 1])[:, ky]
                hz = oracle_mod.hat_1d(lat[2], p[:, 2])[:, kz]
                A = np.ones((p.shape[0], 4))
                A[:, 1:] = p
                lam = A @ np.linalg.inv(np.hstack([np.ones((4, 1)), X]))
                return lam * (hx * hy * hz)[:, None]

            ref = tet_integral(X, f, n=4)
            assert np.max(np.abs(B[:, j] - ref)) <= 1e-15


def test_monte_carlo_entries(oracle_mod):
    """Brute force: B_ij by uniform sampling of each tet (no clipping)."""
    faces = [np.linspace(0, 1, 5)] * 3
    rng = np.random.default_rng(9)
    W = wl.box_body("b", (0.4, 0.3, 0.3), (0.5, 0.5, 0.5), (2, 1, 1), 0.15,
                    np.random.default_rng(1))
    X, tets = W.X, W.tets
    c = oracle_mod.assemble(faces, X, tets)
    ns = 200_000
    for d in range(3):
        lat = oracle_mod.lattice(faces, d)
        nx, ny = lat[0].size, lat[1].size
        est = {}
        var = {}
        vol = oracle_mod.tet_volumes(X, tets)
        for t in range(tets.shape[0]):
            lam = rng.dirichlet(np.ones(4), size=ns)
            p = lam @ X[tets[t]]
            hx = oracle_mod.hat_1d(lat[0], p[:, 0])
            hy = oracle_mod.hat_1d(lat[1], p[:, 1])
            hz = oracle_mod.hat_1d(lat[2], p[:, 2])
            for kx in np.nonzero(hx.any(0))[0]:
                for ky in np.nonzero(hy.any(0))[0]:
                    for kz in np.nonzero(hz.any(0))[0]:
                        N = hx[:, kx] * hy[:, ky] * hz[:, kz]
                        j = kx + nx * (ky + ny * kz)
                        for a in range(4):
                            s = vol[t] * lam[:, a] * N
                            key = (tets[t, a], j)
                            est[key] = est.get(key, 0.0) + s.mean()
                            var[key] = var.get(key, 0.0) + s.var() / ns
        B = c.B[d].tocsr()
        seen = 0
        for (i, j), v in est.items():
            sig = math.sqrt(var[(i, j)])
            assert abs(B[i, j] - v) <= 5 * sig + 1e-12, (d, i, j, B[i, j], v, sig)
            seen += 1
        assert seen > 20
        # nothing in B that sampling never reached
        assert abs(B.sum() - sum(est.values())) <= 5 * math.sqrt(sum(var.values())) + 1e-9


def test_translation_by_one_cell_shifts_columns(oracle_mod, cfg1):
    W, c = cfg1
    h = 1.0 / 32.0                       # exact in binary
    c2 = oracle_mod.assemble(W.faces, W.X + np.array([h, 0.0, 0.0]), W.tets)
    for d in range(3):
        A = c.B[d].tocoo()
        Bm = c2.B[d].tocsr()
        nx = oracle_mod.lattice_shape(W.faces, d)[0]
        assert np.allclose(Bm[A.row, A.col + 1].A.ravel(), A.data, rtol=1e-12, atol=1e-18)
        assert nx > 0


def test_permutation_invariance(oracle_mod, cfg1):
    W, c = cfg1
    rng = np.random.default_rng(4)
    perm_t = rng.permutation(W.tets.shape[0])
    tets = W.tets[perm_t]
    tets = np.stack([np.roll(t, rng.integers(0, 4)) for t in tets]).astype(np.int32)
    c2 = oracle_mod.assemble(W.faces, W.X, tets)
    for d in range(3):
        assert abs(c.B[d] - c2.B[d]).max() <= 1e-17


def test_force_conservation_and_adjoint(oracle_mod, cfg1):
    W, c = cfg1
    f_s = W.f_s()
    alpha = 0.7
    f_f = oracle_mod.transfer_force(c, f_s, alpha)
    m = oracle_mod.lumped_mass(W.X, W.tets)
    for d in range(3):
        assert abs(f_f[d].sum() - alpha * (m * f_s[d]).sum()) <= 1e-15
    # the literal transpose on a load vector, with a consistent-mass load of
    # a density, returns the same field
    M = oracle_mod.consistent_mass(W.X, W.tets)
    load = np.stack([M @ f_s[d] for d in range(3)])
    f2 = oracle_mod.transfer_force(c, load, alpha, load=True)
    for d in range(3):
        assert np.max(np.abs(f2[d] - f_f[d])) <= 1e-12 * np.max(np.abs(f_f[d]))


def test_mass_matrix_against_gauss_rule(oracle_mod, cfg1):
    W, _ = cfg1
    M = oracle_mod.consistent_mass(W.X, W.tets).toarray()
    ref = np.zeros_like(M)
    for t in W.tets:
        P = W.X[t]
        A = np.linalg.inv(np.hstack([np.ones((4, 1)), P]))

        def f(p):
            q = np.hstack([np.ones((p.shape[0], 1)), p]) @ A
            return q[:, :, None] * q[:, None, :]

        ref[np.ix_(t, t)] += tet_integral(P, f, n=3)
    assert np.max(np.abs(M - ref)) <= 1e-15
    assert np.allclose(M.sum(1), oracle_mod.lumped_mass(W.X, W.tets), rtol=1e-13, atol=0)


# ---------------------------------------------------------------------------
# gradients against central finite differences
# ---------------------------------------------------------------------------

def _tiny(oracle_mod):
    faces = [np.linspace(0, 1, 9)] * 3
    b = wl.box_body("b", (0.3, 0.2, 0.2), (0.5, 0.48, 0.51), (2, 1, 1), 0.15,
                    np.random.default_rng(12))
    k, phi = wl.fourier_modes(4, 2, 77)
    u_f = []
    for d in range(3):
        xs, ys, zs = oracle_mod.lattice(faces, d)
        u_f.append(wl.fourier_field(k[d], phi[d], xs, ys, zs).numpy())
    return faces, b.X.copy(), b.tets, u_f


@pytest.mark.parametrize("mass", ["lumped", "consistent"])
def test_velocity_gradient_fd(oracle_mod, mass):
    faces, X, tets, u_f = _tiny(oracle_mod)
    ut = wl.gaussian_nodal(X.shape[0], 99)
    c = oracle_mod.assemble(faces, X, tets)
    us = oracle_mod.transfer_velocity(c, u_f, mass)
    g_uf, gX = oracle_mod.velocity_vjp(c, u_f, us - ut, mass)
    dirs = wl.fd_directions(X.shape[0], 6, 5001)
    h = 1e-6
    for D in dirs:
        Lp = oracle_mod.velocity_loss(faces, X + h * D, tets, u_f, ut, mass)
        Lm = oracle_mod.velocity_loss(faces, X - h * D, tets, u_f, ut, mass)
        fd = (Lp - Lm) / (2 * h)
        an = float(np.sum(gX * D))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)
    # g_uf is exact: L is quadratic in u_f, check one direction
    rng = np.random.default_rng(3)
    du = [rng.standard_normal(u.shape) for u in u_f]
    L0 = oracle_mod.velocity_loss(faces, X, tets, [u + 1e-3 * v for u, v in zip(u_f, du)], ut, mass)
    L1 = oracle_mod.velocity_loss(faces, X, tets, [u - 1e-3 * v for u, v in zip(u_f, du)], ut, mass)
    fd = (L0 - L1) / 2e-3
    an = sum(float(np.dot(g_uf[d], du[d].ravel())) for d in range(3))
    assert abs(fd - an) <= 1e-9 * max(1.0, abs(an))


def test_force_gradient_fd(oracle_mod):
    faces, X, tets, u_f = _tiny(oracle_mod)
    f_s = wl.gaussian_nodal(X.shape[0], 31)
    g_ff = [np.asarray(u).ravel() for u in u_f]       # any fixed fluid cotangent
    alpha = 1.3

    def L(Xp):
        cc = oracle_mod.assemble(faces, Xp, tets)
        ff = oracle_mod.transfer_force(cc, f_s, alpha)
        return sum(float(np.dot(ff[d], g_ff[d])) for d in range(3))

    c = oracle_mod.assemble(faces, X, tets)
    g_fs, gX = oracle_mod.force_vjp(c, f_s, g_ff, alpha)
    h = 1e-6
    for D in wl.fd_directions(X.shape[0], 4, 5002):
        fd = (L(X + h * D) - L(X - h * D)) / (2 * h)
        an = float(np.sum(gX * D))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)
    # g_fs is exact (linear)
    ff = oracle_mod.transfer_force(c, f_s, alpha)
    assert abs(sum(float(np.dot(ff[d], g_ff[d])) for d in range(3)) - float(np.sum(g_fs * f_s))) \
        <= 1e-12 * max(1.0, abs(float(np.sum(g_fs * f_s))))


# ---------------------------------------------------------------------------
# dual ("pseudo" L2) multipliers, Section 2.3 eq. biorth
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def cfg1_dual(oracle_mod):
    W = wl.workload(1)
    return W, oracle_mod.assemble(W.faces, W.X, W.tets, dual=True)


@pytest.fixture(scope="module")
def cfg3s_dual(oracle_mod):
    W = wl.workload(3, small=True)
    return W, oracle_mod.assemble(W.faces, W.X, W.tets, dual=True)


def test_dual_affine_reproduction(oracle_mod, cfg1_dual, cfg3s_dual):
    """Biorthogonality (∫ λ_j ψ_i = δ_ij ∫ ψ_i) makes the transfer with the
    diagonal S reproduce affine fields exactly at the nodes: ∫ ψ_i p =
    Σ_j p(x_j) ∫ ψ_i λ_j = p(x_i) m_i, and the Q1 interpolant of p is p."""
    for W, c in (cfg1_dual, cfg3s_dual):
        co = np.array([-0.4, 0.9, -1.7, 1.3])
        p = lambda x, y, z: co[0] + co[1] * x + co[2] * y + co[3] * z
        u_f = [_lattice_field(oracle_mod, W.faces, d, p) for d in range(3)]
        us = oracle_mod.transfer_velocity(c, u_f, "lumped")
        want = p(W.X[:, 0], W.X[:, 1], W.X[:, 2])
        assert np.max(np.abs(us - want[None, :])) <= 1e-11
    with pytest.raises(ValueError):
        oracle_mod.transfer_velocity(cfg1_dual[1], u_f, "consistent")


def test_dual_row_sums_are_lumped_mass(oracle_mod, cfg1_dual, cfg3s_dual):
    """Σ_j B_ij = ∫ ψ_i = m_i: the dual multipliers integrate like the hats.
    (5 b_i − Σ_k b_k scales the rounding of the λ products by up to 9, hence
    1e-12 where the standard rows are held to 1e-13.)"""
    for W, c in (cfg1_dual, cfg3s_dual):
        m = oracle_mod.lumped_mass(W.X, W.tets)
        for d in range(3):
            rs = np.asarray(c.B[d].sum(axis=1)).ravel()
            assert np.max(np.abs(rs - m)) <= 1e-12 * m.max()


def test_dual_gradients_fd(oracle_mod):
    """Reverse mode of the dual transfers against central differences."""
    faces, X, tets, u_f = _tiny(oracle_mod)
    ut = wl.gaussian_nodal(X.shape[0], 98)
    c = oracle_mod.assemble(faces, X, tets, dual=True)
    us = oracle_mod.transfer_velocity(c, u_f, "lumped")
    _, gX = oracle_mod.velocity_vjp(c, u_f, us - ut, "lumped")
    h = 1e-6
    for D in wl.fd_directions(X.shape[0], 4, 5011):
        Lp = oracle_mod.velocity_loss(faces, X + h * D, tets, u_f, ut, "lumped", dual=True)
        Lm = oracle_mod.velocity_loss(faces, X - h * D, tets, u_f, ut, "lumped", dual=True)
        fd = (Lp - Lm) / (2 * h)
        an = float(np.sum(gX * D))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)
    f_s = wl.gaussian_nodal(X.shape[0], 32)
    g_ff = [np.asarray(u).ravel() for u in u_f]

    def L(Xp):
        cc = oracle_mod.assemble(faces, Xp, tets, dual=True)
        ff = oracle_mod.transfer_force(cc, f_s, 0.7)
        return sum(float(np.dot(ff[d], g_ff[d])) for d in range(3))

    _, gXf = oracle_mod.force_vjp(c, f_s, g_ff, 0.7)
    for D in wl.fd_directions(X.shape[0], 3, 5012):
        fd = (L(X + h * D) - L(X - h * D)) / (2 * h)
        an = float(np.sum(gXf * D))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)


# ---------------------------------------------------------------------------
# Picard coupling (Section 3) and the fluid lattice's lumped volume
# ---------------------------------------------------------------------------

def test_fluid_lumped_volume(oracle_mod):
    """∫ N_j over the lattice hull = product of exact 1D hat integrals; the
    volumes tile the hull."""
    W = wl.workload(3, small=True)                 # stretched y faces
    for d in range(3):
        lat = oracle_mod.lattice(W.faces, d)
        V = oracle_mod.fluid_lumped_volume(W.faces, d)
        I = [np.array([hat_integral_exact(lat[e], k, lat[e][0], lat[e][-1])
                       for k in range(lat[e].size)]) for e in range(3)]
        ref = np.einsum("k,j,i->kji", I[2], I[1], I[0])
        assert np.max(np.abs(V - ref)) <= 1e-15 * ref.max()
        hull = np.prod([lat[e][-1] - lat[e][0] for e in range(3)])
        assert abs(V.sum() - hull) <= 1e-13 * hull


def _fsi_stubs(oracle_mod, n_vert, faces, seed):
    """Linear solid and fluid operators: a spring toward a rest displacement
    and a fluid whose velocity responds linearly to the force."""
    rng = np.random.default_rng(seed)
    u_rest = 1e-3 * rng.standard_normal((3, n_vert))
    k_s = 10.0
    v_base = [rng.standard_normal(oracle_mod.n_fluid(faces, d)) for d in range(3)]
    beta = 0.5

    def solid(u_hat):
        return -k_s * (u_hat - u_rest)

    def fluid(f_tilde):
        return [v_base[d] + beta * f_tilde[d] for d in range(3)]

    return solid, fluid, (u_rest, k_s, v_base, beta)


@pytest.mark.parametrize("mode", ["lumped", "consistent", "dual"])
def test_fsi_picard_reaches_the_fixed_point(oracle_mod, mode):
    """With linear stubs the fixed point of Steps 1-5 solves
    (I + k dt beta alpha T Tᵀ) f = −k (û0 − û_rest + dt T v_base) with
    T = S⁻¹B; the Picard iteration (Step 6 stopping test) must land on the
    direct solution of that dense system."""
    faces, X, tets, _ = _tiny(oracle_mod)
    n = X.shape[0]
    dual = mode == "dual"
    mass = "consistent" if mode == "consistent" else "lumped"
    solid, fluid, (u_rest, k_s, v_base, beta) = _fsi_stubs(oracle_mod, n, faces, 21)
    rng = np.random.default_rng(5)
    u0 = 1e-3 * rng.standard_normal((3, n))
    v0 = [np.zeros(oracle_mod.n_fluid(faces, d)) for d in range(3)]
    dt, alpha = 0.05, 0.8
    r = oracle_mod.fsi_step(faces, X, tets, u0, v0, solid, fluid, dt, alpha, eps_abs=1e-14,
                            eps_rel=0.0, max_iter=200, mass=mass, dual=dual)
    assert r["converged"]
    c = oracle_mod.assemble(faces, X + u0.T, tets, dual=dual)
    S = (oracle_mod.lumped_mass(c.X, tets) if mass == "lumped" else None)
    Sm = np.diag(S) if S is not None else oracle_mod.consistent_mass(c.X, tets).toarray()
    for d in range(3):
        Td = np.linalg.solve(Sm, c.B[d].toarray())
        A = np.eye(n) + k_s * dt * beta * alpha * Td @ Td.T
        rhs = -k_s * (u0[d] - u_rest[d] + dt * Td @ v_base[d])
        f_star = np.linalg.solve(A, rhs)
        assert np.max(np.abs(r["f_fsi"][d] - f_star)) <= 1e-11 * max(1.0, np.max(np.abs(f_star)))


# ---------------------------------------------------------------------------
# Spectrum of the Jacobi-scaled P1 mass (the bounds the consistent solve
# relies on)
# ---------------------------------------------------------------------------

def test_jacobi_scaled_mass_spectrum_bounds(oracle_mod):
    """The eigenvalues of D⁻¹M (D = diag M) for the consistent P1 mass lie in
    [1/2, 5/2] whatever the element shapes: each element's D_e⁻¹M_e =
    (I + 11ᵀ)/2 has eigenvalues 1/2 (three times) and 5/2, and the Rayleigh
    quotient of the assembled pair is a ratio of sums of the elements'
    quotients.  Checked on a jittered mesh with a graded and a sliver
    element, and the single-element extremes attained exactly."""
    _, X, tets, _ = _tiny(oracle_mod)
    rng = np.random.default_rng(8)
    X = X * np.array([1.0, 3.0, 0.2]) + 1e-3 * rng.standard_normal(X.shape)
    M = oracle_mod.consistent_mass(X, tets).toarray()
    d = np.diag(M)
    lam = np.linalg.eigvalsh(M / np.sqrt(np.outer(d, d)))
    assert lam.min() >= 0.5 - 1e-12 and lam.max() <= 2.5 + 1e-12
    T1 = np.array([[0, 0, 0], [1, 0, 0], [0.3, 2, 0], [0.1, 0.2, 1e-3]], dtype=np.float64)
    M1 = oracle_mod.consistent_mass(T1, np.array([[0, 1, 2, 3]])).toarray()
    d1 = np.diag(M1)
    lam1 = np.linalg.eigvalsh(M1 / np.sqrt(np.outer(d1, d1)))
    np.testing.assert_allclose(lam1, [0.5, 0.5, 0.5, 2.5], atol=1e-12)


# ---------------------------------------------------------------------------
# exact rationals
# ---------------------------------------------------------------------------

def _exact_cases():
    """The first tets of the 144-tet beam on its 32^3 grid, and hand-made tets
    on a stretched dyadic grid: one random, one with every vertex on lattice
    planes, two with a face in a lattice plane (z = 0.5 is a plane of
    component 2's lattice, x = 0.3125 of components 1 and 2), all inside the
    lattices' hull [0.125, 0.875]^3."""
    W = wl.workload(1)
    yield "beam144 first tets", W.faces, W.X, W.tets[:2]
    f = np.array([0.0, 0.25, 0.375, 0.5, 0.75, 1.0])
    faces = [f, f, f]
    rng = np.random.default_rng(11)
    X = np.concatenate([
        rng.uniform(0.15, 0.85, size=(4, 3)),
        [[0.25, 0.3125, 0.4375], [0.75, 0.3125, 0.5], [0.3125, 0.75, 0.4375], [0.5, 0.5, 0.75]],
        [[0.2, 0.3, 0.5], [0.7, 0.35, 0.5], [0.4, 0.8, 0.5], [0.45, 0.5, 0.8]],
        [[0.3125, 0.2, 0.3], [0.3125, 0.7, 0.35], [0.3125, 0.4, 0.8], [0.6, 0.45, 0.5]],
    ])
    yield "hand tets", faces, X, np.arange(16, dtype=np.int32).reshape(4, 4)


@pytest.mark.parametrize("case", [0, 1])
def test_B_matches_exact_rationals(oracle_mod, case):
    """Every entry of the oracle's FP64 B on small cases equals the exact
    rational ∫ λ_i N_j (tests/exact_b.py: face-list clipping, monomial
    expansion in each sub-tetrahedron's barycentric coordinates) to 1e-14
    of the largest entry, including vertices and faces lying in lattice
    planes."""
    from tests.exact_b import assemble_exact
    name, faces, X, T = list(_exact_cases())[case]
    E = assemble_exact(faces, X, T)
    R = oracle_mod.assemble(faces, X, T)
    scale = max(abs(float(v)) for v in E.values())
    worst = 0.0
    for (d, i, j), v in E.items():
        worst = max(worst, abs(R.B[d][i, j] - float(v)))
    for d in range(3):
        C = R.B[d].tocoo()
        for i, j, v in zip(C.row, C.col, C.data):
            if (d, int(i), int(j)) not in E:
                worst = max(worst, abs(v))
    assert len(E) > 0
    assert worst <= 1e-14 * scale, (name, worst / scale)
