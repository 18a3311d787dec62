"""Seeded synthetic workloads for the fluid-grid <-> solid-mesh transfer.

The paper's meshes and flow fields are not available, so every input here is
synthetic and shaped like its 3D case (Section 4.3: a P1 tetrahedral solid
with element size close to the fluid spacing, inside a stretched rectilinear
grid).  What is generated:

* fluid grids: monotone face-coordinate arrays per axis, uniform or
  tanh-stretched about the domain centre (finest spacing at the centre);
* solid meshes: structured hexahedra, each split into the six tetrahedra that
  share its main diagonal (a conforming mesh), with seeded node jitter whose
  normal component is zero on the body's faces (so box bodies keep their
  exact volume), then placed by a rigid or curved map;
* fields: sums of Fourier modes sampled at caller-supplied coordinates, and
  Gaussian nodal vectors.

Nothing in this module computes any part of the transfer itself: node
coordinates of the staggered velocity lattices are passed in by the caller.

Seeds for workload c: mesh 1000+c, fluid field 2000+c, solid force 3000+c,
target 4000+c, finite-difference directions 5000+c, displacement phase 6000+c.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "uniform_faces", "stretched_faces", "hex_block", "kuhn_tets", "jitter_block",
    "Body", "Workload", "workload", "fourier_modes", "fourier_field",
    "gaussian_nodal", "fd_directions", "bending_displacement", "signed_volumes6",
    "WORKLOAD_NAMES", "box_body", "tilted_plate", "shell_sector", "merge_bodies",
]


# ----------------------------------------------------------------------------
# Fluid grids
# ----------------------------------------------------------------------------

def uniform_faces(n: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """n uniform cells on [lo, hi]: n+1 face coordinates."""
    f = lo + (hi - lo) * (np.arange(n + 1, dtype=np.float64) / n)
    f[0], f[-1] = lo, hi
    return f


def _tanh_faces(n: int, gamma: float) -> np.ndarray:
    j = np.arange(n + 1, dtype=np.float64)
    t = (2.0 * j / n - 1.0) * math.tanh(gamma)
    return 0.5 + np.arctanh(t) / (2.0 * gamma)


def stretched_faces(n: int, ratio: float, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """tanh-stretched faces on [lo, hi], finest at the centre.

    The stretching parameter is found by bisection so that the discrete
    ratio (largest / smallest spacing) equals `ratio`.
    """
    def disc_ratio(g):
        d = np.diff(_tanh_faces(n, g))
        return d.max() / d.min()

    a, b = 1e-6, 10.0
    for _ in range(200):
        m = 0.5 * (a + b)
        if disc_ratio(m) < ratio:
            a = m
        else:
            b = m
    f = _tanh_faces(n, 0.5 * (a + b))
    f[0], f[-1] = 0.0, 1.0
    f = lo + (hi - lo) * f
    f[0], f[-1] = lo, hi
    assert np.all(np.diff(f) > 0)
    return f


# ----------------------------------------------------------------------------
# Solid meshes
# ----------------------------------------------------------------------------

def hex_block(n: tuple[int, int, int]) -> np.ndarray:
    """Integer lattice indices (i, j, k) of the (n+1)^3 block vertices,
    i fastest.  Returned shape (n_v, 3), int64."""
    nx, ny, nz = n
    k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1),
                          indexing="ij")
    return np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)


def kuhn_tets(n: tuple[int, int, int]) -> np.ndarray:
    """Six tetrahedra per hexahedron, all sharing the (0,0,0)-(1,1,1)
    diagonal; the result is conforming across hexahedra.  int32 (6*nh, 4)."""
    nx, ny, nz = n

    def vid(i, j, k):
        return i + (nx + 1) * (j + (ny + 1) * k)

    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    unit = np.eye(3, dtype=np.int64)
    tets = []
    for perm in ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)):
        p0 = np.zeros(3, dtype=np.int64)
        p1 = unit[perm[0]]
        p2 = p1 + unit[perm[1]]
        p3 = np.ones(3, dtype=np.int64)
        tets.append(np.stack([vid(i + p[0], j + p[1], k + p[2]) for p in (p0, p1, p2, p3)],
                             axis=1))
    # hex-major order: the six tets of one hexahedron are consecutive
    t = np.stack(tets, axis=1).reshape(-1, 4)
    return t.astype(np.int32)


def signed_volumes6(X: np.ndarray, tets: np.ndarray) -> np.ndarray:
    """6x signed volumes (determinants); used only to reject inverted meshes."""
    a = X[tets[:, 1]] - X[tets[:, 0]]
    b = X[tets[:, 2]] - X[tets[:, 0]]
    c = X[tets[:, 3]] - X[tets[:, 0]]
    return np.einsum("ij,ij->i", a, np.cross(b, c))


def jitter_block(idx: np.ndarray, n: tuple[int, int, int], frac: float,
                 rng: np.random.Generator) -> np.ndarray:
    """Parametric coordinates (in units of one hexahedron) with seeded jitter
    U(-frac, frac) per component; the component normal to a block face is
    zero on that face, so the block boundary does not move."""
    q = idx.astype(np.float64)
    d = rng.uniform(-frac, frac, size=q.shape)
    for e in range(3):
        on_face = (idx[:, e] == 0) | (idx[:, e] == n[e])
        d[on_face, e] = 0.0
    return q + d


@dataclass
class Body:
    name: str
    X: np.ndarray          # (n_v, 3) float64
    tets: np.ndarray       # (n_t, 4) int32
    exact_volume: float | None = None   # exact body volume when it is a box
    box: tuple | None = None            # axis-aligned bounds ((lo),(hi)) when it is a box


def _make_body(name, n, frac, rng, mapping, exact_volume=None, box=None):
    idx = hex_block(n)
    tets = kuhn_tets(n)
    q0 = idx.astype(np.float64)
    q = jitter_block(idx, n, frac, rng)
    X0 = mapping(q0)
    X = mapping(q)
    s0 = signed_volumes6(X0, tets)
    s = signed_volumes6(X, tets)
    if not np.all(np.sign(s0) == np.sign(s)) or np.any(s == 0):
        raise ValueError(f"{name}: jitter {frac} inverted a tetrahedron")
    return Body(name, np.ascontiguousarray(X, dtype=np.float64),
                np.ascontiguousarray(tets, dtype=np.int32), exact_volume, box)


def box_body(name, size, centre, n, frac, rng):
    size = np.asarray(size, dtype=np.float64)
    centre = np.asarray(centre, dtype=np.float64)
    lo = centre - 0.5 * size
    h = size / np.asarray(n, dtype=np.float64)

    def mapping(q):
        X = lo + q * h
        # keep the far faces exactly on the box bounds
        for e in range(3):
            X[q[:, e] == n[e], e] = lo[e] + size[e]
        return X

    vol = float(np.prod(size))
    return _make_body(name, n, frac, rng, mapping, exact_volume=vol,
                      box=(tuple(lo), tuple(lo + size)))


def tilted_plate(name, size, centre, angle_deg, n, frac, rng):
    size = np.asarray(size, dtype=np.float64)
    centre = np.asarray(centre, dtype=np.float64)
    h = size / np.asarray(n, dtype=np.float64)
    a = math.radians(angle_deg)
    R = np.array([[math.cos(a), -math.sin(a), 0.0],
                  [math.sin(a), math.cos(a), 0.0],
                  [0.0, 0.0, 1.0]])

    def mapping(q):
        local = q * h - 0.5 * size
        return centre + local @ R.T

    return _make_body(name, n, frac, rng, mapping, exact_volume=float(np.prod(size)))


def shell_sector(name, axis_xy, r_mid, thick, arc_deg, z_lo, width, n, frac, rng):
    """Cylindrical shell sector with axis parallel to z; the arc is centred on
    the +y direction.  n = (arc, thickness, axial) hexahedra."""
    arc = math.radians(arc_deg)
    cx, cy = axis_xy

    def mapping(q):
        th = math.pi / 2 - arc / 2 + arc * q[:, 0] / n[0]
        r = r_mid - thick / 2 + thick * q[:, 1] / n[1]
        z = z_lo + width * q[:, 2] / n[2]
        return np.stack([cx + r * np.cos(th), cy + r * np.sin(th), z], axis=1)

    return _make_body(name, n, frac, rng, mapping)


def merge_bodies(bodies):
    Xs, Ts, offs_v, offs_t = [], [], [0], [0]
    base = 0
    for b in bodies:
        Xs.append(b.X)
        Ts.append(b.tets.astype(np.int64) + base)
        base += b.X.shape[0]
        offs_v.append(base)
        offs_t.append(offs_t[-1] + b.tets.shape[0])
    X = np.ascontiguousarray(np.concatenate(Xs), dtype=np.float64)
    T = np.ascontiguousarray(np.concatenate(Ts).astype(np.int32))
    return X, T, np.array(offs_v, dtype=np.int64), np.array(offs_t, dtype=np.int64)


# ----------------------------------------------------------------------------
# Fields
# ----------------------------------------------------------------------------

def fourier_modes(n_modes: int, kmax: int, seed: int, n_comp: int = 3):
    """Per component: integer wave vectors k in {-kmax..kmax}^3 \\ {0} and
    phases in [0, 2pi).  Returns (k: (n_comp, n_modes, 3) int, phi: (n_comp, n_modes))."""
    rng = np.random.default_rng(seed)
    k = np.zeros((n_comp, n_modes, 3), dtype=np.int64)
    for c in range(n_comp):
        for m in range(n_modes):
            while True:
                kk = rng.integers(-kmax, kmax + 1, size=3)
                if np.any(kk != 0):
                    break
            k[c, m] = kk
    phi = rng.uniform(0.0, 2.0 * math.pi, size=(n_comp, n_modes))
    return k, phi


def fourier_field(k: np.ndarray, phi: np.ndarray, xs, ys, zs, device=None, dtype=None):
    """Sum over modes of sin(2 pi k.x + phi), amplitude 1, sampled on the
    tensor grid xs x ys x zs.  Returns shape (len(zs), len(ys), len(xs))
    (x fastest).  With `device` set, computes with torch on that device."""
    import torch
    dev = torch.device(device) if device is not None else torch.device("cpu")
    dt = dtype if dtype is not None else torch.float64
    xs = torch.as_tensor(np.asarray(xs, dtype=np.float64), device=dev)
    ys = torch.as_tensor(np.asarray(ys, dtype=np.float64), device=dev)
    zs = torch.as_tensor(np.asarray(zs, dtype=np.float64), device=dev)
    out = torch.zeros((zs.numel(), ys.numel(), xs.numel()), dtype=torch.float64, device=dev)
    two_pi = 2.0 * math.pi
    for m in range(k.shape[0]):
        ex = torch.polar(torch.ones_like(xs), two_pi * float(k[m, 0]) * xs)
        ey = torch.polar(torch.ones_like(ys), two_pi * float(k[m, 1]) * ys)
        ez = torch.polar(torch.ones_like(zs), two_pi * float(k[m, 2]) * zs)
        ez = ez * complex(math.cos(phi[m]), math.sin(phi[m]))
        for zi0 in range(0, zs.numel(), 64):
            zi1 = min(zs.numel(), zi0 + 64)
            slab = ez[zi0:zi1, None, None] * ey[None, :, None] * ex[None, None, :]
            out[zi0:zi1] += slab.imag
    return out.to(dt)


def gaussian_nodal(n_v: int, seed: int, n_comp: int = 3) -> np.ndarray:
    """N(0,1) nodal values, shape (n_comp, n_v)."""
    return np.random.default_rng(seed).standard_normal((n_comp, n_v))


def fd_directions(n_v: int, n_dir: int, seed: int) -> np.ndarray:
    """Seeded unit directions in R^(n_v x 3), shape (n_dir, n_v, 3)."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((n_dir, n_v, 3))
    d /= np.linalg.norm(d.reshape(n_dir, -1), axis=1)[:, None, None]
    return d


def bending_displacement(X0: np.ndarray, step: int, seed: int, x0=0.2, length=0.6,
                         amplitude=0.05, n_steps=32) -> np.ndarray:
    """Cantilever bending mode along x, y-displacement of tip amplitude
    `amplitude`, oscillating over `n_steps` with a seeded phase."""
    phase = np.random.default_rng(seed).uniform(0.0, 1.0)
    s = np.clip((X0[:, 0] - x0) / length, 0.0, 1.0)
    shape = s * s * (3.0 - s) / 2.0
    u = np.zeros_like(X0)
    u[:, 1] = amplitude * shape * math.sin(2.0 * math.pi * (step + phase) / n_steps)
    return u


# ----------------------------------------------------------------------------
# The five workloads
# ----------------------------------------------------------------------------

WORKLOAD_NAMES = {
    1: "beam144_grid32",
    2: "beam48k_grid128",
    3: "plate397k_grid256s",
    4: "beam200k_grid192_series32",
    5: "three_bodies4.5M_grid512x256x256s",
}


@dataclass
class Workload:
    cfg: int
    name: str
    faces: list                 # 3 arrays of face coordinates
    X: np.ndarray
    tets: np.ndarray
    body_vert_offsets: np.ndarray
    body_tet_offsets: np.ndarray
    bodies: list
    n_modes: int
    kmax: int
    extra: dict = field(default_factory=dict)

    @property
    def n_cells(self):
        return tuple(len(f) - 1 for f in self.faces)

    def modes(self):
        return fourier_modes(self.n_modes, self.kmax, 2000 + self.cfg)

    def f_s(self):
        return gaussian_nodal(self.X.shape[0], 3000 + self.cfg)

    def u_target(self):
        return gaussian_nodal(self.X.shape[0], 4000 + self.cfg)


def _shrink(size, n_full, n_small):
    """Same element size as the full body, fewer elements (smaller extent)."""
    return tuple(float(s) * a / b for s, a, b in zip(size, n_small, n_full))


def workload(cfg: int, small: bool = False) -> Workload:
    """Build workload `cfg` (1..5).  `small=True` keeps the element size and
    the grid of the full workload but shrinks each body to a few thousand
    tets (used where the oracle must finish in seconds)."""
    rng = np.random.default_rng(1000 + cfg)

    def sized(size, n_full, n_small):
        return (_shrink(size, n_full, n_small), n_small) if small else (size, n_full)

    if cfg == 1:
        faces = [uniform_faces(32)] * 3
        b = box_body("beam", (0.4, 0.1, 0.1), (0.5, 0.5, 0.5), (6, 2, 2), 0.10, rng)
        bodies, n_modes, kmax = [b], 8, 4
    elif cfg == 2:
        faces = [uniform_faces(128)] * 3
        size, n = sized((0.6, 0.1, 0.1), (66, 11, 11), (20, 4, 4))
        b = box_body("beam", size, (0.5, 0.5, 0.5), n, 0.20, rng)
        bodies, n_modes, kmax = [b], 32, 8
    elif cfg == 3:
        faces = [uniform_faces(256), stretched_faces(256, 4.0), uniform_faces(256)]
        size, n = sized((0.5, 0.02, 0.5), (115, 5, 115), (12, 5, 12))
        b = tilted_plate("plate", size, (0.5, 0.5, 0.5), 15.0, n, 0.10, rng)
        bodies, n_modes, kmax = [b], 8, 4
    elif cfg == 4:
        faces = [uniform_faces(192)] * 3
        size, n = sized((0.6, 0.1, 0.1), (103, 18, 18), (24, 5, 5))
        b = box_body("beam", size, (0.5, 0.5, 0.5), n, 0.10, rng)
        bodies, n_modes, kmax = [b], 8, 4
    elif cfg == 5:
        faces = [uniform_faces(512, 0.0, 2.0), stretched_faces(256, 4.0), uniform_faces(256)]
        sb, nb = sized((0.6, 0.1, 0.1), (228, 38, 38), (16, 4, 4))
        sp, npl = sized((0.5, 0.02, 0.5), (189, 7, 189), (12, 7, 12))
        arc, nsh = (90.0, (183, 8, 117)) if not small else (90.0 * 12 / 183, (12, 8, 8))
        width = 0.3 if not small else 0.3 * 8 / 117
        bodies = [
            box_body("beam", sb, (0.4, 0.5, 0.5), nb, 0.10, rng),
            tilted_plate("plate", sp, (1.05, 0.5, 0.5), 15.0, npl, 0.10, rng),
            shell_sector("shell", (1.65, 0.2), 0.3, 0.02, arc, 0.35, width, nsh, 0.10, rng),
        ]
        n_modes, kmax = 32, 8
    else:
        raise ValueError(f"unknown workload {cfg}")
    X, T, ov, ot = merge_bodies(bodies)
    return Workload(cfg, WORKLOAD_NAMES[cfg] + ("_small" if small else ""), faces, X, T,
                    ov, ot, bodies, n_modes, kmax)
