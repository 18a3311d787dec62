"""Seeded synthetic two-dimensional workloads: P1 triangle meshes in a
stretched rectilinear 2D grid, shaped like the paper's 2D experiments
(Section 4):

* Turek–Hron-like: channel 3 x 0.41, a disk of radius 0.05 centred at
  (0.2, 0.2) and an elastic tail 0.35 x 0.02 whose right bottom corner is at
  (0.6, 0.19), in grids of 576x96 up to 4608x762 points clustered around the
  structure, with triangle counts close to the paper's refinement table
  (about 500, 1200, 3300, 15000 and 44000 triangles);
* inertia test: channel 2 x 0.2 centred at y = 0, a plate of length 1 and
  thickness 0.012 meshed with spacing 0.001 (24000 triangles), grid of
  2048x129 points.

The paper's meshes are not available: the disk is a structured square mesh
mapped onto the disk by the elliptical square-to-disk map,
the tail and the plate are structured rectangles; two triangles per quad
with checkerboard diagonals and seeded node jitter that keeps boundary nodes
on the boundary.  Grid points are the cell faces.

Nothing in this module computes any part of the transfer.
Seeds for workload w: mesh 1100+w, fluid field 2100+w, solid force 3100+w,
target 4100+w, finite-difference directions 5100+w.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = ["clustered_faces", "quad_tris", "signed_areas2", "Body2", "Workload2", "workload2",
           "WORKLOADS_2D", "fourier_modes2", "fourier_field2", "gaussian_nodal2",
           "fd_directions2", "rect_body", "disk_body", "merge_bodies2"]


def clustered_faces(n_pts: int, lo: float, hi: float, a: float, b: float, ratio: float,
                    width: float) -> np.ndarray:
    """n_pts face coordinates on [lo, hi], finest and nearly uniform on
    [a, b], the spacing growing smoothly to `ratio` times the finest beyond
    about `width` outside it (inverse CDF of a point density)."""
    x = np.linspace(lo, hi, 400001)
    dist = np.maximum(0.0, np.maximum(a - x, x - b))
    rho = 1.0 / ratio + (1.0 - 1.0 / ratio) * np.exp(-(dist / width) ** 2)
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (rho[1:] + rho[:-1]) * np.diff(x))])
    cdf /= cdf[-1]
    f = np.interp(np.linspace(0.0, 1.0, n_pts), cdf, x)
    f[0], f[-1] = lo, hi
    assert np.all(np.diff(f) > 0)
    return f


def quad_tris(nx: int, ny: int) -> np.ndarray:
    """Two counter-clockwise triangles per quad of an nx x ny block (vertex
    ids i + (nx+1) j), diagonals alternating in a checkerboard.  int32."""
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    i, j = i.ravel(), j.ravel()
    v00 = i + (nx + 1) * j
    v10, v01 = v00 + 1, v00 + nx + 1
    v11 = v01 + 1
    flip = (((i + j) % 2) == 1)[:, None]
    t1 = np.where(flip, np.stack([v00, v10, v01], 1), np.stack([v00, v10, v11], 1))
    t2 = np.where(flip, np.stack([v10, v11, v01], 1), np.stack([v00, v11, v01], 1))
    return np.stack([t1, t2], 1).reshape(-1, 3).astype(np.int32)


def signed_areas2(X: np.ndarray, tris: np.ndarray) -> np.ndarray:
    """2x signed areas; used only to reject inverted meshes."""
    a = X[tris[:, 1]] - X[tris[:, 0]]
    b = X[tris[:, 2]] - X[tris[:, 0]]
    return a[:, 0] * b[:, 1] - a[:, 1] * b[:, 0]


def _block_params(nx, ny, frac, rng):
    j, i = np.meshgrid(np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    q = np.stack([i.ravel(), j.ravel()], axis=1).astype(np.float64)
    d = rng.uniform(-frac, frac, size=q.shape)
    d[(q[:, 0] == 0) | (q[:, 0] == nx), 0] = 0.0
    d[(q[:, 1] == 0) | (q[:, 1] == ny), 1] = 0.0
    return q, q + d


@dataclass
class Body2:
    name: str
    X: np.ndarray          # (n_v, 2) float64
    tris: np.ndarray       # (n_t, 3) int32
    exact_area: float | None = None
    box: tuple | None = None


def _make_body(name, nx, ny, frac, rng, mapping, exact_area=None, box=None):
    tris = quad_tris(nx, ny)
    q0, q = _block_params(nx, ny, frac, rng)
    X0, X = mapping(q0), mapping(q)
    s0, s = signed_areas2(X0, tris), signed_areas2(X, tris)
    if not np.all(np.sign(s0) == np.sign(s)) or np.any(s == 0):
        raise ValueError(f"{name}: jitter {frac} inverted a triangle")
    return Body2(name, np.ascontiguousarray(X, dtype=np.float64),
                 np.ascontiguousarray(tris, dtype=np.int32), exact_area, box)


def rect_body(name, lo, hi, nx, ny, frac, rng):
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    n = np.array([nx, ny], dtype=np.float64)

    def mapping(q):
        X = lo + q * (hi - lo) / n
        X[q[:, 0] == nx, 0] = hi[0]
        X[q[:, 1] == ny, 1] = hi[1]
        return X

    area = float(np.prod(hi - lo))
    return _make_body(name, nx, ny, frac, rng, mapping, exact_area=area,
                      box=(tuple(lo), tuple(hi)))


def disk_body(name, centre, radius, nsq, frac, rng):
    """Structured nsq x nsq square mapped onto the disk by the elliptical
    square-to-disk map x = u sqrt(1 - v^2/2), y = v sqrt(1 - u^2/2)
    (boundary nodes stay on the circle)."""
    c = np.asarray(centre, dtype=np.float64)

    def mapping(q):
        u = 2.0 * q[:, 0] / nsq - 1.0
        v = 2.0 * q[:, 1] / nsq - 1.0
        x = u * np.sqrt(1.0 - 0.5 * v * v)
        y = v * np.sqrt(1.0 - 0.5 * u * u)
        return c + radius * np.stack([x, y], axis=1)

    return _make_body(name, nsq, nsq, frac, rng, mapping)


def merge_bodies2(bodies):
    Xs, Ts, ov, ot = [], [], [0], [0]
    base = 0
    for b in bodies:
        Xs.append(b.X)
        Ts.append(b.tris.astype(np.int64) + base)
        base += b.X.shape[0]
        ov.append(base)
        ot.append(ot[-1] + b.tris.shape[0])
    return (np.ascontiguousarray(np.concatenate(Xs), dtype=np.float64),
            np.ascontiguousarray(np.concatenate(Ts).astype(np.int32)),
            np.array(ov, dtype=np.int64), np.array(ot, dtype=np.int64))


# ----------------------------------------------------------------------------
# Fields
# ----------------------------------------------------------------------------

def fourier_modes2(n_modes: int, kmax: int, seed: int, n_comp: int = 2):
    """Per component: wave vectors k in {-kmax..kmax}^2 \\ {0} and phases.
    Returns (k: (n_comp, n_modes, 2) int, phi: (n_comp, n_modes))."""
    rng = np.random.default_rng(seed)
    k = np.zeros((n_comp, n_modes, 2), dtype=np.int64)
    for c in range(n_comp):
        for m in range(n_modes):
            while True:
                kk = rng.integers(-kmax, kmax + 1, size=2)
                if np.any(kk != 0):
                    break
            k[c, m] = kk
    phi = rng.uniform(0.0, 2.0 * math.pi, size=(n_comp, n_modes))
    return k, phi


def fourier_field2(k, phi, xs, ys, scale=(1.0, 1.0)) -> np.ndarray:
    """Σ_m sin(2π (k_x x / L_x + k_y y / L_y) + φ_m) on the tensor grid
    xs x ys, shape (len(ys), len(xs)), x fastest."""
    xs = np.asarray(xs, dtype=np.float64)
    ys = np.asarray(ys, dtype=np.float64)
    out = np.zeros((ys.size, xs.size))
    for m in range(k.shape[0]):
        ax = 2.0 * math.pi * k[m, 0] / scale[0] * xs
        ay = 2.0 * math.pi * k[m, 1] / scale[1] * ys
        out += np.sin(ay[:, None] + ax[None, :] + phi[m])
    return out


def gaussian_nodal2(n_v: int, seed: int, n_comp: int = 2) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal((n_comp, n_v))


def fd_directions2(n_v: int, n_dir: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((n_dir, n_v, 2))
    d /= np.linalg.norm(d.reshape(n_dir, -1), axis=1)[:, None, None]
    return d


# ----------------------------------------------------------------------------
# Workloads
# ----------------------------------------------------------------------------

# Turek–Hron levels: grid points (x, y), disk squares per side, tail quads.
_TH = {
    "coarse": ((576, 96), 11, (44, 3)),
    "medium": ((769, 128), 18, (70, 4)),
    "fine": ((1153, 193), 30, (117, 7)),
    "finest": ((2304, 384), 64, (250, 14)),
    "reference": ((4608, 762), 108, (427, 24)),
}

WORKLOADS_2D = {1: "th_coarse", 2: "th_medium", 3: "th_fine", 4: "th_finest",
                5: "th_reference", 6: "inertia_plate24k"}


@dataclass
class Workload2:
    key: int
    name: str
    faces: list             # 2 arrays of face coordinates
    X: np.ndarray           # (n_v, 2)
    tris: np.ndarray        # (n_t, 3)
    body_vert_offsets: np.ndarray
    body_tri_offsets: np.ndarray
    bodies: list
    n_modes: int
    kmax: int
    extra: dict = field(default_factory=dict)

    @property
    def n_cells(self):
        return tuple(len(f) - 1 for f in self.faces)

    @property
    def extent(self):
        return tuple(float(f[-1] - f[0]) for f in self.faces)

    def modes(self):
        return fourier_modes2(self.n_modes, self.kmax, 2100 + self.key)

    def f_s(self):
        return gaussian_nodal2(self.X.shape[0], 3100 + self.key)

    def u_target(self):
        return gaussian_nodal2(self.X.shape[0], 4100 + self.key)


def workload2(key: int) -> Workload2:
    """Build 2D workload `key` (1..6, names in WORKLOADS_2D)."""
    rng = np.random.default_rng(1100 + key)
    if 1 <= key <= 5:
        level = WORKLOADS_2D[key][3:]
        (px, py), nsq, (bx, by) = _TH[level]
        faces = [clustered_faces(px, 0.0, 3.0, 0.1, 0.7, 4.0, 0.3),
                 clustered_faces(py, 0.0, 0.41, 0.13, 0.27, 4.0, 0.05)]
        x0 = 0.2 + math.sqrt(0.05 ** 2 - 0.01 ** 2)     # tail corners on the circle
        bodies = [disk_body("disk", (0.2, 0.2), 0.05, nsq, 0.10, rng),
                  rect_body("tail", (x0, 0.19), (0.6, 0.21), bx, by, 0.15, rng)]
        n_modes, kmax = 16, 6
    elif key == 6:
        faces = [np.linspace(0.0, 2.0, 2048), np.linspace(-0.1, 0.1, 129)]
        bodies = [rect_body("plate", (0.5, -0.006), (1.5, 0.006), 1000, 12, 0.15, rng)]
        n_modes, kmax = 16, 6
    else:
        raise ValueError(f"unknown 2D workload {key}")
    X, T, ov, ot = merge_bodies2(bodies)
    return Workload2(key, WORKLOADS_2D[key], faces, X, T, ov, ot, bodies, n_modes, kmax)
