"""Seeded synthetic workloads with an unstructured fluid background: a P1
tetrahedral fluid mesh of a box whose interior nodes are warped and
jittered (no cell is axis-aligned and no lattice exists), with a P1 solid
beam inside, shaped like the structured 3D cases (element sizes of the two
meshes within a factor of two).

The fluid mesh: n^3 hexahedra of the box [0, 1]^3 split into six
tetrahedra each, interior nodes moved by a smooth warp (amplitude `amp`
fluid spacings, zero on the boundary) plus seeded jitter whose normal
component is zero on the box faces; the solid: a jittered box beam as in
workloads/gen.py.

Nothing in this module computes any part of the transfer.
Seeds for workload w: fluid mesh 1200+w, solid mesh 1300+w, fluid field
2200+w, solid force 3200+w.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .gen import _make_body, box_body

__all__ = ["warped_box", "WorkloadU", "workload_u", "WORKLOADS_U", "linear_fields"]

WORKLOADS_U = {1: "warped24k_beam192", 2: "warped384k_beam4.5k", 3: "warped5.3M_beam200k"}

_SIZES = {  # fluid hexes per side, beam size, beam hexes
    1: (16, (0.4, 0.1, 0.1), (8, 2, 2)),
    2: (40, (0.6, 0.1, 0.1), (30, 5, 5)),
    3: (96, (0.6, 0.1, 0.1), (103, 18, 18)),
}


def warped_box(name, n, frac, amp, rng):
    """The unit box as n^3 hexahedra, six tetrahedra each, interior nodes
    warped by amp·h·(sin πx sin πy sin πz)·(1, 1, 1)-rotated directions and
    jittered by frac·h."""
    h = 1.0 / n

    def mapping(q):
        x = q * h
        s = (np.sin(math.pi * x[:, 0]) * np.sin(math.pi * x[:, 1]) * np.sin(math.pi * x[:, 2]))
        w = np.stack([np.sin(2 * math.pi * x[:, 1]), np.sin(2 * math.pi * x[:, 2]),
                      np.sin(2 * math.pi * x[:, 0])], axis=1)
        X = x + amp * h * s[:, None] * w
        for e in range(3):
            X[q[:, e] == 0, e] = 0.0
            X[q[:, e] == n, e] = 1.0
        return X

    return _make_body(name, (n, n, n), frac, rng, mapping)


@dataclass
class WorkloadU:
    key: int
    name: str
    Xf: np.ndarray
    tets_f: np.ndarray
    X: np.ndarray
    tets: np.ndarray

    def f_s(self):
        return np.random.default_rng(3200 + self.key).standard_normal((3, self.X.shape[0]))

    def u_f(self):
        """Three smooth fluid nodal fields (n_vert_fluid each)."""
        rng = np.random.default_rng(2200 + self.key)
        out = []
        for d in range(3):
            k = rng.integers(-3, 4, size=(6, 3))
            ph = rng.uniform(0, 2 * math.pi, size=6)
            out.append(sum(np.sin(2 * math.pi * self.Xf @ k[m] + ph[m]) for m in range(6)))
        return np.stack(out)


def workload_u(key: int) -> WorkloadU:
    n, size, nb = _SIZES[key]
    fluid = warped_box("fluid", n, 0.15, 0.5, np.random.default_rng(1200 + key))
    beam = box_body("beam", size, (0.5, 0.5, 0.5), nb, 0.10, np.random.default_rng(1300 + key))
    return WorkloadU(key, WORKLOADS_U[key], fluid.X, fluid.tets, beam.X, beam.tets)


def linear_fields(X, coef):
    """Affine nodal values c0 + c·x at the points X (for reproduction tests)."""
    coef = np.asarray(coef, dtype=np.float64)
    return coef[0] + X @ coef[1:]
