"""Build a seeded synthetic workload and describe it (optionally save it).

  python -m workloads --config 5            # three bodies, 4.5M tets
  python -m workloads --config 3 --small    # the shrunk plate the oracle tests use
  python -m workloads --planar 1            # planar (triangles in a quad lattice)
  python -m workloads --unstructured 3      # tetrahedral fluid mesh + solid tets
  python -m workloads --config 2 --save beam.npz

--save writes the arrays with numpy.savez (no pickles): the fluid grid's
face coordinates per axis (faces_x, faces_y[, faces_z]) or the fluid mesh
(Xf, tets_f), the solid vertices X and elements (tets or tris)."""
import argparse
import sys
import time

import numpy as np

from . import gen, plane, unstructured


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(prog="python -m workloads", description=__doc__.splitlines()[0])
    g = ap.add_mutually_exclusive_group(required=True)
    g.add_argument("--config", type=int, choices=range(1, 6), help="3D grid workload 1..5")
    g.add_argument("--planar", type=int, help="planar workload key")
    g.add_argument("--unstructured", type=int, help="unstructured-background workload key")
    ap.add_argument("--small", action="store_true", help="shrunk bodies (3D configs only)")
    ap.add_argument("--save", help="write the arrays to this .npz file")
    a = ap.parse_args(argv)
    t0 = time.perf_counter()
    arrays = {}
    if a.config is not None:
        W = gen.workload(a.config, small=a.small)
        cells = "x".join(str(len(f) - 1) for f in W.faces)
        print(f"{W.name}: {W.tets.shape[0]:,} tets, {W.X.shape[0]:,} vertices, grid {cells} cells, "
              f"bodies {[b.name for b in W.bodies]}")
        arrays = dict(faces_x=W.faces[0], faces_y=W.faces[1], faces_z=W.faces[2], X=W.X,
                      tets=W.tets, body_tet_offsets=W.body_tet_offsets,
                      body_vert_offsets=W.body_vert_offsets)
    elif a.planar is not None:
        W = plane.workload2(a.planar)
        cells = "x".join(str(len(f) - 1) for f in W.faces)
        print(f"planar {a.planar}: {W.tris.shape[0]:,} triangles, {W.X.shape[0]:,} vertices, "
              f"grid {cells} cells")
        arrays = dict(faces_x=W.faces[0], faces_y=W.faces[1], X=W.X, tris=W.tris)
    else:
        W = unstructured.workload_u(a.unstructured)
        print(f"unstructured {a.unstructured}: {W.tets_f.shape[0]:,} fluid tets, "
              f"{W.Xf.shape[0]:,} fluid vertices; {W.tets.shape[0]:,} solid tets, "
              f"{W.X.shape[0]:,} solid vertices")
        arrays = dict(Xf=W.Xf, tets_f=W.tets_f, X=W.X, tets=W.tets)
    print(f"built in {time.perf_counter() - t0:.1f} s")
    if a.save:
        np.savez(a.save, **arrays)
        print(f"saved {a.save}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
