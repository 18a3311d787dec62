"""The workload generator's command line: a 3D, a planar and an
unstructured workload are built, described and saved without pickles."""
import subprocess
import sys

import numpy as np

import workloads as wl


def _run(*args):
    r = subprocess.run([sys.executable, "-m", "workloads", *args], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    return r.stdout


def test_cli_describes_and_saves(tmp_path):
    out = _run("--config", "1", "--save", str(tmp_path / "c1.npz"))
    assert "144 tets" in out
    d = np.load(tmp_path / "c1.npz")  # allow_pickle stays False
    W = wl.workload(1)
    assert np.array_equal(d["tets"], W.tets) and np.array_equal(d["X"], W.X)
    assert np.array_equal(d["faces_z"], W.faces[2])
    assert "triangles" in _run("--planar", "1")
    assert "fluid tets" in _run("--unstructured", "1")
