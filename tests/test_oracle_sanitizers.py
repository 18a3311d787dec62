"""The oracle's C parts under AddressSanitizer and UndefinedBehaviorSanitizer
(host code only, on the CPU).  Each of the three libraries (3D, planar,
unstructured) is rebuilt with both sanitizers into a temporary directory,
and a child process, with the sanitizer runtime preloaded, runs the oracle
on small workloads through them: assembly with both multiplier bases, the
transfers, and the reverse mode's shape terms (the pair kernel called with
fields).  Any report aborts the child; the test checks that it ran to the
end."""
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOURCES = {"_o1.so": "o1.c", "_o2.so": "o2.c", "_o3.so": "o3.c"}

CHILD = textwrap.dedent("""
    import os, sys
    root, libdir = sys.argv[1], sys.argv[2]
    sys.path.insert(0, root)
    import numpy as np
    import oracle
    from oracle import plane, unstructured
    for mod, name in ((oracle, "_o1.so"), (plane, "_o2.so"), (unstructured, "_o3.so")):
        mod._LIB = os.path.join(libdir, name)
        mod._lib = None
    import workloads as wl

    rng = np.random.default_rng(3)
    W = wl.workload(1)
    oracle.assemble(W.faces, W.X, W.tets, dual=True)
    cpl = oracle.assemble(W.faces, W.X, W.tets)
    u_f = [rng.standard_normal(oracle.n_fluid(W.faces, d)) for d in range(3)]
    us = oracle.transfer_velocity(cpl, u_f, mass="consistent")
    ff = oracle.transfer_force(cpl, rng.standard_normal((3, W.X.shape[0])))
    g = oracle.velocity_vjp(cpl, u_f, rng.standard_normal(np.shape(us)), mass="lumped")
    print("3d", cpl.B[0].nnz, flush=True)

    P = wl.plane.workload2(1)
    c2 = plane.assemble(P.faces, P.X, P.tris)
    print("planar", c2.B[0].nnz, flush=True)

    U = wl.unstructured.workload_u(1)
    c3 = unstructured.assemble(U.Xf, U.tets_f, U.X, U.tets)
    print("unstructured", c3.B[0].nnz if hasattr(c3.B, "__getitem__") else c3.B.nnz, flush=True)
    maps = open("/proc/self/maps").read()
    assert "libasan" in maps, "the sanitizer runtime is not loaded"
    for name in ("_o1.so", "_o2.so", "_o3.so"):
        assert os.path.join(libdir, name) in maps, name
    print("sanitized oracle run complete", flush=True)
""")


def _runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True,
                          text=True).stdout.strip()
    return path if path and os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_c_under_address_and_undefined_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("the AddressSanitizer runtime is not installed")
    for lib, src in SOURCES.items():
        subprocess.check_call(
            ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all", "-fopenmp", "-fPIC", "-shared", "-std=gnu11", "-o",
             str(tmp_path / lib), os.path.join(ROOT, "oracle", src), "-lm"])
    env = dict(os.environ)
    env["LD_PRELOAD"] = asan
    # the interpreter itself is not instrumented: leave its allocations alone
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["OMP_NUM_THREADS"] = "4"
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT, str(tmp_path)], env=env,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "sanitized oracle run complete" in r.stdout, r.stdout[-2000:]
