"""Build libibvt.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1810_13046_amd.build

Every translation unit under csrc/ is compiled to an object in _build/ and
linked into paper_1810_13046_amd/libibvt.so.  The library exports exactly the
functions declared in include/ibvt.h: a linker version script written from
the header's declarations keeps every other symbol local.
"""
from __future__ import annotations

import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libibvt.so")
SOURCES = ["scan.hip", "sort.hip", "assemble.hip", "matfree.hip", "assemble2d.hip", "unstructured.hip", "transpose.hip",
           "apply.hip", "grad.hip", "api.hip", "fsi.hip", "noalloc.hip"]
ARCH = "gfx950"
HEADER = os.path.join(os.path.dirname(HERE), "include", "ibvt.h")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # no packed-FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas",
]


def _hipcc():
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def _compile(src):
    obj = os.path.join(OUT, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc(), *HIPCC_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def declared_functions(header: str = HEADER) -> list:
    """Names of the functions the public header declares (a declaration
    starts a line with its return type: int, void or const char*)."""
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    pat = re.compile(r"^(?:int|void|const char\s*\*)\s*(\w+)\s*\(", re.M)
    return sorted(set(pat.findall(text)))


def _version_script() -> str:
    names = declared_functions()
    path = os.path.join(OUT, "exports.map")
    with open(path, "w") as fh:
        fh.write("{\n  global:\n")
        for n in names:
            fh.write(f"    {n};\n")
        fh.write("  local:\n    *;\n};\n")
    return path


def build(verbose: bool = True) -> str:
    os.makedirs(OUT, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), 8)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs,
           f"-Wl,--version-script={_version_script()}", "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
