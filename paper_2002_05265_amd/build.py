"""Build liblbm.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import pathlib
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

PKG = pathlib.Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
LIB_PATH = PKG / "liblbm.so"

HIP_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # contraction only inside one expression: the same source expression rounds the same way
    # in every kernel that inlines it (plain, batched and adjoint kernels stay bit-identical)
    "-ffp-contract=on",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and pathlib.Path(cand).exists():
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def build_library(verbose: bool = False) -> pathlib.Path:
    """Compile each HIP source to an object in parallel, then link liblbm.so."""
    srcs = sorted(CSRC.glob("*.hip"))
    obj_dir = PKG / "_build"
    obj_dir.mkdir(exist_ok=True)
    compile_flags = [f for f in HIP_FLAGS if f != "-shared"]
    inc = [f"-I{ROOT / 'include'}", f"-I{CSRC}"]
    cmds = [[hipcc(), *compile_flags, *inc, "-c", str(s), "-o", str(obj_dir / (s.stem + ".o"))]
            for s in srcs]
    if verbose:
        for c in cmds:
            print(" ".join(c), flush=True)
    with ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 1)) as ex:
        results = list(ex.map(lambda c: subprocess.run(c, capture_output=True, text=True), cmds))
    for c, res in zip(cmds, results):
        if res.returncode != 0:
            raise RuntimeError(f"hipcc failed ({res.returncode}) on {c[-3]}:\n{res.stderr[-4000:]}")
    tmp = LIB_PATH.with_name(LIB_PATH.name + ".tmp")
    link = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC",
            *[str(obj_dir / (s.stem + ".o")) for s in srcs], "-o", str(tmp)]
    if verbose:
        print(" ".join(link), flush=True)
    res = subprocess.run(link, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc link failed ({res.returncode}):\n{res.stderr[-4000:]}")
    tmp.replace(LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build_library(verbose=True))
