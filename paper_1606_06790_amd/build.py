"""Build libidmrg.so for gfx950 in-tree with hipcc (no torch types involved)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libidmrg.so")
SOURCES = ["api.cpp", "plan.cpp", "gemm.hip", "mix.hip", "lanczos.hip", "svd.hip", "bjsvd.hip"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-I" + SRC]


def build(verbose=False):
    """Compile every source and link the shared library; returns its path."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src.rsplit(".", 1)[0] + ".o")
        cmd = ["hipcc", "-c", os.path.join(SRC, src), "-o", obj] + FLAGS
        if src.endswith(".cpp"):
            cmd = ["hipcc", "-x", "hip", "-c", os.path.join(SRC, src), "-o", obj] + FLAGS
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    failed = False
    for src, pr in procs:
        out, _ = pr.communicate()
        text = out.decode(errors="replace")
        lines = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
        if pr.returncode != 0:
            failed = True
            sys.stderr.write(f"--- {src}\n" + "\n".join(lines) + "\n")
        elif verbose and lines:
            sys.stderr.write(f"--- {src}\n" + "\n".join(lines) + "\n")
    if failed:
        raise RuntimeError("hipcc compilation failed")
    tmp = OUT + ".tmp"
    subprocess.check_call(["hipcc", "-shared", "--offload-arch=gfx950", "-o", tmp] + objs)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
