"""Build libacr.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_1712_08872_amd.build   (or build() from Python)
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libacr.so")
# (source, extra flags, object name): the accumulation kernel is built for
# two round widths
SOURCES = [("k_harith.hip", ["-DKCV=64"], "k_harith_64"), ("k_harith.hip", ["-DKCV=38"], "k_harith_38"),
           ("k_apply.hip", [], "k_apply"), ("k_vec.hip", [], "k_vec"), ("geometry.cpp", [], "geometry"),
           ("program.cpp", [], "program"), ("runtime.cpp", [], "runtime"), ("cr.cpp", [], "cr"), ("import.cpp", [], "import"), ("krylov.cpp", [], "krylov"), ("static_ws.cpp", [], "static_ws"),
           ("api.cpp", [], "api")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# extra compiler flags for tuning builds (e.g. ACR_HIPFLAGS="-DDENSE_WPE=5")
FLAGS += os.environ.get("ACR_HIPFLAGS", "").split()


def build(verbose=False, jobs=None):
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    procs = []
    for src, extra, name in SOURCES:
        obj = os.path.join(objdir, name + ".o")
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        cmd = [HIPCC] + FLAGS + extra + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    failed = []
    for src, p in procs:
        out = p.communicate()[0].decode(errors="replace")
        lines = [ln for ln in out.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
        if p.returncode != 0:
            failed.append((src, "\n".join(lines)))
        elif verbose and lines:
            print(f"[{src}]\n" + "\n".join(lines))
    if failed:
        msg = "\n".join(f"--- {s}\n{o}" for s, o in failed)
        raise RuntimeError("libacr build failed:\n" + msg)
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("libacr link failed:\n" + r.stdout.decode(errors="replace"))
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
