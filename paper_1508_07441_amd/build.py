"""Build libwpcd.so for gfx950 with hipcc (in-tree)."""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = ["wpcd_api.hip", "wpcd_coupling.hip", "k_pair.hip", "k_p0.hip", "k_solve.hip",
       "k_mlp.hip", "wpcd_learn.hip", "k_model.hip", "k_reduce.hip"]
OUT = os.path.join(HERE, "libwpcd.so")
# Per-file flags.  The element kernels see only finite tables, so their
# min/max need no NaN quieting (without this flag every fmax/fmin of a value
# from memory or from another block costs an extra canonicalising max).
EXTRA = {"k_p0.hip": ["-fno-honor-nans"]}


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, jobs: int = 4) -> str:
    csrc = os.path.join(HERE, "csrc")
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    flags = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-result", "-I", os.path.join(HERE, "..", "include")]
    procs, objs = [], []
    for s in SRC:
        obj = os.path.join(objdir, s.replace(".hip", ".o"))
        objs.append(obj)
        cmd = [hipcc(), "-c", os.path.join(csrc, s), "-o", obj] + flags + EXTRA.get(s, [])
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((s, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for s, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        if p.returncode != 0:
            failed.append((s, text))
        elif verbose and text.strip():
            print(text)
    if failed:
        for s, text in failed:
            sys.stderr.write(f"--- {s}\n{text}\n")
        raise RuntimeError("hipcc failed: " + ", ".join(s for s, _ in failed))
    tmp = OUT + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
