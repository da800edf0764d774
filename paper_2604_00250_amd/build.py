"""Build libprism.so (HIP kernels + C ABI) for gfx950, in-tree.

    python -m paper_2604_00250_amd.build      (or build() from Python)

Every HIP translation unit is compiled with packed-FP32 instructions turned
off (``-target-feature -packed-fp32-ops``): the kernels are written for
scalar FP32 issue.
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libprism.so")
# (source, object, extra flags): the fused pass is compiled once per fibre count K
# so that its 48 template variants build in parallel
SOURCES = ([("prism_kernels.hip", "prism_kernels.o", []), ("prism_persistent.hip", "prism_persistent.o", [])]
           + [("prism_pass_k.hip", f"prism_pass_k{k}.o", [f"-DPRISM_PASS_K={k}"]) for k in range(1, 7)]
           + [("prism_host.cpp", "prism_host.o", [])])
ARCH = "gfx950"


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libprism)")


def source_hash() -> str:
    """SHA-1 (12 hex digits) of the library's sources: the csrc files and the C header."""
    import hashlib
    h = hashlib.sha1()
    names = sorted(n for n in os.listdir(CSRC) if n.endswith((".hip", ".h", ".cpp")) and n != "microbench.hip")
    for n in names:
        h.update(n.encode())
        with open(os.path.join(CSRC, n), "rb") as f:
            h.update(f.read())
    with open(os.path.join(HERE, "..", "include", "prism.h"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:12]


def build(verbose: bool = False) -> str:
    objs = []
    procs = []
    flags = [f"-DPRISM_SOURCE_HASH=\"{source_hash()}\"",
             "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(HERE, "..", "include")]
    for src, obj_name, extra in SOURCES:
        obj = os.path.join(CSRC, obj_name)
        objs.append(obj)
        cmd = [hipcc()] + flags + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    for cmd, p in procs:
        out = p.communicate()[0].decode(errors="replace")
        # the host pass does not know the device-only feature name: drop that notice
        out = "\n".join(l for l in out.splitlines() if "not a recognized feature" not in l)
        if p.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{out}")
        if out.strip() and verbose:
            print(out)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    # roofline microbenchmarks (a separate small library; the product path never loads it)
    mb = os.path.join(HERE, "libprism_mb.so")
    cmd = [hipcc()] + flags + ["-shared", os.path.join(CSRC, "microbench.hip"), "-o", mb + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"microbenchmark build failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(mb + ".tmp", mb)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
