"""Build step: compiles the HIP library libstrassen.so for gfx950, in-tree.

    python -m paper_1605_01078_amd.build

Every HIP translation unit is compiled with packed-FP32 instruction selection disabled
(-Xclang -target-feature -Xclang -packed-fp32-ops); the host pass prints a harmless warning
that it does not know that feature.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libstrassen.so")
BLAS_LIB = os.path.join(HERE, "libstrassen_blas.so")
SOURCES = ["kernels_fp64.hip", "fused_fp64.hip", "classical_fp64.hip", "kernels_bf16.hip", "kernels_batched.hip", "kernels_mlp.hip",
           "probe_rates.hip", "noalloc.hip", "kernels_lu.hip", "lu.cpp", "cholesky.cpp",
           "tables.cpp", "api.cpp", "batched.cpp", "selector.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-result",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-ffp-contract=off", "-munsafe-fp-atomics"]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every source to an object (in parallel) and link libstrassen.so."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs, objs = [], []
    for src in sources():
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        cmd = [HIPCC] + FLAGS + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
        if len(procs) >= jobs:
            _wait(procs.pop(0), verbose)
    for p in procs:
        _wait(p, verbose)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    # the drop-in BLAS (dgemm_, cblas_dgemm) on top of it, found beside it at run time
    blas_obj = os.path.join(objdir, "blas_dgemm.cpp.o")
    cmd = [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, "blas_dgemm.cpp"), "-o", blas_obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    _wait(("blas_dgemm.cpp", subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)),
          verbose)
    tmp = BLAS_LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, blas_obj, "-L" + HERE,
           "-lstrassen", "-Wl,-rpath,$ORIGIN"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, BLAS_LIB)
    return LIB


def _wait(item, verbose):
    src, p = item
    out, _ = p.communicate()
    text = out.decode(errors="replace")
    noise = "is not a recognized feature for this target"
    shown = "\n".join(l for l in text.splitlines() if noise not in l)
    if p.returncode != 0:
        sys.stderr.write(shown + "\n")
        raise RuntimeError(f"hipcc failed on {src}")
    if verbose and shown.strip():
        print(shown, flush=True)


if __name__ == "__main__":
    print(build(verbose=True))
