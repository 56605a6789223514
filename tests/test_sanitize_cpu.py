"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only, no device).

The C oracle is built with gcc and the sanitizers into a driver that runs every oracle function
on small ragged shapes with exactly sized heap operands (tests/sanitize/oracle_driver.c).  The
library's host sources are built with the sanitizers on their host pass only (the device
kernels are linked from the regular build, unsanitized and never launched) into a driver that
exercises every entry point whose work is host-side (tests/sanitize/host_driver.c).  A report of
either sanitizer (out-of-bounds access, use after free, leak, undefined behaviour) fails the
test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")


def _run(cmd, **kw):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-4000:]}"
    return r.stdout


def test_oracle_under_sanitizers(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_san")
    _run(["gcc", "-O1", "-g", "-fopenmp", "-ffp-contract=off", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-std=c11", "-Wall",
          os.path.join(HERE, "oracle_driver.c"), os.path.join(ROOT, "oracle", "oracle_gemm.c"),
          "-lm", "-o", exe])
    out = _run([exe], env=ENV, timeout=600)
    assert "oracle checks passed" in out and "ERROR" not in out


def test_library_host_code_under_sanitizers(tmp_path):
    from paper_1605_01078_amd import build as B
    rocm = "/opt/rocm"
    hipcc, clang = os.path.join(rocm, "bin", "hipcc"), os.path.join(rocm, "llvm", "bin", "clang")
    if not (os.path.exists(hipcc) and os.path.exists(clang)):
        pytest.skip("ROCm compilers not found")
    objdir = os.path.join(ROOT, "paper_1605_01078_amd", "_build")
    device = [os.path.join(objdir, s + ".o") for s in B.SOURCES if s.endswith(".hip")]
    if not all(os.path.exists(o) for o in device):
        pytest.skip("the library is not built (python -m paper_1605_01078_amd.build)")
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", f"--offload-arch={B.ARCH}"]
    for f in ("-fsanitize=address", "-fsanitize=undefined", "-fno-omit-frame-pointer",
              "-fno-sanitize-recover=undefined"):
        flags += ["-Xarch_host", f]   # host pass only
    procs, host = [], []
    for s in B.SOURCES:
        if s.endswith(".cpp"):
            obj = str(tmp_path / (s + ".o"))
            host.append(obj)
            procs.append(subprocess.Popen([hipcc] + flags + ["-c", os.path.join(B.CSRC, s), "-o", obj],
                                          stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
    for p in procs:
        out, _ = p.communicate()
        assert p.returncode == 0, out.decode(errors="replace")[-4000:]
    drv = str(tmp_path / "driver.o")
    _run([clang, "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-c",
          os.path.join(HERE, "host_driver.c"), "-o", drv])
    exe = str(tmp_path / "host_san")
    _run([clang + "++", "-fsanitize=address,undefined", drv] + host + device +
         [f"-L{rocm}/lib", "-lamdhip64", f"-Wl,-rpath,{rocm}/lib", "-o", exe])
    out = _run([exe], env=ENV, timeout=900)
    assert "host checks passed" in out and "ERROR" not in out
