"""AddressSanitizer and UndefinedBehaviorSanitizer builds on the CPU: the
oracle's C code (gcc), and the library's host code (hipcc, sanitizers on the
host side only) driven through the entry points that need no GPU.  Any
report aborts the driver (no recovery), so a clean run is an exit code of 0
with no sanitizer output."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
REPO = os.path.dirname(HERE)
SAN_ENV = dict(os.environ, ASAN_OPTIONS="abort_on_error=1:detect_leaks=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, env=None, timeout=600):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    return r.returncode, r.stdout + r.stderr


def _clean(out):
    return "AddressSanitizer" not in out and "LeakSanitizer" not in out and "runtime error" not in out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_asan_and_ubsan(tmp_path):
    counts, edges = oracle.mc_table()
    table = tmp_path / "mc_table.bin"
    table.write_bytes(np.ascontiguousarray(counts, np.uint8).tobytes() +
                      np.ascontiguousarray(edges, np.int8).tobytes())
    exe = tmp_path / "oracle_driver"
    rc, out = _run(["gcc", "-std=c11", "-O1", "-g", "-fopenmp", "-ffp-contract=off",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                    "-o", str(exe), os.path.join(HERE, "sanitize", "oracle_driver.c"),
                    os.path.join(REPO, "oracle", "fvr_oracle.c"), "-lm"])
    assert rc == 0, out
    rc, out = _run([str(exe), str(table)], env=dict(SAN_ENV, OMP_NUM_THREADS="2"))
    print(out)
    assert rc == 0 and out.startswith("ok") and _clean(out), out


def _host_san_flags():
    # sanitizers on the host side of every translation unit only: the device
    # code is built as usual
    san = []
    for f in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all"):
        san += ["-Xarch_host", f]
    return ["-O1", "-g", "-fno-omit-frame-pointer"] + san


@pytest.mark.skipif(not os.path.exists("/opt/rocm/llvm/bin/clang"), reason="ROCm clang not found")
def test_host_runtime_under_asan_and_ubsan(tmp_path):
    """The library's host code (checks, tuning table, marching-cubes table
    generator, status strings, NULL handling) with AddressSanitizer,
    LeakSanitizer and UndefinedBehaviorSanitizer, driven by
    tests/sanitize/host_driver.c without a GPU."""
    import concurrent.futures

    from paper_1712_03084_amd import build as B
    flags = [f for f in B._flags() if f != "-O3"] + _host_san_flags()

    def compile_one(src):
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        cmd = [B.hipcc()] + flags + (["-x", "hip"] if src.endswith(".hip") else []) + \
            ["-c", os.path.join(B.CSRC, src), "-o", obj]
        rc, out = _run(cmd, timeout=900)
        assert rc == 0, out
        return obj

    with concurrent.futures.ThreadPoolExecutor(min(8, len(B.SOURCES))) as ex:
        objs = list(ex.map(compile_one, B.SOURCES))
    lib = str(tmp_path / "libfvr_san.so")
    rc, out = _run([B.hipcc(), "-shared", "-fPIC", f"--offload-arch={B.ARCH}", "-o", lib] + objs)
    assert rc == 0, out
    exe = str(tmp_path / "host_driver")
    rc, out = _run(["/opt/rocm/llvm/bin/clang", "-std=c11", "-O1", "-g", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-I", os.path.join(REPO, "include"), "-o", exe,
                    os.path.join(HERE, "sanitize", "host_driver.c"), "-L", str(tmp_path), "-lfvr_san",
                    "-Wl,-rpath," + str(tmp_path)])
    assert rc == 0, out
    rc, out = _run([exe], env=SAN_ENV, timeout=300)
    print(out)
    assert rc == 0 and out.startswith("ok") and _clean(out), out
