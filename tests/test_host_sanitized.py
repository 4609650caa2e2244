"""The library's host code under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only).

The host sources are compiled with the sanitizers on their host side only
(-Xarch_host; the device code and the kernels are built as usual) and
linked with the kernel objects of the normal build into a separate library;
tests/sanitize/host_checks.cpp drives it: argument validation, the geometry
and level tables of several hundred decompositions (through the memory
plan, which builds every table and counts every array without a device),
the weight-file parser on malformed files, and the status strings.  Any
sanitizer report fails the run (UBSan halts on the first error)."""

import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, " ".join(cmd) + "\n" + r.stdout[-4000:] + r.stderr[-4000:]
    return r


def test_host_code_under_sanitizers(tmp_path):
    import torch
    from paper_2009_07965_amd import build as B
    objdir = os.path.join(B.HERE, "_build")
    kernels = [os.path.join(objdir, s.replace(".", "_") + ".o") for s in B.SOURCES if s.endswith(".hip")]
    if not all(os.path.exists(o) for o in kernels):
        B.build()
    cc = B.hipcc()
    host = []
    for src in ("api.cpp", "cnn.cpp"):
        obj = str(tmp_path / (src + ".o"))
        run([cc, "-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", *SAN,
             "-Wno-unused-command-line-argument", "-c", os.path.join(B.CSRC, src), "-o", obj])
        host.append(obj)
    lib = str(tmp_path / "librmrcm_san.so")
    run([cc, "--offload-arch=gfx950", "-shared", "-fPIC", "-shared-libasan", *SAN, *host, *kernels, "-o", lib])
    clang = os.path.join(os.path.dirname(os.path.realpath(cc)), "..", "llvm", "bin", "clang++")
    if not os.path.exists(clang):
        clang = "/opt/rocm/llvm/bin/clang++"
    rt = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                        text=True).stdout.strip()
    if not os.path.isabs(rt):
        rt = subprocess.run([clang, "--print-runtime-dir"], capture_output=True, text=True).stdout.strip()
    else:
        rt = os.path.dirname(rt)
    exe = str(tmp_path / "host_checks")
    run([clang, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
         "-shared-libasan", "-I", os.path.join(ROOT, "include"),
         os.path.join(ROOT, "tests", "sanitize", "host_checks.cpp"), lib,
         "-Wl,-rpath," + str(tmp_path), "-Wl,-rpath," + rt, "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    gpu = "gpu" if torch.cuda.is_available() else "cpu"
    r = subprocess.run([exe, str(tmp_path), gpu], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout[-2000:])
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    assert " 0 failures" in r.stdout
