"""The FP64 oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, any report is fatal) and driven through every entry point by
tests/oracle_sanitize_driver.c on small lattices: no out-of-bounds access,
leak, use after free, signed overflow or other undefined behaviour, and the
amounts conserved along the way (no GPU)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_sanitize_driver")
    cmd = ["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fopenmp",
           "-ffp-contract=off", "-Wall", "-Wextra", "-Werror",
           os.path.join(HERE, "oracle_sanitize_driver.c"), os.path.join(ROOT, "oracle", "dsm_oracle.c"),
           "-lm", "-o", exe]
    subprocess.run(cmd, check=True, cwd=HERE)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "all checks passed" in r.stdout


def test_host_side_of_the_library_under_sanitizers(tmp_path):
    """The host code of libdsm.so (argument checks, buffer sizing, error
    strings, the NULL-handle paths of every entry point, the batch calls),
    built with AddressSanitizer and UndefinedBehaviorSanitizer on the host
    side only (the device code is the same gfx950 code as always) and driven
    by tests/host_sanitize_driver.c without a GPU: no report, including leaks."""
    import concurrent.futures

    from paper_2504_19941_amd import build as B

    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    clang = "/opt/rocm/llvm/bin/clang"
    if not os.path.exists(clang):
        pytest.skip("ROCm clang not available")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-g", "-Xarch_host", "-O1"]
    base = B.hipcc_command(out="unused")
    flags = [a for a in base[: base.index("-o")] if a not in ("-shared",)]
    objs = []

    def compile_one(src):
        obj = str(tmp_path / (src + ".o"))
        subprocess.run(flags + san + ["-c", os.path.join(B.CSRC, src), "-o", obj], check=True, cwd=B.PKG)
        return obj

    with concurrent.futures.ThreadPoolExecutor(max_workers=len(B.SOURCES)) as ex:
        objs = list(ex.map(compile_one, B.SOURCES))
    lib = str(tmp_path / "libdsm_san.so")
    subprocess.run(["hipcc", f"--offload-arch={B.ARCH}", "-shared", "-fPIC", *san, "-o", lib, *objs], check=True)
    exe = str(tmp_path / "host_sanitize_driver")
    subprocess.run([clang, "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-I", os.path.join(ROOT, "include"), os.path.join(HERE, "host_sanitize_driver.c"),
                    "-o", exe, lib, f"-Wl,-rpath,{tmp_path}", "-lm"], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "all checks passed" in r.stdout
