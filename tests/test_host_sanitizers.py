"""The library's host code built with AddressSanitizer and
UndefinedBehaviorSanitizer (api.hip's host pass; the device code and the
other sources' objects are the regular build's), driven by
tests/host_checks.cpp on the CPU: argument checks, error reporting, handle
creation without a GPU and the autotuner cache parser on malformed files.
No GPU is used: any sanitizer report fails the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# host-only sanitizer flags: each -fsanitize option applies to the host pass
# of the HIP compile only (the GPU code is built as usual)
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-g"]
DRIVER_SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined",
              "-fno-omit-frame-pointer", "-g"]


def _clangxx():
    for cand in ("/opt/rocm/llvm/bin/clang++", shutil.which("amdclang++")):
        if cand and os.path.exists(cand):
            return cand
    pytest.skip("ROCm clang++ not found")


@pytest.mark.slow
def test_host_code_under_asan_and_ubsan(tmp_path):
    from paper_2112_01508_amd import build
    objs = [os.path.join(build.BUILD, os.path.splitext(s)[0] + ".o") for s in build.SOURCES]
    if not all(os.path.exists(o) for o in objs):
        build.build()
    san = tmp_path / "san"
    san.mkdir()
    api_o = str(san / "api.o")
    compile_cmd = [build.hipcc(), *build.HIPCC_FLAGS, *HOST_SAN, "-c",
                   os.path.join(build.CSRC, "api.hip"), "-o", api_o]
    subprocess.run(compile_cmd, check=True, capture_output=True)
    lib = str(san / "libp3msr_san.so")
    others = [o for o in objs if not o.endswith("api.o")]
    link_cmd = [build.hipcc(), "--offload-arch=" + build.ARCH, "-shared", "-fPIC", "-o", lib,
                api_o, *others]
    subprocess.run(link_cmd, check=True, capture_output=True)
    exe = str(san / "host_checks")
    driver_cmd = [_clangxx(), *DRIVER_SAN, "-std=c++17", "-I" + os.path.join(ROOT, "include"),
                  os.path.join(ROOT, "tests", "host_checks.cpp"), lib,
                  "-Wl,-rpath," + str(san), "-o", exe]
    subprocess.run(driver_cmd, check=True, capture_output=True)
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:exitcode=86"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    # no device for the HIP runtime to find, even on a machine with one
    env["HIP_VISIBLE_DEVICES"] = ""
    env["ROCR_VISIBLE_DEVICES"] = ""
    work = tmp_path / "files"
    work.mkdir()
    r = subprocess.run([exe, str(work)], env=env, capture_output=True, text=True, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "host checks passed" in out
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
