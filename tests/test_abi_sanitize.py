"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only).

Every source of the library is compiled for gfx950 with the sanitizers on
the host side only (device code is built as usual; nothing here launches a
kernel), and linked
with tests/abi_sanitize_driver.cpp, which drives every validation and error
path of include/sca.h: valid and invalid parameter points on every route,
NULL contexts and servers, option checks, device errors, the per-thread
error message.  The run must report no sanitizer finding and print OK.
"""
import concurrent.futures
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")

# sanitizers for the host side of every translation unit only
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host",
       "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=all"]


def _gpu_present() -> bool:
    return os.path.exists("/dev/kfd") and bool(glob.glob("/dev/dri/renderD*"))


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_abi_paths_under_asan_ubsan(tmp_path):
    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_2311_04435_amd", "csrc",
                                         "*.hip")) +
                  glob.glob(os.path.join(ROOT, "paper_2311_04435_amd", "csrc",
                                         "*.cpp")))
    common = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
              "--offload-arch=gfx950", "-Xclang", "-target-feature",
              "-Xclang", "-packed-fp32-ops",
              "-I", os.path.join(ROOT, "include")] + SAN

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        r = subprocess.run([HIPCC, *common, "-x", "hip", "-c", src, "-o", obj],
                           capture_output=True, text=True)
        return obj, r

    with concurrent.futures.ThreadPoolExecutor(max_workers=8) as ex:
        built = list(ex.map(compile_one, srcs))
    objs = []
    for obj, r in built:
        assert r.returncode == 0, r.stderr[-2000:]
        objs.append(obj)
    drv = os.path.join(ROOT, "tests", "abi_sanitize_driver.cpp")
    exe = str(tmp_path / "abi_sanitize")
    r = subprocess.run([HIPCC, *common, "-x", "hip", drv, "-x", "none", *objs,
                        "-o", exe, "-L/opt/rocm/lib",
                        "-Wl,-rpath,/opt/rocm/lib",
                        "-lrocprofiler-sdk-roctx"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ)
    # the HIP runtime's own allocations are not this code's; leaks are not
    # what this checks
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    args = [exe] + (["--no-gpu"] if not _gpu_present() else [])
    r = subprocess.run(args, capture_output=True, text=True, env=env,
                       timeout=300)
    report = r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in report, report[-4000:]
    assert "runtime error:" not in report, report[-4000:]
    assert r.returncode == 0 and "OK" in r.stdout, report[-4000:]
