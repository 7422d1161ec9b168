"""The library's host code under AddressSanitizer and UBSan, on the CPU, with the tuner's live timing on.

srbe_tune's live timing is switched off in the library: three processes that ran it
aborted with host heap corruption.  This test looks for the cause in the library's own
host code.  It builds srbe_api.hip host-only (hipcc --offload-host-only) with
``kLiveTiming`` set to true in a copy, links it against host stubs of the HIP runtime,
rocBLAS/rocSOLVER and the kernel launchers (``host_harness/hip_stub.cpp``: "device"
memory is heap memory, graphs and events are heap objects freed on destroy), and runs
``host_harness/tuner_driver.cpp``.  The driver does what the aborted runs did, on two
handles: eager steps in both precisions, 24 srbe_tune calls (about 1,700 capture ->
instantiate -> replay -> destroy cycles on the handle's capture stream, shared events and
side stream), graph create/replay/destroy, phase timing on and off.  Under ASan and UBSan
every call must succeed, nothing may be reported, and every graph, executable graph,
event, stream and allocation must be released.  Skipped where hipcc is absent.
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not (os.path.exists(HIPCC) and shutil.which("g++")), reason="needs hipcc and g++")
def test_tuner_host_code_is_clean_under_asan(tmp_path):
    src = open(os.path.join(ROOT, "paper_2509_24742_amd", "csrc", "srbe_api.hip")).read()
    assert src.count("constexpr bool kLiveTiming = false;") == 1
    api = tmp_path / "api_live.hip"
    api.write_text(src.replace("constexpr bool kLiveTiming = false;", "constexpr bool kLiveTiming = true;"))
    csrc = os.path.join(ROOT, "paper_2509_24742_amd", "csrc")
    inc = os.path.join(ROOT, "include")
    harness = os.path.join(ROOT, "tests", "host_harness")
    hip = [HIPCC, "-x", "hip", "--offload-host-only", "-O1", "-g", "-std=c++17", "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined", "-fno-omit-frame-pointer", "-I" + inc, "-I" + csrc, "-w"]
    env = dict(os.environ, TMPDIR=str(tmp_path))
    subprocess.run(hip + ["-c", str(api), "-o", str(tmp_path / "api.o")], check=True, env=env)
    subprocess.run(hip + ["-c", os.path.join(harness, "hip_stub.cpp"), "-o", str(tmp_path / "stub.o")], check=True,
                   env=env)
    # the host-only object references its (absent) device code blob: give it an empty one
    nm = subprocess.run(["nm", "-u", str(tmp_path / "api.o")], check=True, capture_output=True, text=True).stdout
    blobs = sorted({w for w in nm.split() if w.startswith("__hip_fatbin_")})
    (tmp_path / "blob.cpp").write_text("".join(f'extern "C" {{ char {b}[16]; }}\n' for b in blobs))
    san = ["-fsanitize=address", "-fsanitize=undefined"]
    gxx = ["g++", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer", "-I" + inc] + san
    subprocess.run(gxx + ["-c", os.path.join(harness, "tuner_driver.cpp"), "-o", str(tmp_path / "driver.o")],
                   check=True)
    subprocess.run(gxx + ["-c", str(tmp_path / "blob.cpp"), "-o", str(tmp_path / "blob.o")], check=True)
    exe = str(tmp_path / "tunecheck")
    subprocess.run(["/opt/rocm/llvm/bin/clang++"] + san + [str(tmp_path / f) for f in
                                                          ("driver.o", "api.o", "stub.o", "blob.o")] + ["-o", exe],
                   check=True)
    run = subprocess.run([exe], capture_output=True, text=True, timeout=600,
                         env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
                                  UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1"))
    print(run.stdout[-600:])
    assert run.returncode == 0, run.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in run.stderr and "runtime error" not in run.stderr, run.stderr[-4000:]
    last = run.stdout.strip().splitlines()[-1]
    assert last.startswith("24 tune calls") and last.endswith("graphs 0 execs 0 events 0 streams 0 allocations 0")
