"""Host code under the sanitizers (CPU only, no GPU).

* The serving engine core (paper_2210_07667_amd/csrc/server_core.hpp: lanes, admission,
  workspace slots, worker / completer / submitter / waiter threads) driven by the fake
  executor of tests/host/server_core_check.cpp, built with g++ under the thread
  sanitizer and under the address and undefined-behaviour sanitizers.
* The library's host code -- planner, batched schedule and launch tables, capture fork
  plan, server policy -- built host-only (hipcc, no device code objects) with the address
  and undefined-behaviour sanitizers on the host side, driven by
  tests/host/batch_plan_check.cpp over the 512 problems of the batched workload.
* The run rule of the deferred plan-build uploads (csrc/stage_runs.hpp), driven by
  tests/host/stage_runs_check.cpp: joined copies stay inside one device allocation.
Each run must report no sanitizer error and pass its own checks."""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2210_07667_amd", "csrc")
HOST = os.path.join(ROOT, "tests", "host")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


def build_and_run(tmp_path, src, flags, env_extra):
    exe = str(tmp_path / "check")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", *flags, f"-I{CSRC}", src, "-o", exe,
                    "-lpthread"], check=True, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    env = dict(os.environ, **env_extra)
    r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True,
                       env=env, timeout=300)
    print(r.stdout[-4000:])
    return r


@pytest.mark.parametrize("kind", ["thread", "address+undefined"])
def test_server_core_under_sanitizer(tmp_path, kind):
    if kind == "thread":
        flags, env = ["-fsanitize=thread"], {"TSAN_OPTIONS": "halt_on_error=1 exitcode=66"}
    else:
        flags = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
        env = {"ASAN_OPTIONS": "halt_on_error=1 detect_leaks=1 exitcode=66"}
    r = build_and_run(tmp_path, os.path.join(HOST, "server_core_check.cpp"), flags, env)
    assert r.returncode == 0, r.stdout[-4000:]
    assert "server core check passed" in r.stdout
    assert "WARNING: ThreadSanitizer" not in r.stdout and "ERROR: AddressSanitizer" not in r.stdout


def test_staged_upload_runs_stay_in_one_allocation(tmp_path):
    r = build_and_run(tmp_path, os.path.join(HOST, "stage_runs_check.cpp"),
                      ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
                      {"ASAN_OPTIONS": "halt_on_error=1 exitcode=66"})
    assert r.returncode == 0, r.stdout[-4000:]
    assert "stage runs check passed" in r.stdout


HIPCC = "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="needs hipcc")
def test_library_host_code_under_address_and_ub_sanitizers(tmp_path):
    # problems file of the batched workload (see batch_plan_check.cpp)
    probs = workloads.config_batch()
    path = tmp_path / "problems.bin"
    with open(path, "wb") as f:
        f.write(struct.pack("<i", len(probs)))
        sizes = sorted({m for b in probs for m in b.n})
        for m in sizes:
            f.write(struct.pack("<i", m))
            f.write(np.ascontiguousarray(workloads.cheb_d2_dirichlet(m), dtype="<f8").tobytes())
        f.write(struct.pack("<i", 0))
        for b in probs:
            f.write(struct.pack("<i", len(b.n)))
            f.write(struct.pack(f"<{len(b.n)}i", *b.n))
            f.write(struct.pack("<d", b.tau))
    inc = os.path.join(ROOT, "include")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all"]
    objs = []
    steps = [
        [HIPCC, "--offload-arch=gfx950", "-fgpu-rdc", "--offload-host-only", "-O1", "-g",
         "-std=c++17", "-fPIC", *san, f"-I{inc}", "-c", os.path.join(CSRC, "phiks.hip"),
         "-o", str(tmp_path / "phiks.o")],
        ["/opt/rocm/llvm/bin/clang++", "-O1", "-g", "-std=c++17", "-fPIC",
         "-fsanitize=address,undefined", "-fno-sanitize-recover=all", f"-I{inc}", "-c",
         os.path.join(CSRC, "planner.cpp"), "-o", str(tmp_path / "planner.o")],
        ["/opt/rocm/llvm/bin/clang++", "-O1", "-g", "-std=c++17",
         "-fsanitize=address,undefined", "-fno-sanitize-recover=all", f"-I{inc}", "-c",
         os.path.join(HOST, "batch_plan_check.cpp"), "-o", str(tmp_path / "driver.o")],
        [HIPCC, "-fgpu-rdc", "--hip-link", "--offload-arch=gfx950", *san,
         str(tmp_path / "driver.o"), str(tmp_path / "phiks.o"), str(tmp_path / "planner.o"),
         "-lpthread", "-o", str(tmp_path / "check")],
    ]
    for cmd in steps:
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        assert r.returncode == 0, r.stdout[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="halt_on_error=1 detect_leaks=0 exitcode=66",
               UBSAN_OPTIONS="halt_on_error=1 print_stacktrace=1")
    r = subprocess.run([str(tmp_path / "check"), str(path)], stdout=subprocess.PIPE,
                       stderr=subprocess.STDOUT, text=True, env=env, timeout=600)
    print(r.stdout[-4000:])
    assert r.returncode == 0, r.stdout[-4000:]
    assert "batch / planner check passed" in r.stdout
    assert "runtime error" not in r.stdout and "ERROR: AddressSanitizer" not in r.stdout
