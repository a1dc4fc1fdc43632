"""Host code under the sanitizers (CPU only, no GPU): the serving engine core
(paper_2210_07667_amd/csrc/server_core.hpp: lanes, admission, workspace slots, worker /
completer / submitter / waiter threads) driven by the fake executor of
tests/host/server_core_check.cpp, built with g++ under the thread sanitizer and under the
address and undefined-behaviour sanitizers; each run must report no error and pass its
own checks."""
import os
import shutil
import subprocess

import pytest

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
