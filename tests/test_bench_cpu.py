"""CPU checks of bench.py's command-line contract: more than one GPU is refused with a
message (the path is single-GPU), and without a GPU the bench stops instead of running
anything on the CPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ph = pytest.importorskip("paper_2210_07667_amd")


def run_bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=300,
                          cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = run_bench("--gpus", "2")
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""          # no JSON line


def test_no_gpu_means_no_bench_line():
    if ph.device_count() > 0:
        pytest.skip("a GPU is present: this checks the CPU-only case")
    r = run_bench("--steps", "1", "--warmup", "0")
    assert r.returncode != 0
    assert "needs a GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_kernel_tuner_contract(tmp_path):
    """tune_kernels.py lists its variants, the committed kernel_tuning.inc holds one of them,
    and `run` refuses (exit 2) when the variant libraries have not been built."""
    import re
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tune_kernels.py"), "list"],
                       stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=120)
    assert r.returncode == 0
    import json
    listed = [json.loads(line.split(" ", 1)[1]) for line in r.stdout.strip().splitlines()]
    assert len(listed) == 8 and listed[0] == {"PHIKS_DL_BK": 8, "PHIKS_DL_MIN_WAVES": 4,
                                              "PHIKS_DL_MIN_WAVES_LC": 4}
    inc = open(os.path.join(ROOT, "paper_2210_07667_amd", "csrc", "kernel_tuning.inc")).read()
    chosen = {k: int(v) for k, v in re.findall(r"#define (PHIKS_\w+) (\d+)", inc)}
    assert chosen in listed
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tune_kernels.py"), "run",
                        str(tmp_path)], stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                       text=True, timeout=120)
    assert r.returncode == 2 and "missing" in r.stderr
