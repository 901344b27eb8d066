"""Host-only checks of bench.py's argument handling (no GPU is touched: every
case here is decided before the first HIP call)."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    env = dict(os.environ, HIP_VISIBLE_DEVICES="")
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True,
                          text=True, timeout=300, env=env)


@pytest.mark.parametrize("args", [["--steps", "21"], ["--steps", "0"], ["--warmup", "-1"]])
def test_out_of_range_step_counts_are_refused(args):
    r = _run(*args)
    assert r.returncode == 2, r.stderr
    assert "--steps must be in 1..20" in r.stderr


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def test_driver_command_passes_argument_checks():
    # the round-end command; without a GPU it must fail only at the device check
    r = _run("--gpus", "1", "--steps", "20", "--warmup", "5")
    if r.returncode == 0:
        return  # a GPU is present
    assert r.returncode == 1 and "needs a GPU" in r.stderr, r.stderr


@pytest.mark.parametrize("launch", ["per-step", "graph"])
def test_launch_modes_pass_argument_checks(launch):
    # every launch mode is accepted; without a GPU the run stops at the device check
    r = _run("--launch", launch, "--workload", "mixed_batch")
    if r.returncode == 0:
        return
    assert r.returncode == 1 and "needs a GPU" in r.stderr, r.stderr


def test_unknown_launch_mode_is_refused():
    r = _run("--launch", "stream")
    assert r.returncode == 2 and "invalid choice" in r.stderr
