"""Host-side checks of the benchmark script (no GPU): the one-GPU guard, its
arguments, and that the committed rocprofv3 summary belongs to the kernel
sources in the tree (the benchmark takes its measured traffic from it)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _run(args, env=None):
    e = dict(os.environ)
    e.update(env or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          env=e, timeout=120)


@pytest.mark.parametrize("args,env", [(["--gpus", "2"], None), ([], {"WORLD_SIZE": "4"})])
def test_more_than_one_gpu_exits_with_a_message(args, env):
    r = _run(args, env)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_default_arguments(monkeypatch):
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    a = bench.parse()
    assert (a.gpus, a.workload, a.job) == (1, "large", "both")
    assert a.steps >= 1 and a.warmup >= 0
    assert set(a.sections.split(",")) == {"batched", "precision", "serving"}


@pytest.mark.parametrize("job", ["both", "concurrent", "sequential"])
def test_job_choices(monkeypatch, job):
    monkeypatch.setattr(sys, "argv", ["bench.py", "--job", job])
    assert bench.parse().job == job


def test_unknown_job_rejected(monkeypatch):
    monkeypatch.setattr(sys, "argv", ["bench.py", "--job", "parallel"])
    with pytest.raises(SystemExit):
        bench.parse()


def test_profile_summary_matches_kernel_sources():
    # The summary records the hash of csrc/*.hip, *.h it was measured on;
    # the benchmark reports measured traffic only while the two agree.
    name = "lse::step_fast_kernel<5, 4, false, float>"
    traffic, source = bench.measured_traffic(name)
    assert traffic is not None, "profiles/ summary is stale for the current kernel sources"
    assert traffic > 0 and source.startswith("profiles/")
