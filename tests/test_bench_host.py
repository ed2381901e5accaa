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
    assert (a.gpus, a.workload, a.job) == (1, "precision", "all")
    assert a.steps >= 1 and a.warmup >= 0
    assert set(a.sections.split(",")) == {"batched", "precision", "serving"}


@pytest.mark.parametrize("job", ["all", "concurrent", "sequential", "dense"])
def test_job_choices(monkeypatch, job):
    monkeypatch.setattr(sys, "argv", ["bench.py", "--job", job])
    assert bench.parse().job == job


def test_unknown_job_rejected(monkeypatch):
    monkeypatch.setattr(sys, "argv", ["bench.py", "--job", "parallel"])
    with pytest.raises(SystemExit):
        bench.parse()


def test_profile_summary_matches_kernel_sources():
    # The summary records the hash of csrc/*.hip, *.h it was measured on;
    # the benchmark reports measured traffic only while the two agree.  The
    # region step kernel of the 8192^2 workload (radius 6, 4 bands) appears
    # under the variant the benchmark's autotuning chose.
    import glob
    import json
    sha = bench.kernel_source_digest()
    names = []
    for path in glob.glob(os.path.join(ROOT, "profiles", "*.md")):
        for block in open(path).read().split("```json")[1:]:
            data = json.loads(block.split("```")[0])
            if data.get("kernel_source_sha256") == sha:
                names += [k for k in data["per_launch_traffic"].get("dense", {})
                          if k.startswith("lse::step_fast_kernel<6, 4, false, float")]
    assert names, "profiles/ summary is stale for the current kernel sources"
    traffic, source = bench.measured_traffic(names[0], "dense")
    assert traffic > 0 and source.startswith("profiles/")


def test_checkerboard_state_is_fully_active():
    cb = bench.checkerboard(40, 50)
    assert cb.shape == (40, 50) and cb.dtype.name == "uint8"
    assert cb[0, 0] == 0 and cb[0, 8] == 1 and cb[8, 0] == 1 and cb[8, 8] == 0
    # every 8-row, 16-column window holds both values
    for y in range(0, 33, 4):
        for x in range(0, 35, 5):
            assert 0 < cb[y:y + 8, x:x + 16].sum() < 128


def test_profile_commands_are_single_counter_block_runs():
    # rocprofv3 does not split counters over passes: at most 8 SQ counters per run.
    for cmd in bench.PROFILE_COMMANDS:
        if "--pmc" in cmd:
            counters = cmd.split("--pmc")[1].split("--")[0].split()
            assert len([c for c in counters if c.startswith("SQ_")]) <= 8, cmd
