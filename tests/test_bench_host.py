"""Host-side parts of the benchmark (CPU): one GPU only, and the HBM traffic record of the roofline."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args, env=None):
    e = dict(os.environ)
    e.update(env or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, env=e)


def test_more_than_one_gpu_exits_with_a_message():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_launch_under_a_multi_rank_launcher_exits_with_a_message():
    r = _run(env={"WORLD_SIZE": "4"})
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_record_names_its_kernels():
    tj = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    assert set(tj["bytes_per_launch"]) >= {"render_fwd", "render_bwd"}
    assert tj["calibration"]["write_factor"] == 1.0 and 1.9 < tj["calibration"]["fetch_factor"] < 2.1
