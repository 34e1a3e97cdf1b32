"""Host logic of bench.py (no GPU): the one-GPU contract and the rule that the
traffic figure is reported only for the kernel source it was measured on (the
FLOP models are pinned by the oracle's op-counting build, test_oracle_opcount.py)."""
import hashlib
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused_before_any_gpu_work():
    env = {k: v for k, v in os.environ.items() if k not in ("WORLD_SIZE", "RANK", "LOCAL_RANK")}
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, env=env, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_traffic_is_reported_only_for_the_profiled_source(tmp_path):
    b = _bench()
    src = tmp_path / "kernels.hip"
    src.write_text("// kernel source\n")
    h = hashlib.sha256(src.read_bytes()).hexdigest()
    prof = tmp_path / "profile.md"
    prof.write_text(f"# summary\n\ntraffic_kernel_sha256: {h}\ntraffic_bytes_per_generation: 1449129700\n")
    assert b.measured_traffic(str(prof), str(src)) == 1449129700.0
    src.write_text("// kernel source, changed\n")
    assert b.measured_traffic(str(prof), str(src)) is None
    assert b.measured_traffic(str(tmp_path / "missing.md"), str(src)) is None
