"""Host logic of bench.py (no GPU): the one-GPU contract, the FLOP model and
the rule that the traffic figure is reported only for the kernel source it
was measured on."""
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


def test_flop_model_counts_each_term():
    b = _bench()
    zero = dict(n_pairs=0, n_atoms=0, n_torsions=0, depth_sum=0)
    assert b.flops_per_eval(zero, True) == 40 and b.flops_per_eval(zero, False) == 40
    for key, g, e in (("n_pairs", 62, 36), ("n_atoms", 129, 84), ("depth_sum", 33, 18), ("n_torsions", 38, 22)):
        one = dict(zero, **{key: 1})
        assert b.flops_per_eval(one, True) - 40 == g and b.flops_per_eval(one, False) - 40 == e
    # linear in every count
    info = dict(n_pairs=400, n_atoms=32, n_torsions=7, depth_sum=90)
    assert b.flops_per_eval(info, True) == 40 + 62 * 400 + 129 * 32 + 38 * 7 + 33 * 90


def test_traffic_is_reported_only_for_the_profiled_source(tmp_path):
    b = _bench()
    src = tmp_path / "kernels.hip"
    src.write_text("// kernel source\n")
    h = hashlib.sha256(src.read_bytes()).hexdigest()
    prof = tmp_path / "profile.md"
    prof.write_text(f"# summary\n\ntraffic_kernel_sha256: {h}\ntraffic_bytes_per_launch: 1449129700\n")
    assert b.measured_traffic(str(prof), str(src)) == 1449129700.0
    src.write_text("// kernel source, changed\n")
    assert b.measured_traffic(str(prof), str(src)) is None
    assert b.measured_traffic(str(tmp_path / "missing.md"), str(src)) is None
