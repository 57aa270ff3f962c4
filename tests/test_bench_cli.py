"""Host side of bench.py: the one-GPU guard, the byte counts the roofline is
priced with, and the counter summaries it reads (taken only while they match
the kernel source)."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_bytes_per_update_are_two_lattices_of_nineteen_values():
    b = _bench()
    for st, size in (("f64", 8), ("f32", 4), ("f16s", 2)):
        assert b.BYTES_PER_UPDATE[st] == 2 * 19 * size


def test_counter_summaries_are_used_only_for_the_current_kernel_source(tmp_path):
    from paper_1611_02445_amd.profiling import kernel_source_hash
    b = _bench()
    b.PROFILE_DIR = str(tmp_path)
    assert b.counter_traffic("step_f64_spheres256") is None
    d = {"kernel_source_hash": kernel_source_hash(), "hbm_bytes_per_launch": 123.0}
    with open(tmp_path / "counters_step_f64_spheres256.json", "w") as fh:
        json.dump(d, fh)
    assert b.counter_traffic("step_f64_spheres256") == 123.0
    d["kernel_source_hash"] = "0" * 16
    with open(tmp_path / "counters_step_f64_spheres256.json", "w") as fh:
        json.dump(d, fh)
    assert b.counter_traffic("step_f64_spheres256") is None

