"""bench.py's command line on the host: a run on more than one GPU is refused
before anything touches a device, and the committed counter summaries name the
step kernels' current source."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_counter_summaries_match_the_step_source():
    import bench
    h = bench.kernel_source_hash()
    for name in ("step2_f32_4096_valu.json", "step2_f32_4096_traffic.json"):
        with open(os.path.join(ROOT, "profiles", name)) as fh:
            assert json.load(fh)["kernel_hash"] == h, name
