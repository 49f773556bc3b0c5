"""CPU checks of bench.py's command line: asked for more than one GPU it exits
with a message before touching a device, and prints no result line."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 2, (r.returncode, r.stderr[-2000:])
    assert "one GPU" in r.stderr
    assert not any(line.startswith("{") for line in r.stdout.splitlines())
