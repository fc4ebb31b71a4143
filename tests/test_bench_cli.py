"""The benchmark's command-line contract that needs no GPU: more than one GPU
is refused with a message (the path runs on one GPU; instances shard without
exchange), before anything touches a device."""
from __future__ import annotations

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    line = [l for l in r.stdout.splitlines() if l.startswith("{")][-1]
    msg = json.loads(line)["error"]
    assert "one GPU" in msg
