"""Command-line contract of bench.py that needs no GPU: a request for more
than one GPU exits with status 2 and says why, before touching the device;
the stage-kernel source hash that gates the reported traffic is stable and
covers the sources of the stage kernel."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_stage_source_hash_covers_the_stage_kernel():
    sys.path.insert(0, ROOT)
    import bench

    h = bench.stage_source_hash()
    assert len(h) == 16 and h == bench.stage_source_hash()
    csrc = os.path.join(ROOT, "paper_1710_09578_amd", "csrc")
    for f in bench.STAGE_SOURCES:
        assert os.path.exists(os.path.join(csrc, f)), f
    # every header the stage kernel's source includes from csrc is hashed
    text = open(os.path.join(csrc, "batch.hip")).read()
    local = {line.split('"')[1] for line in text.splitlines() if line.startswith('#include "')}
    assert local <= set(bench.STAGE_SOURCES) | {"runtime.h", "solve.h"}, local - set(bench.STAGE_SOURCES)
