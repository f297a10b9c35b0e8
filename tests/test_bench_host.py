"""Host-side checks of the benchmark script (no GPU): the one-GPU contract,
the committed counter summaries it reads, and its algorithmic byte counts."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_source_digest_is_stable_and_covers_the_kernels():
    a, b = bench.source_digest(), bench.source_digest()
    assert a == b and len(a) == 40


def test_committed_counter_lines_parse():
    # every "pmc:" line of the committed summaries is key=value pairs naming
    # a kernel and the source digest it was taken with
    n = 0
    for f in sorted(os.listdir(bench.PROFILE_DIR)):
        if not f.endswith(".md"):
            continue
        for line in open(os.path.join(bench.PROFILE_DIR, f)):
            if not line.startswith("pmc:"):
                continue
            kv = dict(t.split("=", 1) for t in line[4:].split() if "=" in t)
            assert "kernel" in kv and len(kv.get("source_sha1", "")) == 40, line
            for k, v in kv.items():
                if k not in ("kernel", "source_sha1"):
                    assert float(v) >= 0.0, (k, v)
            n += 1
    assert n > 0
    got = bench.committed_counters("collide", "0" * 40)
    assert got == {}  # figures of other sources are never used


def test_algorithmic_bytes_per_particle():
    # streaming: x, y, cx, cy read (16 B) and one code byte written (the
    # gather, which loads every particle anyway, stores the moved position)
    assert bench.ALGO_BYTES["stream"] == 4 * 4 + 1
    # collision pass: 28 B of state read and written, a code byte, and
    # 26 running FP64 sums per cell of 100 particles read and written
    assert abs(bench.ALGO_BYTES["collide"] - (28 + 28 + 1 + 2 * 26 * 8 / 100.0)) < 1e-9
