"""The bounds-checking build of the library (-DDSMC_BOUNDS_CHECK, built
beside the release library): on workloads that take every kernel of the path
no index check fails, and the results are bit-identical to the release
build's.  The checking build runs in a child process (one library per
process); the release build in this one."""
import json
import os
import subprocess
import sys

import pytest

from paper_2301_05985_amd import build as B
from tests import bounds_cases as C

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bounds_checked_build_is_clean_and_identical(gpu):
    assert os.path.exists(B.LIB_BOUNDS), "build the libraries first (python -m paper_2301_05985_amd.build)"
    print("[gpu case] bounds-checking build (child process)", flush=True)
    env = dict(os.environ, DSMC_HIP_LIB=B.LIB_BOUNDS)
    r = subprocess.run([sys.executable, "-m", "tests.bounds_cases"], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    checked = json.loads(r.stdout.strip().splitlines()[-1])
    for name, p, parts, steps, net in C.cases():
        print("[gpu case] release build: %s" % name, flush=True)
        got = checked[name]
        assert got["bounds_checked"] == 1, name
        assert got["status"] == 0, (name, got)
        assert got["bounds_violations"] == 0, (name, got)
        rel = C.run_case(name, p, parts, steps, net)
        assert rel["bounds_checked"] == 0, name
        assert rel["digest"] == got["digest"], name
