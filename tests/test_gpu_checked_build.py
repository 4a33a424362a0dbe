"""The bounds-checked build (-DSPMVC_CHECK, libspmvc_check.so): the detector
reports an index out of range (spmvc_check_probe), and every kernel family
on every format then runs with no index out of range and gives the oracle's
results (tests/checked_build_cases.py, in a process of its own
because the binding holds one library per process)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CHECK_LIB = os.path.join(ROOT, "paper_1612_00530_amd", "libspmvc_check.so")

pytestmark = pytest.mark.gpu


def test_checked_build_reports_no_violation():
    if not os.path.exists(CHECK_LIB):
        pytest.skip("libspmvc_check.so is not built (the package build with check=True makes it)")
    env = dict(os.environ, SPMVC_LIBRARY=CHECK_LIB)
    r = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "tests", "checked_build_cases.py")],
                       capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout[-3000:], r.stderr[-3000:])
    assert r.returncode == 0
    assert "probe ok" in r.stdout and "violations 0" in r.stdout
