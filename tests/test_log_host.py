"""MILS_LOG_LEVEL: errors (level 1) and plan, workspace and tuning events
(level 2) go to stderr with a "[mils]" prefix; level 0 prints nothing.
Host-only contexts, no GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROBE = """
import sys
sys.path.insert(0, {root!r})
from paper_2409_08090_amd import mils
try:
    mils.plan_info(100, 0, 1e-9, "fp64")
except mils.MilsError:
    pass
"""


def _run(level):
    env = dict(os.environ)
    env["MILS_LOG_LEVEL"] = str(level)
    r = subprocess.run([sys.executable, "-c", PROBE.format(root=ROOT)], capture_output=True,
                       text=True, timeout=120, env=env)
    assert r.returncode == 0, r.stderr
    return r.stderr


def test_errors_are_logged_at_level_one():
    err = _run(1)
    assert "[mils] error" in err, err


def test_nothing_is_logged_at_level_zero():
    assert "[mils]" not in _run(0)
