"""OBK_LOG: the library's log level (read once from the environment).

Level 0 (unset) prints nothing; level 1 prints every failed call with its
status name and message; a successful call prints nothing at level 1.  Each
case runs in a child process, since the level is read once per process.
"""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import ctypes, sys
sys.path.insert(0, {root!r})
import numpy as np
import paper_2401_00672_amd as obk
L = obk.lib()
# a failing host call: negative size
rc = L.obk_first_fit_host(-1, None, None, None, None, None)
assert rc == -1, rc
# a succeeding host call: first-fit on two conflicting rows
cptr = np.array([0, 0, 1], dtype=np.int64)
cidx = np.array([0], dtype=np.int32)
active = np.ones(2, dtype=np.uint8)
group = np.zeros(2, dtype=np.int32)
ng = ctypes.c_int32(0)
rc = L.obk_first_fit_host(2, cptr.ctypes.data, cidx.ctypes.data, active.ctypes.data, group.ctypes.data,
                          ctypes.byref(ng))
assert rc == 0 and ng.value == 2, (rc, ng.value)
print("child done", flush=True)
"""


def _run(level):
    env = dict(os.environ)
    env.pop("OBK_LOG", None)
    if level is not None:
        env["OBK_LOG"] = str(level)
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT)], capture_output=True, text=True,
                       timeout=300, env=env)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "child done" in r.stdout
    return [l for l in r.stderr.splitlines() if l.startswith("[obk]")]


def test_log_unset_is_silent():
    assert _run(None) == []


def test_log_level_1_reports_each_failure_once():
    lines = _run(1)
    assert lines == ["[obk] error OBK_E_ARG: bad argument"], lines


def test_log_level_0_is_silent():
    assert _run(0) == []
