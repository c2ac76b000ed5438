"""MC_LOG: the library's log lines on stderr (CPU; a validate-only context).

Level 1 writes every failure an entry point returns, with its message; unset or
0 writes nothing; the level is read when a context is created.  The emulated
host runtime checks the higher levels' lines (context, launches, admission).
"""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import numpy as np
import paper_2104_10073_amd as Z
from paper_2104_10073_amd import workloads as W
t = W.mixed_batch(5, dim_range=(1, 4), log10_samples=(3.0, 4.0), gen_seed=1)
t["dim"][2] = 13
with Z.Context(device=0, flags=Z.MC_VALIDATE_ONLY) as c:
    try:
        c.submit(t, Z.PREC_FP32)
    except Z.McError as e:
        print("status", e.status)
"""


def _run(level):
    env = dict(os.environ)
    env.pop("MC_LOG", None)
    if level is not None:
        env["MC_LOG"] = str(level)
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
    proc = subprocess.run([sys.executable, "-c", SCRIPT], capture_output=True, text=True, env=env, cwd=ROOT,
                          timeout=300)
    assert proc.returncode == 0, proc.stderr[-2000:]
    assert "status -3" in proc.stdout
    return [ln for ln in proc.stderr.splitlines() if ln.startswith("[zmc] ")]


def test_log_levels():
    assert _run(None) == []
    assert _run(0) == []
    lines = _run(1)
    assert len(lines) == 1, lines
    assert lines[0].startswith("[zmc] error -3: function 2:"), lines
