"""A tuner ended by SIGTERM restores the DVFS knob it set (the default action
of SIGTERM ends a process without running atexit): a child process registers
a recording backend, sets a clock limit through a measurement (which writes
the state file), then receives SIGTERM from itself after the GPU work has
finished.  The backend must have restored the knob and the state file must
be gone.  No device setting is touched (the backend only records)."""
import os
import signal
import subprocess
import sys
import textwrap

import pytest
import torch

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = textwrap.dedent("""
    import os, signal, sys
    sys.path.insert(0, {root!r})
    import torch
    import paper_2211_07260_amd as gt
    log = open({log!r}, "a", buffering=1)
    gt.set_dvfs_backend(lambda dev, kind, value: log.write("apply %d %d\\n" % (kind, value)) and 0,
                        lambda dev: log.write("restore\\n") and 0)
    gt.init(0, gt.INIT_ALLOW_DVFS)
    buf = torch.empty(1 << 22, dtype=torch.float32, device=torch.device("cuda:0"))
    gt.measure_load(gt.LOAD_COPY, buf, gt.clock(gt.CLOCK_SCLK_MHZ, 1600), window_s=0.05, discard_s=0.01)
    torch.cuda.synchronize()
    log.write("state files %d\\n" % len([f for f in os.listdir({tmp!r}) if f.startswith("greentune-dvfs-")]))
    os.kill(os.getpid(), signal.SIGTERM)
    log.write("not reached\\n")
""")


def test_sigterm_restores_knob(tmp_path):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    log = tmp_path / "child.log"
    code = CHILD.format(root=ROOT, log=str(log), tmp=str(tmp_path))
    env = dict(os.environ, TMPDIR=str(tmp_path))
    print("case: child process sets a clock limit, then SIGTERM", flush=True)
    p = subprocess.run([sys.executable, "-c", code], env=env, timeout=120, capture_output=True, text=True)
    assert p.returncode == -signal.SIGTERM, (p.returncode, p.stderr[-2000:])
    lines = log.read_text().split("\n")
    assert lines[:3] == ["apply %d 1600" % 1, "state files 1", "restore"], lines
    assert "not reached" not in lines
    assert not list(tmp_path.glob("greentune-dvfs-*.state"))
