"""bench.py measures one GPU: asked for more (by --gpus or by a multi-rank launch) it exits
with a message before touching any device.  CPU only."""
import os
import subprocess
import sys

import pytest

from tests.conftest import ROOT


@pytest.mark.parametrize("args,env", [(["--gpus", "2"], {}), (["--gpus", "8"], {}),
                                      ([], {"WORLD_SIZE": "2", "RANK": "0", "LOCAL_RANK": "0"})])
def test_more_than_one_gpu_exits_with_a_message(args, env):
    e = dict(os.environ, **env)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                       env=e, timeout=300, cwd=ROOT)
    assert r.returncode == 2, (r.returncode, r.stderr[-500:])
    assert "one GPU only" in r.stderr
    assert r.stdout.strip() == ""          # no JSON line
