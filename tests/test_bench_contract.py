"""bench.py runs on one GPU: asked for more it exits with a message before
touching a GPU, in every mode."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("mode", [[], ["--diffusion"], ["--strang"], ["--groups", "8"], ["--reshuffle"],
                                  ["--batch", "4"]])
def test_more_than_one_gpu_is_refused(mode):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", *mode],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr or "single-GPU" in r.stderr
