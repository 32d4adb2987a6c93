"""The C ABI used from C++ alone (no Python binding, no PyTorch): the example
program runs a Taylor-Green vortex and checks its viscous decay against the
analytic rate and its mass conservation (Sec. III.B)."""
import os
import subprocess

import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu
EXE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2312_10318_amd", "examples", "taylor_green")


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_c_example_decay_and_mass(storage):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert os.path.exists(EXE), "the C-ABI example is not built (run __graft_entry__.build())"
    r = subprocess.run([EXE, "64", storage, "1000"], capture_output=True, text=True, timeout=120)
    say("case: C example %s: %s" % (storage, (r.stdout + r.stderr).strip()))
    assert r.returncode == 0, r.stdout + r.stderr
    assert "within bounds" in r.stdout
