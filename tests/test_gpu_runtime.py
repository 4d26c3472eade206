"""The library and torch share one HIP runtime whatever the import order
(a second runtime in the process cannot open the device)."""
import subprocess
import sys
import os

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import ctypes, sys
from paper_2303_14119_amd import flashkin as fk     # the library first
import torch
assert torch.cuda.is_available()
from paper_2303_14119_amd import workloads as W
cfg = W.config(nx=16, nvx=16, nvy=64, length=1e-3, ey=-5e6, delta_max=2.5, a_max_ev=400.0)
t = torch.zeros(16 * 16 * 64, dtype=torch.float32, device="cuda")
with fk.Solver(cfg, "f32", stream=torch.cuda.current_stream().cuda_stream) as s:
    s.step(3)
    s.f_to_device(t.data_ptr(), t.numel() * 4)
    torch.cuda.synchronize()
    assert torch.isfinite(t).all().item()
print("ok")
"""


def test_library_loaded_before_torch():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    r = subprocess.run([sys.executable, "-c", SCRIPT], cwd=ROOT, capture_output=True, text=True, timeout=240)
    assert r.returncode == 0 and "ok" in r.stdout, r.stdout + r.stderr
