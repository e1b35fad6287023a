"""GPU: importing the binding first (before torch) leaves torch's device usable.

torch ships its own HIP runtime under the same soname as the system one; the
binding imports torch before it loads the library, so the runtime that serves
the process is torch's.  Checked in a fresh interpreter, where nothing has
imported torch yet.
"""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_binding_import_before_torch():
    code = ("import paper_2605_28525_amd.mpm as M\n"
            "import torch\n"
            "from paper_2605_28525_amd import workloads as wl\n"
            "sim = M.Simulation(wl.tiny_3d(n=48, ties=False))\n"
            "sim.step(2)\n"
            "rc, flags = sim.status()\n"
            "sim.close()\n"
            "assert rc == 0, flags\n"
            "print('ok', torch.cuda.device_count())\n")
    print("CASE binding import before torch", flush=True)
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().startswith("ok"), r.stdout
