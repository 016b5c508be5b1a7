"""GPU: the package works when it is imported before torch.

The library links the HIP runtime; torch carries its own copy.  The package
imports torch before loading the library so that the process holds one
runtime.  This runs in a fresh process that imports the package first (no
torch import of its own), creates the n = 1024, k = 3 handle (where two
runtimes made creation fail) and applies the operator."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

REPO = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CODE = """
import paper_1705_09907_amd as H
import numpy as np
from workloads import kappa_lognormal
S = H.Solver(1024, 3, kappa_lognormal(1024, 2.0, 3))
import torch
x = torch.ones(S.num_dofs(), dtype=torch.float64, device="cuda")
y = S.apply(3, x)
torch.cuda.synchronize()
assert bool(torch.isfinite(y).all())
S.close()
print("ok")
"""


def test_package_imported_before_torch():
    print("case import order", flush=True)
    r = subprocess.run([sys.executable, "-c", CODE], cwd=REPO, capture_output=True, text=True, timeout=240)
    assert r.returncode == 0 and "ok" in r.stdout, r.stderr[-3000:]
