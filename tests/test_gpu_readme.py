"""The usage example of the README runs as written."""
import os
import re

import pytest
import torch

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_readme_example_runs():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    text = open(os.path.join(ROOT, "README.md")).read()
    block = re.search(r"## Use\s+```python\n(.*?)```", text, re.S).group(1)
    ns = {}
    exec(compile(block, "README.md", "exec"), ns)
    pT, gw, gp, y = ns["pT"], ns["gw"], ns["gp"], ns["y"]
    assert torch.isfinite(pT).all() and torch.isfinite(gw).all() and torch.isfinite(gp).all()
    assert abs(float(pT.sum()) - 1.0) < 1e-3 and float(y.min()) >= 0
