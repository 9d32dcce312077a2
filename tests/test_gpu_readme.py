"""The Python example of README.md runs as written (the documented API)."""
import os
import re

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_readme_python_example_runs():
    text = open(os.path.join(ROOT, "README.md")).read()
    blocks = re.findall(r"```python\n(.*?)```", text, flags=re.S)
    assert blocks, "README has no python example"
    ns = {}
    exec(compile(blocks[0], "README.md", "exec"), ns)  # raises if diagnostics find a NaN/Inf
    phi1, mu1 = ns["phi1"], ns["mu1"]
    assert phi1.shape[0] == 3 and mu1.shape[0] == 2
    assert np.isfinite(phi1).all() and np.isfinite(mu1).all()
    assert np.max(np.abs(phi1.sum(axis=0) - 1.0)) < 1e-12
