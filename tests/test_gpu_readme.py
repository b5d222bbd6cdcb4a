"""The Python example in the README runs as written (every shot converges)."""
import os
import re

import pytest

from oracle import OK

from _gpu import log, torch_cuda

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_readme_example_runs():
    torch_cuda()
    with open(os.path.join(ROOT, "README.md")) as f:
        blocks = re.findall(r"```python\n(.*?)```", f.read(), re.S)
    assert blocks, "the README has a Python example"
    log("README example")
    ns = {}
    exec(compile(blocks[0], "README.md", "exec"), ns)
    res = ns["res"]
    assert res.statuses == [OK] * len(res.statuses)
    assert max(res.relres) <= 1e-9
