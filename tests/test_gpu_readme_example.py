"""The README's Python example runs as written (on a GPU) and its results are
consistent: the survivor list holds exactly the pairs whose pass bit is set."""
import os
import re

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_readme_python_example():
    from tests.gpu_helpers import lib
    lib()  # the built library, loaded the way every GPU test loads it
    text = open(os.path.join(ROOT, "README.md")).read()
    blocks = re.findall(r"```python\n(.*?)```", text, flags=re.S)
    assert blocks, "README has no Python example"
    env = {}
    exec(compile(blocks[0], "README.md", "exec"), env)
    torch = env["torch"]
    torch.cuda.synchronize()
    grim = env["grim"]
    assert env["rc"] == grim.GRIM_OK
    n = int(env["n"])
    bits = env["bits"].cpu().numpy().view(np.uint32)
    n_pairs = env["batch"].n_pairs
    set_bits = int(np.unpackbits(bits.view(np.uint8), bitorder="little")[:n_pairs].sum())
    assert n == set_bits
    assert env["dist"].shape[0] >= n
