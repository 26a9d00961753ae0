"""Structure of the compiled bin-window kernel (AMD assembly of this
library's own source, cross-compiled for gfx950 on the CPU).

The kernel's persistent loop fetches its next read in thread 0 and hands it to
the block through LDS between two barriers.  A skip path that ends in a branch
on the thread index (if (t == 0) ...; continue) lets the compiler thread that
branch across the loop's back edge: the other threads then re-enter the loop
at its barriers, an inner loop that thread 0 never joins, and the block spins
on the same slot for ever.  The test checks, for every instantiation, that the
first barrier after the fetch sits in the same loop as the fetch and that no
loop of depth 2 or more is headed by a barrier."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1711_01177_amd", "csrc")


def block_info(body, j):
    """Loop depth of the block whose label is body[j], and whether it heads a loop."""
    d = int(re.search(r"Depth=(\d+)", body[j]).group(1)) if "Depth=" in body[j] else 0
    head = "Loop Header" in body[j]
    k = j + 1
    while k < len(body) and body[k].strip().startswith(";"):
        m = re.search(r"Loop Header: Depth=(\d+)", body[k])
        if m:
            d, head = int(m.group(1)), True
        k += 1
    return d, head


def check_persistent_loops(asm, kernel):
    lines = asm.splitlines()
    starts = [i for i, l in enumerate(lines) if re.match(rf"^_Z\S*{kernel}\S*:", l)]
    assert starts, f"no {kernel} in the assembly"
    ends = starts[1:] + [len(lines)]
    for a, b in zip(starts, ends):
        body = lines[a:b]
        name = body[0].split(":")[0]
        labels = [j for j, l in enumerate(body) if l.startswith(".LBB")]

        def block_of(k):
            return max(j for j in labels if j <= k)

        fetch = next(k for k, l in enumerate(body) if "global_atomic_add" in l)
        bar = next(k for k in range(fetch, len(body)) if "s_barrier" in body[k])
        assert block_info(body, block_of(fetch))[0] == 1, name
        assert block_info(body, block_of(bar))[0] == 1, f"{name}: barrier in an inner loop"
        for j in labels:
            d, head = block_info(body, j)
            if not head or d < 2:
                continue
            k = j + 1
            while k < len(body) and not body[k].startswith(".LBB"):
                assert "s_barrier" not in body[k], f"{name}: {body[j].split(':')[0]} loops on a barrier"
                k += 1


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not installed")
def test_window_kernel_loop_has_one_entry(tmp_path):
    out = tmp_path / "window.s"
    subprocess.check_call(
        ["hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature",
         "-Xclang", "-packed-fp32-ops", f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}",
         "--cuda-device-only", "-S", "-o", str(out), os.path.join(CSRC, "grim_window.hip")],
        stderr=subprocess.DEVNULL)
    check_persistent_loops(out.read_text(), "window_kernel")
