"""Host-side helpers of bench.py: the kernel-source hash that ties a committed
HBM-traffic profile to the code it was measured on."""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import bench  # noqa: E402

SRC = """// header comment
__global__ void k(int *a) {   /* block
comment */
    a[threadIdx.x] = 8;   // trailing
}
"""


def test_comment_and_whitespace_edits_keep_the_hash():
    h = bench._code_hash(SRC)
    assert bench._code_hash(SRC.replace("// trailing", "// another note")) == h
    assert bench._code_hash(SRC.replace("/* block\ncomment */", "")) == h
    assert bench._code_hash(SRC.replace("    a[", "\ta[")) == h


def test_code_edits_change_the_hash():
    h = bench._code_hash(SRC)
    assert bench._code_hash(SRC.replace("= 8", "= 9")) != h
    assert bench._code_hash(SRC.replace("threadIdx.x", "threadIdx.y")) != h

