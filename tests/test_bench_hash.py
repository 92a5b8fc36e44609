"""The key under which bench.py trusts the committed counter summaries."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_code_text_ignores_comments_and_spacing():
    a = "int f(int x) {  // one\n  return x + 1; /* two\n lines */ }\n"
    b = "int f(int x) {\n\treturn x + 1;\n}  // other words\n"
    assert bench.code_text(a) == bench.code_text(b)


def test_code_text_sees_code_changes():
    assert bench.code_text("return x + 1;") != bench.code_text("return x + 2;")


def test_committed_traffic_summaries_match_the_current_kernels():
    # both counter summaries were taken on the kernels in the tree
    for spl in (1, 2):
        assert bench.measured_traffic(8192 * 8192, spl) is not None, spl
