"""Host-side pieces of bench.py: the code digest that ties a committed
counter table to the kernel sources it was measured on."""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def test_code_only_drops_comments_and_keeps_literals():
    src = ('const char* s = "a // b /* c */";  // trailing\n'
           "char q = '/'; /* block\n spanning */ int x = 1;\n\n   int y;")
    assert bench._code_only(src) == "const char* s = \"a // b /* c */\"; char q = '/'; int x = 1; int y;"


def _write_tree(root, body):
    d = os.path.join(root, "paper_2507_02420_amd", "csrc")
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "k.hpp"), "w") as f:
        f.write(body)


def test_digest_ignores_comments_but_not_code(tmp_path, monkeypatch):
    a, b, c = (str(tmp_path / n) for n in "abc")
    _write_tree(a, "int f(int x) { return 2 * x; }  // doubles\n")
    _write_tree(b, "/* doubles x */\nint f(int x) {\n    return 2 * x;\n}\n")
    _write_tree(c, "int f(int x) { return 3 * x; }  // doubles\n")
    digests = []
    for root in (a, b, c):
        monkeypatch.setattr(bench, "ROOT", root)
        digests.append(bench.kernel_source_digest())
    assert digests[0] == digests[1]
    assert digests[0] != digests[2]
