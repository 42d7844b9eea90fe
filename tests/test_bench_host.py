"""Host-side pieces of bench.py: the hash that ties the committed HBM
counter files to the sweep's source code."""
import os
import shutil
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_code_only_drops_comments_and_blank_lines():
    src = "int a; // first\n\n/* a block\n   comment */ int b;   \n  // only a comment\nint c;\n"
    assert bench._code_only(src) == "int a;\n int b;\nint c;"


def test_kernel_hash_ignores_comments_not_code(tmp_path, monkeypatch):
    files = []
    for path in bench.KERNEL_SOURCES:
        dst = tmp_path / os.path.basename(path)
        shutil.copy(path, dst)
        files.append(str(dst))
    monkeypatch.setattr(bench, "KERNEL_SOURCES", files)
    h0 = bench.kernel_source_sha()
    with open(files[0], "a", encoding="utf-8") as f:
        f.write("\n// a comment added at the end\n/* and a block */\n")
    assert bench.kernel_source_sha() == h0
    with open(files[0], "a", encoding="utf-8") as f:
        f.write("static const int kAddedForTheTest = 1;\n")
    assert bench.kernel_source_sha() != h0

