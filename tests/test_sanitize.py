"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU): the
oracle (every routine, on closed-form and random graphs, through
tests/sanitize/oracle_driver.c) and the edge-file reader (gc_io.cpp, on
TSV and Matrix Market files, well formed and malformed, through
tests/sanitize/io_driver.cpp).  A sanitizer finding makes the driver exit
non-zero with its report."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all",
       "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1")


def _need(tool):
    if shutil.which(tool) is None:
        pytest.skip("%s not available" % tool)


def test_oracle_under_sanitizers(tmp_path):
    _need("gcc")
    exe = str(tmp_path / "oracle_driver")
    subprocess.check_call(["gcc"] + SAN + ["-pthread", "-o", exe,
                                           os.path.join(HERE, "oracle_driver.c"),
                                           os.path.join(ROOT, "oracle", "oracle.c")])
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr


def test_edge_reader_under_sanitizers(tmp_path):
    _need("g++")
    exe = str(tmp_path / "io_driver")
    subprocess.check_call(["g++"] + SAN + ["-std=c++17", "-pthread", "-I",
                                           os.path.join(ROOT, "include"), "-o", exe,
                                           os.path.join(HERE, "io_driver.cpp"),
                                           os.path.join(ROOT, "paper_1708_06866_amd", "csrc",
                                                        "gc_io.cpp")])
    rng = np.random.default_rng(3)
    pairs = rng.integers(1, 500, size=(20000, 2))
    files = {}
    # a TSV file large enough for several reader chunks, with comments,
    # blank lines and CRLF endings
    lines = ["# comment", ""]
    for i, (a, b) in enumerate(pairs):
        lines.append("%d\t%d\t1%s" % (a, b, "\r" if i % 7 == 0 else ""))
    files["ok.tsv"] = ("0", "\n".join(lines) + "\n")
    mm = ["%%MatrixMarket matrix coordinate pattern symmetric", "% comment",
          "600 600 %d" % len(pairs)] + ["%d %d" % (a, b) for a, b in pairs]
    files["ok.mtx"] = ("0", "\n".join(mm) + "\n")
    files["bad_line.tsv"] = ("-1", "1\t2\t1\n3\tx\t1\n")
    files["id_zero.tsv"] = ("-2", "1\t2\t1\n0\t3\t1\n")
    files["count.mtx"] = ("-1", "%%MatrixMarket matrix coordinate pattern general\n4 4 3\n1 2\n")
    files["range.mtx"] = ("-2", "%%MatrixMarket matrix coordinate pattern general\n4 4 1\n1 9\n")
    files["huge.tsv"] = ("-6", "1\t3000000000\t1\n")
    files["empty.tsv"] = ("0", "")
    args = []
    for name, (expect, text) in files.items():
        p = tmp_path / name
        p.write_text(text)
        args.append("%s:%s" % (expect, p))
    r = subprocess.run([exe] + args, capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
    # the pairs read back: 0-based ids, in file order
    blocks = {}
    cur = None
    for line in r.stdout.splitlines():
        if line.startswith("# "):
            cur = os.path.basename(line.split()[1])
            blocks[cur] = []
        else:
            blocks[cur].append(tuple(int(x) for x in line.split()))
    want = [(int(a) - 1, int(b) - 1) for a, b in pairs]
    assert blocks["ok.tsv"] == want
    assert blocks["ok.mtx"] == want
    assert blocks["empty.tsv"] == []
