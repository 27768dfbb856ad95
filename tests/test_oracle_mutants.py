"""The oracle's pins catch plausible mistakes.  Each case plants one mistake
in a copy of ``oracle/oracle.c`` (a dropped term, a wrong threshold or index,
a missing liveness check, an off-by-one truss number), builds it with gcc,
and runs ``tests/test_oracle_pins.py`` against that build: the pins must
fail.  The planted code runs on the CPU only, in a child process."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

# (name, exact text in oracle.c, replacement)
MUTANTS = [
    ("duplicates kept",
     "if (i > 0 && key[i] == key[i - 1]) continue;", "if (0) continue;"),
    ("self-loops kept",
     "if (a == b) continue;", "if (0) continue;"),
    ("degree order not strict",
     "  return x > y;\n}", "  return 1;\n}"),
    ("count merge skips the head of N+(y)",
     "{\n      int32_t y = out[i];\n      int64_t a = ooff[x], ae = ooff[x + 1], b = ooff[y],",
     "{\n      int32_t y = out[i];\n      int64_t a = ooff[x], ae = ooff[x + 1], b = ooff[y] + 1,"),
    ("search misses the last element",
     "return (lo < end && nbr[lo] == y) ? lo : -1;",
     "return (lo + 1 < end && nbr[lo] == y) ? lo : -1;"),
    ("second edge of a triangle not required alive",
     "    if (alive && !alive[g->eid[j]]) continue;    /* edge {b, w} must be alive */\n", ""),
    ("bulk threshold k-3",
     "if (in_out[e] && s[e] < k - 2) { in_out[e] = 0; ++dropped; }",
     "if (in_out[e] && s[e] < k - 3) { in_out[e] = 0; ++dropped; }"),
    ("listing drops the third edge",
     "if (cnt) { cnt[exy]++; cnt[exz]++; cnt[eyz]++; }",
     "if (cnt) { cnt[exy]++; cnt[exz]++; }"),
    ("peeling misses a decrement",
     "if (--s[e2] < thr", "if (s[e2] < thr"),
    ("peeling destroys a triangle twice",
     "if (!alive[e1] || !alive[e2]) continue;     /* already destroyed */", "if (0) continue;"),
    ("truss number one too high",
     "if (alive[live[i]]) { tau[live[i]] = k; live[w++] = live[i]; }",
     "if (alive[live[i]]) { tau[live[i]] = k + 1; live[w++] = live[i]; }"),
    ("kmax one too high",
     "  *kmax = k - 1;\n", "  *kmax = k;\n"),
    ("search route restarts past a miss",
     "    lb = lo;\n", "    lb = lo + 1;\n"),
    ("search route misses the end of a list",
     "if (lo == hb || nbr[lo] != w) continue;", "if (lo + 1 >= hb || nbr[lo] != w) continue;"),
    ("search route: first edge not required present",
     "    if (!alive[eaw]) continue;                    /* {a, w} already removed */\n", ""),
    ("search route: second edge not required present",
     "    if (!alive[ebw]) continue;                    /* {b, w} removed: destroyed before */\n", ""),
    ("search route misses a decrement",
     "    lose_one(s, ebw, thr, queued, queue, qtail);\n", ""),
    ("threaded count deals vertices with a gap",
     "for (int32_t x = w->t; x < w->n; x += w->nthreads)",
     "for (int32_t x = w->t; x < w->n; x += w->nthreads + 1)"),
    ("search route: rewriting a list drops its last entry",
     "  for (int64_t i = b; i < e; ++i)\n    if (alive[L->g.eid[i]])",
     "  for (int64_t i = b; i + 1 < e; ++i)\n    if (alive[L->g.eid[i]])"),
]


def run_pins(tmp_path, text):
    """Build `text` as the oracle library and run the pins against it."""
    src = os.path.join(tmp_path, "oracle_mutant.c")
    lib = os.path.join(tmp_path, "liboracle_mutant.so")
    with open(src, "w") as f:
        f.write(text)
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-pthread", "-o", lib, src])
    env = dict(os.environ, ORACLE_LIB=lib, PYTHONPATH=ROOT)
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                           os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                          env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)


def test_unmodified_copy_passes_the_pins(tmp_path):
    """Control: the same route with nothing planted passes, so a failure
    below comes from the planted mistake."""
    r = run_pins(tmp_path, open(SRC).read())
    assert r.returncode == 0, (r.returncode, r.stdout[-1500:])


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_fails_the_pins(tmp_path, name, old, new):
    text = open(SRC).read()
    assert text.count(old) == 1, "mutation site not unique or gone: %s" % name
    r = run_pins(tmp_path, text.replace(old, new))
    # 1 = tests ran and failed (not a crash, a hang or a collection error)
    assert r.returncode == 1, (name, r.returncode, r.stdout[-1500:])
