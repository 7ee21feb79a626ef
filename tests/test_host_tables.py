"""CPU checks of host logic built as plain C++ under the address and
undefined-behaviour sanitizers.

The Schwarz block tables (csrc/block_tables.h):
in-block neighbours, the face lists with the site across the face feeding
each entry, the face-exchange neighbour blocks with the antiperiodic sign,
and the colour-major block layout, compared with the global site
coordinates by tests/host_tables_check.cpp.  The same checker, built against
copies of the header with a planted mistake, must fail (so that the checks
are not vacuous).

The AMA driver's batch rule (csrc/batch_rule.h) on a grid of memory sizes
and requests: a request that 90% of the available memory holds is kept;
otherwise the batch is what 60% holds, at least 1, at most 48 and at most
the request, a multiple of 12 from 12 on, else even."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1605_00564_amd", "csrc")
SRC = os.path.join(ROOT, "tests", "host_tables_check.cpp")
FLAGS = ["-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         "-fno-omit-frame-pointer"]

GEOMETRIES = [
    ((8, 8, 8, 8), (4, 4, 4, 4), -1),
    ((4, 4, 4, 4), (2, 2, 2, 2), 1),
    ((8, 4, 4, 8), (2, 2, 2, 2), -1),
    ((16, 8, 8, 8), (8, 4, 4, 4), -1),
    ((12, 12, 12, 12), (6, 6, 6, 6), -1),
    ((16, 16, 16, 16), (8, 8, 8, 8), 1),
    ((64, 32, 32, 32), (4, 4, 4, 4), -1),
]

# (what the planted mistake breaks, the text replaced, its replacement)
MUTATIONS = [
    ("face source", "c[mu] = d == 0 ? 0 : b[mu] - 1;", "c[mu] = d == 0 ? b[mu] - 1 : 0;"),
    ("neighbour block", "cc[mu] = (cc[mu] + (d == 0 ? -1 : 1) + nb[mu]) % nb[mu];",
     "cc[mu] = (cc[mu] + (d == 0 ? 1 : -1) + nb[mu]) % nb[mu];"),
    ("boundary sign", "(d == 0 ? cb[0] == 0 : cb[0] == nb[0] - 1)", "(d == 0 ? cb[0] == nb[0] - 1 : cb[0] == 0)"),
    ("face order", "return da != dc ? da < dc : a < c;", "return da != dc ? da > dc : a < c;"),
]


def _compile(include_dir, out):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    r = subprocess.run(["g++", *FLAGS, "-I", include_dir, SRC, "-o", out], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("host_tables") / "check")
    _compile(CSRC, out)
    return out


def _run(exe, dims, block, bc):
    args = [exe, *map(str, dims), *map(str, block), str(bc)]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    return subprocess.run(args, capture_output=True, text=True, env=env, timeout=300)


@pytest.mark.parametrize("dims,block,bc", GEOMETRIES)
def test_block_tables_match_the_lattice(checker, dims, block, bc):
    r = _run(checker, dims, block, bc)
    print(r.stdout.strip())
    assert r.returncode == 0, r.stdout + r.stderr


@pytest.mark.parametrize("what,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_checker_finds_a_planted_mistake(tmp_path, what, old, new):
    text = open(os.path.join(CSRC, "block_tables.h")).read()
    assert text.count(old) == 1, what
    (tmp_path / "block_tables.h").write_text(text.replace(old, new))
    out = str(tmp_path / "check")
    _compile(str(tmp_path), out)
    # four blocks along t and x, so that the blocks on the two sides of a
    # block differ (with two blocks per direction they coincide)
    r = _run(out, (16, 16, 8, 8), (4, 4, 4, 4), -1)
    assert r.returncode == 1 and "mismatch" in r.stderr, (what, r.stdout, r.stderr)


def test_batch_rule():
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "batch")
        r = subprocess.run(["g++", *FLAGS, "-I", CSRC, os.path.join(ROOT, "tests", "batch_rule_check.cpp"), "-o", exe],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
        GB = 1 << 30
        cases = [(a * GB, p, w) for a in (0, 1, 7, 50, 120, 250, 280)
                 for p in (1, 11 * 2 ** 20, 5800 * 2 ** 20, 29 * GB, 46 * GB)
                 for w in (0, 1, 5, 7, 12, 24, 48, 1000, 10 ** 6)]
        inp = "".join(f"{a} {p} {w}\n" for a, p, w in cases)
        r = subprocess.run([exe], input=inp, capture_output=True, text=True, timeout=60)
        assert r.returncode == 0, r.stderr
        got = [int(v) for v in r.stdout.split()]
    assert len(got) == len(cases)
    for (a, p, w), n in zip(cases, got):
        if w > 0 and w <= int(0.9 * a) // p:
            assert n == w, (a, p, w, n)
            continue
        assert 1 <= n <= 48, (a, p, w, n)
        if w > 0:
            assert n <= w, (a, p, w, n)
        assert n == 1 or n % 2 == 0, (a, p, w, n)
        if n >= 12:
            assert n % 12 == 0, (a, p, w, n)
        fit = max(int(0.6 * a) // p, 1)
        assert n <= fit, (a, p, w, n)
        # the largest count of that form below the caps
        cap = min(fit, 48, w if w > 0 else 48)
        best = cap - cap % 12 if cap >= 12 else (cap - cap % 2 if cap > 1 else 1)
        assert n == best, (a, p, w, n, best)
