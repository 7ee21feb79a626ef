"""CPU checks of the host-built Schwarz block tables (csrc/block_tables.h):
in-block neighbours, the face lists with the site across the face feeding
each entry, the face-exchange neighbour blocks with the antiperiodic sign,
and the colour-major block layout, compared with the global site
coordinates by tests/host_tables_check.cpp, which is built with the address
and undefined-behaviour sanitizers.  The same checker, built against copies
of the header with a planted mistake, must fail (so that the checks are not
vacuous)."""

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
