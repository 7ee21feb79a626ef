"""The C ABI without a GPU: the library built for gfx950 loads, exports
every function include/dfl.h declares, and its host-side error strings
answer without touching a device."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dfl.h")
LIB = os.path.join(ROOT, "paper_1605_00564_amd", "libdfl.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)     # drop comments
    text = re.sub(r"//[^\n]*", " ", text)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|void|char|size_t|double)\s*\**\s*(\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("dirac_apply", "sap_precond", "deflation_setup", "little_dirac_apply", "gcr_solve",
                     "ama_solve"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built (run __graft_entry__.build())")
def test_library_exports_every_declared_function():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built (run __graft_entry__.build())")
def test_error_strings_without_a_device():
    lib = ctypes.CDLL(LIB)
    lib.qcd_strerror.restype = ctypes.c_char_p
    lib.qcd_strerror.argtypes = [ctypes.c_int]
    seen = set()
    for code in (0, 1, -1, -2, -3, -4, -5, -6, -7):
        s = lib.qcd_strerror(code).decode()
        assert s and s not in seen, (code, s)
        seen.add(s)
    assert lib.qcd_strerror(-99).decode()


def test_autotuner_block_candidates_follow_the_checkerboard_rule():
    """Block shapes must divide the lattice with an even number of blocks per
    direction; on 24^3 x 48 that excludes 8^4 (three blocks across 24)."""
    from paper_1605_00564_amd import tune
    cands = ((4, 4, 4, 4), (8, 4, 4, 4), (6, 6, 6, 6), (8, 8, 8, 8))
    assert tune.valid_blocks((48, 24, 24, 24), cands) == [(4, 4, 4, 4), (8, 4, 4, 4), (6, 6, 6, 6)]
    assert tune.valid_blocks((64, 32, 32, 32), cands) == [(4, 4, 4, 4), (8, 4, 4, 4), (8, 8, 8, 8)]
    assert tune.valid_blocks((96, 48, 48, 48), cands) == list(cands)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built (run __graft_entry__.build())")
def test_workspace_cache_calls_without_a_device():
    """An empty workspace cache answers and trims without touching a device;
    a null byte count is an argument error."""
    lib = ctypes.CDLL(LIB)
    n = ctypes.c_size_t(123)
    assert lib.qcd_workspace_cached(0, ctypes.byref(n)) == 0 and n.value == 0
    assert lib.qcd_workspace_cached(0, None) == -1
    assert lib.qcd_workspace_trim(-1) == 0
    lib.qcd_field_trim.argtypes = [ctypes.c_void_p]
    assert lib.qcd_field_trim(None) == -1


def test_autotuner_prior_ranks_block_shapes_per_site():
    """A previous tuning's table (another lattice) orders the candidates by
    time per source per site; shapes it never timed go last."""
    from paper_1605_00564_amd import tune
    prior = [{"block": (4, 4, 4, 4), "per_source_s": 8.0, "volume": 100},
             {"block": (8, 4, 4, 4), "per_source_s": 5.4, "volume": 100},
             {"block": (6, 6, 6, 6), "per_source_s": 30.0, "volume": 400},
             {"block": (8, 4, 4, 4), "per_source_s": 6.0, "volume": 100}]
    cands = [(4, 4, 4, 4), (8, 4, 4, 4), (6, 6, 6, 6), (8, 8, 8, 8)]
    assert tune.rank_by_prior(cands, prior) == [(8, 4, 4, 4), (6, 6, 6, 6), (4, 4, 4, 4), (8, 8, 8, 8)]
    assert tune.rank_by_prior(cands, None) == cands


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU; asking for more exits with a message."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_binding_covers_every_declared_function():
    """The Python binding reaches every function include/dfl.h declares."""
    src = open(os.path.join(ROOT, "paper_1605_00564_amd", "_lib.py")).read()
    missing = [n for n in declared_functions() if n not in src]
    assert not missing, missing


class _Lattice(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int * 4), ("block", ctypes.c_int * 4), ("kappa", ctypes.c_double),
                ("csw", ctypes.c_double), ("bc_t", ctypes.c_int)]


def _create(lib, dims, block, kappa=0.124, bc_t=-1):
    lat = _Lattice((ctypes.c_int * 4)(*dims), (ctypes.c_int * 4)(*block), kappa, 1.5, bc_t)
    dummy = (ctypes.c_double * 8)()          # never read: the checks come first
    h = ctypes.c_void_p()
    lib.qcd_field_create.argtypes = [ctypes.POINTER(_Lattice), ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.POINTER(ctypes.c_void_p)]
    rc = lib.qcd_field_create(ctypes.byref(lat), ctypes.cast(dummy, ctypes.c_void_p), None, ctypes.byref(h))
    lib.qcd_last_error.restype = ctypes.c_char_p
    return rc, lib.qcd_last_error().decode(), h.value


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built (run __graft_entry__.build())")
def test_lattice_checks_come_before_any_device_call():
    """Geometry and parameter errors are reported without a device: an odd
    block, an odd number of blocks, a bad boundary flag, and lattices whose
    largest buffer offset (384 bytes per site) reaches 2^32.  48^3 x 96 is
    the largest lattice of the workloads and stays inside the limit."""
    lib = ctypes.CDLL(LIB)
    assert _create(lib, (8, 8, 8, 8), (3, 4, 4, 4))[0] == -2
    assert _create(lib, (12, 8, 8, 8), (4, 4, 4, 4))[0] == -2
    assert _create(lib, (8, 8, 8, 8), (4, 4, 4, 4), bc_t=0)[0] == -1
    rc, msg, h = _create(lib, (64, 64, 64, 64), (4, 4, 4, 4))
    assert rc == -1 and "32-bit buffer offsets" in msg and h is None
    rc, msg, _ = _create(lib, (112, 56, 56, 56), (4, 4, 4, 4))
    assert rc == -1 and "32-bit buffer offsets" in msg
    assert 96 * 48 ** 3 * 384 < 2 ** 32 <= 112 * 56 ** 3 * 384


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors of the parameter structs have the C header's sizes
    and field offsets (a host program built against include/dfl.h prints
    them)."""
    import ctypes
    import shutil
    import subprocess

    from paper_1605_00564_amd import _lib as L

    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    mirrors = {"qcd_lattice": L._Lattice, "qcd_sap": L._Sap, "qcd_dfl_params": L._DflParams, "qcd_gcr": L._Gcr,
               "qcd_info": L._Info, "qcd_source": L._Source, "qcd_ama": L._Ama}
    lines = ["#include <cstddef>", "#include <cstdio>", '#include "dfl.h"', "int main() {"]
    for cname, py in mirrors.items():
        lines.append(f'    std::printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'    std::printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.cpp"
    src.write_text("\n".join(lines) + "\n")
    exe = str(tmp_path / "layout")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run(["g++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                        "-I" + os.path.join(root, "include"), str(src), "-o", exe], capture_output=True, text=True)
    if r.returncode != 0 and "hip_runtime_api.h" in r.stderr:
        pytest.skip("HIP headers not available")
    assert r.returncode == 0, r.stderr
    out = [v for v in subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n") if v]
    assert len(out) == sum(len(py._fields_) + 1 for py in mirrors.values())
    for line in out:
        parts = line.split()
        py = mirrors[parts[0]]
        if parts[1] == "size":
            assert ctypes.sizeof(py) == int(parts[2]), line
        else:
            assert getattr(py, parts[1]).offset == int(parts[2]), line
