"""Host-side checks of the C ABI (no GPU needed).

  * the built library loads and exports every function include/tlrmdd.h declares;
  * hilbert_order (host C++) equals the oracle bit for bit on many grids;
  * the ctypes mirrors of the header structs have its sizes and field offsets;
  * layout validation: tlrmdd_theta_size rejects every malformed layout and
    otherwise equals the oracle's packed size.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tlrmdd.h")

lib_mod = pytest.importorskip("paper_2412_14973_amd._lib")


@pytest.fixture(scope="module")
def lib():
    return lib_mod.load()


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(tlrmdd_\w+|hilbert_order)\s*\(", txt)))


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert "tlrmdd_solve" in names and "hilbert_order" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(lib_mod.EXPORTS)


def test_status_strings(lib):
    for s in range(7):
        assert lib.tlrmdd_status_string(s) and lib.tlrmdd_status_string(s) != b"unknown status"
    assert lib.tlrmdd_status_string(0) == b"ok"


@pytest.mark.parametrize("nx,ny", [(1, 1), (2, 2), (3, 3), (4, 4), (8, 8), (5, 7), (32, 32), (48, 48),
                                   (64, 64), (90, 17), (96, 96), (177, 90)])
def test_hilbert_bit_exact_vs_oracle(nx, ny):
    import paper_2412_14973_amd as tl
    g = synth.make_geometry(nx, ny)
    got = tl.hilbert_order(g.rec_ix, g.rec_iy)
    ref = O.hilbert_order(g.rec_ix, g.rec_iy)
    assert got.dtype == np.int64
    assert np.array_equal(got, ref)


def test_hilbert_duplicates_and_scattered_points():
    import paper_2412_14973_amd as tl
    rng = np.random.default_rng(5)
    ix = rng.integers(0, 37, 500).astype(np.int32)
    iy = rng.integers(0, 11, 500).astype(np.int32)
    assert np.array_equal(tl.hilbert_order(ix, iy), O.hilbert_order(ix, iy))


def test_hilbert_rejects_bad_input(lib):
    import paper_2412_14973_amd as tl
    with pytest.raises(tl.TLRMDDError):
        tl.hilbert_order(np.array([0, -1]), np.array([0, 0]))
    assert lib.hilbert_order(None, None, -1, None) == 1
    assert lib.hilbert_order(None, None, 0, None) == 0
    assert lib.hilbert_order(None, None, 3, None) == 1


def _theta_size(lib, tile_size, rank_off, rank_diag, ns=4, nr=None):
    ts = np.ascontiguousarray(tile_size, dtype=np.int32)
    ro = np.ascontiguousarray(rank_off, dtype=np.int32)
    rd = np.ascontiguousarray(rank_diag, dtype=np.int32)
    P = ctypes.POINTER(ctypes.c_int32)
    lay = lib_mod.c_layout(int(ts.sum()) if nr is None else nr, ns, int(ts.shape[0]), ts.ctypes.data_as(P),
                           ro.ctypes.data_as(P) if ro.size else None, rd.ctypes.data_as(P))
    return lib.tlrmdd_theta_size(ctypes.byref(lay))


@pytest.mark.parametrize("layout", [
    synth.uniform_layout(64, 16, 4, 8),
    synth.uniform_layout(64, 16, 4, -1),
    synth.uniform_layout(2304, 512, 33, -1),
    synth.adaptive_layout(1024, 40),
    synth.uniform_layout(30, 8, 3, 2),
])
def test_theta_size_matches_oracle(lib, layout):
    T = O.tiling(layout.tile_size, layout.rank_off, layout.rank_diag)
    assert _theta_size(lib, layout.tile_size, layout.rank_off, layout.rank_diag) == T.size


@pytest.mark.parametrize("ts,ro,rd,nr", [
    ([4, 4], [5], [2, 2], None),        # off rank > min(d_i, d_j)
    ([4, 4], [0], [2, 2], None),        # off rank 0
    ([4, 4], [2], [5, 2], None),        # diag rank > d_i
    ([4, 4], [2], [0, 2], None),        # diag rank 0
    ([4, 4], [2], [-2, 2], None),       # diag rank neither -1 nor >= 1
    ([4, 0], [1], [2, 1], None),        # empty tile
    ([4, 4], [2], [2, 2], 9),           # sum d_i != nr
])
def test_invalid_layouts_rejected(lib, ts, ro, rd, nr):
    assert _theta_size(lib, ts, ro, rd, nr=nr) < 0
    assert lib.tlrmdd_last_error()


def test_null_layout(lib):
    assert lib.tlrmdd_theta_size(None) < 0
    h = ctypes.c_void_p()
    assert lib.tlrmdd_plan_create(None, ctypes.byref(h)) == 1


def test_ctypes_structs_match_the_header(tmp_path):
    """Every struct the binding mirrors has the header's size and field offsets (a C++ program
    compiled against include/tlrmdd.h prints them)."""
    import shutil
    import subprocess
    if shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("g++ or the HIP headers are missing")
    structs = {"tlrmdd_layout": lib_mod.c_layout, "tlrmdd_opts": lib_mod.c_opts,
               "tlrmdd_admm_opts": lib_mod.c_admm_opts, "tlrmdd_kernel_stats": lib_mod.c_kernel_stats}
    cfield = {"lam": "lambda"}   # Python spelling -> C member
    lines = ['#include <cstdio>', '#include <cstddef>', '#include "tlrmdd.h"', 'int main() {']
    for cname, ct in structs.items():
        lines.append(f'  std::printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for fname, _ in ct._fields_:
            lines.append(f'  std::printf("{cname} {fname} %zu\\n", offsetof({cname}, {cfield.get(fname, fname)}));')
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.cpp"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["g++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"),
                    str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, ct in structs.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(ct), cname
        for fname, _ in ct._fields_:
            assert got[(cname, fname)] == getattr(ct, fname).offset, (cname, fname)


def test_graph_calls_reject_bad_arguments_without_a_device(lib):
    """The HIP-graph calls check their arguments before any HIP call: a null stream cannot be
    captured, nothing can be closed that was not opened, a null graph cannot be launched, and
    destroying a null graph is a no-op."""
    h = ctypes.c_void_p()
    assert lib.tlrmdd_graph_begin(ctypes.c_void_p(0)) == lib_mod.INVALID_ARGUMENT
    assert b"null stream" in lib.tlrmdd_last_error()
    assert lib.tlrmdd_graph_end(ctypes.c_void_p(0), ctypes.byref(h)) == lib_mod.INVALID_ARGUMENT
    assert h.value is None
    assert lib.tlrmdd_graph_end(ctypes.c_void_p(0), None) == lib_mod.INVALID_ARGUMENT
    assert lib.tlrmdd_graph_launch(ctypes.c_void_p(0), ctypes.c_void_p(0)) == lib_mod.INVALID_ARGUMENT
    assert lib.tlrmdd_graph_destroy(ctypes.c_void_p(0)) == lib_mod.OK


def test_timing_kind_sets_without_a_device(lib):
    """tlrmdd_timing_begin_kinds takes a non-empty set of kind bits below TLRMDD_K_NKINDS; with no
    launch in between, timing_end reports zero for every kind."""
    n = len(lib_mod.KIND_NAMES)
    assert lib.tlrmdd_timing_begin_kinds(0) == lib_mod.INVALID_ARGUMENT
    assert lib.tlrmdd_timing_begin_kinds(1 << n) == lib_mod.INVALID_ARGUMENT
    assert lib.tlrmdd_timing_begin_kinds((1 << n) | 1) == lib_mod.INVALID_ARGUMENT
    st = (lib_mod.c_kernel_stats * n)()
    assert lib.tlrmdd_timing_begin_kinds(1 << lib_mod.KIND_NAMES.index("gemm_line")) == lib_mod.OK
    assert lib.tlrmdd_timing_end(st) == lib_mod.OK
    assert all(s.launches == 0 and s.ms == 0.0 and s.flop_dtype == lib_mod.DT_NONE for s in st)
    assert lib.tlrmdd_timing_begin() == lib_mod.OK
    assert lib.tlrmdd_timing_end(None) == lib_mod.OK
