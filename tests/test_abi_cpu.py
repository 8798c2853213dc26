"""CPU checks of the C ABI: the library loads, exports every function that
include/hom.h declares, and validates arguments before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hom.h")


def _lib():
    from paper_1404_3614_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        from paper_1404_3614_amd import build
        build.build(verbose=False)
    return L, L.load()


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hom_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["hom_setup", "hom_solve_primal", "hom_solve_dual", "hom_bounds", "hom_workspace_bytes",
              "hom_field_len", "hom_coef_inclusions", "hom_coef_pixels", "hom_apply", "hom_destroy"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    L, lib = _lib()
    for n in declared_functions():
        assert hasattr(lib, n), n
        assert n in L.EXPORTS, f"{n} has no ctypes declaration"


def _desc(L, d=2, N=(13, 13, 1), prec=0, nc=1, Y=(1.0, 1.0, 1.0)):
    ds = L.Desc()
    ds.d = d
    for a in range(3):
        ds.N[a] = N[a]
        ds.Y[a] = Y[a]
    ds.precision = prec
    ds.ncoef = nc
    return ds


@pytest.mark.parametrize("N,expect", [((13, 13, 1), 0), ((12, 13, 1), -2), ((7, 13, 1), -2),
                                      ((313, 313, 1), 0), ((1, 13, 1), -2), ((63, 41, 1), 0)])
def test_size_validation(N, expect):
    # N even -> unsupported; N = 7 gives M = 13, not of the form 3^p 5^q
    L, lib = _lib()
    n = C.c_size_t()
    assert lib.hom_workspace_bytes(C.byref(_desc(L, N=N)), 2, C.byref(n)) == expect


def test_argument_validation_without_device():
    L, lib = _lib()
    n = C.c_size_t()
    assert lib.hom_workspace_bytes(C.byref(_desc(L, d=4)), 1, C.byref(n)) == L.HOM_E_INVALID
    assert lib.hom_workspace_bytes(C.byref(_desc(L, nc=2)), 1, C.byref(n)) == L.HOM_E_INVALID
    assert lib.hom_workspace_bytes(C.byref(_desc(L, prec=7)), 1, C.byref(n)) == L.HOM_E_INVALID
    assert lib.hom_workspace_bytes(C.byref(_desc(L)), 0, C.byref(n)) == L.HOM_E_INVALID
    assert lib.hom_workspace_bytes(C.byref(_desc(L)), 4, C.byref(n)) == L.HOM_E_INVALID
    assert lib.hom_workspace_bytes(C.byref(_desc(L, Y=(1.0, -1.0, 1.0))), 1, C.byref(n)) == L.HOM_E_INVALID
    assert lib.hom_workspace_bytes(None, 1, C.byref(n)) == L.HOM_E_INVALID
    h = C.c_void_p()
    # null coefficient pointers are rejected before any device call
    assert lib.hom_setup(C.byref(_desc(L)), 1, None, None, None, 0, None, C.byref(h)) == L.HOM_E_INVALID
    assert lib.hom_bounds(None, None, None, None) == L.HOM_E_INVALID
    assert lib.hom_status_str(-3) == b"HOM_E_NOT_SPD"
    lib.hom_destroy(None)


def test_field_len_matches_layout():
    L, lib = _lib()
    n = C.c_size_t()
    assert lib.hom_field_len(C.byref(_desc(L, N=(13, 13, 1))), 0, C.byref(n)) == 0
    assert n.value == 7 * 13
    assert lib.hom_field_len(C.byref(_desc(L, d=3, N=(5, 13, 41))), 1, C.byref(n)) == 0
    assert n.value == 2 * 3 * 13 * 41
    # the field length depends on N only (N1 = 9, whose 2N - 1 = 17 needs a larger quadrature grid)
    assert lib.hom_field_len(C.byref(_desc(L, d=3, N=(5, 9, 13))), 1, C.byref(n)) == 0
    assert n.value == 2 * 3 * 9 * 13
    assert lib.hom_field_len(C.byref(_desc(L, d=3, N=(5, 8, 13))), 1, C.byref(n)) == L.HOM_E_UNSUPPORTED_SIZE
    # a problem on N1 = 9 needs a quadrature grid: 2N - 1 = 17 has a factor 17, M = 25 is accepted
    ws = C.c_size_t()
    assert lib.hom_workspace_bytes(C.byref(_desc(L, d=3, N=(5, 9, 13))), 3, C.byref(ws)) == L.HOM_E_UNSUPPORTED_SIZE
    ds = _desc(L, d=3, N=(5, 9, 13))
    ds.M[0], ds.M[1], ds.M[2] = 9, 25, 25
    assert lib.hom_workspace_bytes(C.byref(ds), 3, C.byref(ws)) == 0
    for bad in ((9, 23, 25), (9, 26, 25), (9, 49, 25)):      # below 2N - 1, even, factor 7
        ds.M[0], ds.M[1], ds.M[2] = bad
        assert lib.hom_workspace_bytes(C.byref(ds), 3, C.byref(ws)) == L.HOM_E_UNSUPPORTED_SIZE


def test_workspace_grows_with_loads_and_precision():
    L, lib = _lib()
    sizes = {}
    for prec in (0, 1):
        for loads in (1, 2):
            n = C.c_size_t()
            assert lib.hom_workspace_bytes(C.byref(_desc(L, N=(41, 41, 1), prec=prec)), loads, C.byref(n)) == 0
            sizes[(prec, loads)] = n.value
            assert n.value % 256 == 0
    assert sizes[(0, 2)] > sizes[(0, 1)]
    assert sizes[(1, 1)] != sizes[(0, 1)]


def test_sizes_beyond_the_lds_of_the_passes_are_refused():
    # the column pass holds one FP64 column of every pack (2D bounds: two packs): M0 = 5625
    # (3^2 5^4) does not fit in 160 KB, M0 = 3125 does; the rows stay within their split form
    L, lib = _lib()
    ws = C.c_size_t()
    for prec in (0, 1):
        ok = _desc(L, N=(1563, 1563, 1), prec=prec)
        ok.M[0], ok.M[1] = 3125, 3125
        assert lib.hom_workspace_bytes(C.byref(ok), 2, C.byref(ws)) == 0
        big = _desc(L, N=(2813, 13, 1), prec=prec)
        big.M[0], big.M[1] = 5625, 25
        assert lib.hom_workspace_bytes(C.byref(big), 2, C.byref(ws)) == L.HOM_E_UNSUPPORTED_SIZE
    # GaNi grids: N or N + 1 with a radix-2/3/5 transform, and not beyond the quadrature grid
    ds = _desc(L, N=(15, 15, 1))
    ds.M[0], ds.M[1] = 45, 45
    for grid, expect in (((15, 15), 0), ((16, 15), 0), ((16, 16), 0), ((17, 15), -2), ((14, 15), -2)):
        g = (C.c_int32 * 3)(grid[0], grid[1], 1)
        assert lib.hom_gani_workspace_bytes(C.byref(ds), g, C.byref(ws)) == expect, grid


def test_phase_eig_range_matches_eigvalsh():
    """hom_phase_eig_range (host arithmetic, no device) against LAPACK's
    symmetric eigenvalues, with ill-conditioned and rotated phases."""
    L, lib = _lib()
    import homgen
    rng = np.random.default_rng(11)
    for d in (2, 3):
        for trial in range(20):
            mats = [homgen.random_spd(rng, d, 1e-3, 1e3) for _ in range(1 + trial % 4)]
            A = np.ascontiguousarray(np.stack(mats).reshape(-1))
            out = (C.c_double * 2)()
            st = lib.hom_phase_eig_range(d, len(mats), A.ctypes.data_as(C.POINTER(C.c_double)), out)
            assert st == 0
            ev = np.concatenate([np.linalg.eigvalsh(m) for m in mats])
            assert abs(out[0] - ev.min()) <= 1e-12 * ev.max()
            assert abs(out[1] - ev.max()) <= 1e-12 * ev.max()
    bad = np.ascontiguousarray(np.array([[1.0, 2.0], [2.0, 1.0]]).reshape(-1))     # eigenvalues -1, 3
    out = (C.c_double * 2)()
    assert lib.hom_phase_eig_range(2, 1, bad.ctypes.data_as(C.POINTER(C.c_double)), out) == L.HOM_E_NOT_SPD
    assert lib.hom_phase_eig_range(4, 1, bad.ctypes.data_as(C.POINTER(C.c_double)), out) == L.HOM_E_INVALID


def test_coef_scratch_bytes():
    L, lib = _lib()
    n = C.c_size_t()
    ds = _desc(L)
    assert lib.hom_coef_scratch_bytes(C.byref(ds), 10, None, C.byref(n)) == 0
    small = n.value
    assert lib.hom_coef_scratch_bytes(C.byref(ds), 100, None, C.byref(n)) == 0
    assert n.value > small >= 64
    P = (C.c_int32 * 3)(125, 125, 1)
    assert lib.hom_coef_scratch_bytes(C.byref(ds), 0, P, C.byref(n)) == 0
    assert n.value >= 125 * 125 * 16
    assert lib.hom_coef_scratch_bytes(C.byref(ds), -1, None, C.byref(n)) == L.HOM_E_INVALID
    P0 = (C.c_int32 * 3)(0, 125, 1)
    assert lib.hom_coef_scratch_bytes(C.byref(ds), 0, P0, C.byref(n)) == L.HOM_E_INVALID


def test_tuner_cache_file_roundtrip(tmp_path):
    """The tuner cache on disk (host code, no device): entries of the named
    architecture are merged, others skipped; saving writes them back; a line
    that does not parse is an error."""
    L, lib = _lib()
    src = tmp_path / "tune.jsonl"
    src.write_text(
        '{"arch": "gfx950", "M0": 625, "M1": 1, "M2": 625, "d": 2, "loads": 2, "dual": 0, "nc": 1, "packs": 1, '
        '"row_pairs": 2, "row_threads": 256, "apply_points": 10, "apply_half_exchange": 1, "apply_all_packs": 0, '
        '"row_ms": 0.1505, "apply_ms": 0.0672, "candidates": 11}\n'
        '{"arch": "gfx942", "M0": 81, "M1": 81, "M2": 81, "d": 3, "loads": 3, "dual": 1, "nc": 1, "packs": 5, '
        '"row_pairs": 7, "row_threads": 0, "apply_points": 14, "apply_half_exchange": 0, "apply_all_packs": 0, '
        '"row_ms": 0.2, "apply_ms": 0.1, "candidates": 9}\n')
    assert lib.hom_tune_cache_clear() == 0
    n = C.c_int32()
    assert lib.hom_tune_cache_load(str(src).encode(), b"gfx950", C.byref(n)) == 0
    assert n.value == 1
    out = tmp_path / "out.jsonl"
    assert lib.hom_tune_cache_save(str(out).encode(), b"gfx950") == 0
    lines = out.read_text().strip().splitlines()
    assert len(lines) == 1
    import json
    rec = json.loads(lines[0])
    assert rec["arch"] == "gfx950" and rec["M0"] == 625 and rec["apply_points"] == 10
    assert rec["apply_half_exchange"] == 1 and abs(rec["row_ms"] - 0.1505) < 1e-12 and rec["candidates"] == 11
    bad = tmp_path / "bad.jsonl"
    bad.write_text('{"arch": "gfx950", "M0": 625}\n')
    assert lib.hom_tune_cache_load(str(bad).encode(), b"gfx950", C.byref(n)) == L.HOM_E_INVALID
    assert lib.hom_tune_cache_load(str(tmp_path / "missing").encode(), b"gfx950", C.byref(n)) == L.HOM_E_INVALID
    assert lib.hom_tune_cache_clear() == 0


def test_unet_sizes_validation():
    """hom_unet_sizes (host code): parameters and work memory grow with the
    width; descriptors outside the documented ranges are refused."""
    L, lib = _lib()
    npar, work = C.c_size_t(), C.c_size_t()

    def sizes(d, size, levels=3, base=8, batch=2):
        ds = L.UNetDesc(d, levels, base, 2, 4, (C.c_int32 * 3)(*size), batch)
        st = lib.hom_unet_sizes(C.byref(ds), C.byref(npar), C.byref(work))
        return st, npar.value, work.value

    st, p8, w8 = sizes(2, (33, 33, 0))
    assert st == 0 and p8 > 0 and w8 > 0
    st, p16, w16 = sizes(2, (33, 33, 0), base=16)
    assert st == 0 and p16 > 3 * p8 and w16 > w8
    assert sizes(3, (17, 17, 17))[0] == 0
    assert sizes(2, (4096, 4096, 0))[0] == 0                  # 2^24 points: the largest plane
    assert sizes(2, (4097, 4096, 0))[0] == L.HOM_E_INVALID
    assert sizes(2, (1, 33, 0))[0] == L.HOM_E_INVALID
    assert sizes(2, (33, 33, 0), levels=7)[0] == L.HOM_E_INVALID
    assert sizes(4, (33, 33, 33))[0] == L.HOM_E_INVALID
