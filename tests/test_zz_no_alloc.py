"""GPU: the allocation-free coefficient entry point (hom_coef_inclusions_static)
against hom_coef_inclusions with caller scratch, called through the C ABI.

Both launch the same kernel on the same inputs, so the outputs must be equal
bit for bit.  Two calls in a row, the second with fewer inclusions and a
smaller grid, check that nothing of the first call's table survives in the
shared device array; sizes above its limit are refused before any launch."""
import ctypes as C

import numpy as np
import pytest

import homgen

pytestmark = pytest.mark.gpu


def _setup():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_1404_3614_amd import _lib as L
    from paper_1404_3614_amd import api
    return torch, L, L.load(), api


def _call(torch, L, lib, api, cell, N, inverse, static):
    d = cell.d
    ncoef = api.cell_ncoef(cell)
    ds = api._desc(d, N, cell.Y, "fp64", ncoef)
    M = api.quad_grid(N[:d])
    out = torch.full((ncoef,) + tuple(M), float("nan"), dtype=torch.complex128, device="cuda")
    A0, n, kind, cen, siz, Ain = api._incl_args(cell)
    dbl = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    if static:
        st = lib.hom_coef_inclusions_static(C.byref(ds), dbl(A0), n, kind, dbl(cen), dbl(siz), dbl(Ain), int(inverse),
                                            C.c_void_p(out.data_ptr()), stream)
    else:
        nb = C.c_size_t()
        assert lib.hom_coef_scratch_bytes(C.byref(ds), n, None, C.byref(nb)) == 0
        scr = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
        st = lib.hom_coef_inclusions(C.byref(ds), dbl(A0), n, kind, dbl(cen), dbl(siz), dbl(Ain), int(inverse),
                                     C.c_void_p(out.data_ptr()), C.c_void_p(scr.data_ptr()), nb.value, stream)
    assert st == 0, (static, st)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_static_coefficients_equal_scratch_version_on_consecutive_calls():
    torch, L, lib, api = _setup()
    big, _ = homgen.random_squares_cell(777, kmin=10, kmax=10)
    small = homgen.square_inclusion_cell(d=2, side=0.3, rho_in=50.0)
    sph = homgen.sphere_cell(seed=3, n=6, anisotropic=True)
    cases = [(big, (63, 63)), (small, (13, 13)), (sph, (13, 13, 13)), (small, (41, 13))]
    for cell, N in cases:
        print(f"[no_alloc] d={cell.d} n_incl={cell.n} N={N}", flush=True)
        for inverse in (False, True):
            ref = _call(torch, L, lib, api, cell, N, inverse, static=False)
            got = _call(torch, L, lib, api, cell, N, inverse, static=True)
            assert np.all(np.isfinite(got))
            assert np.array_equal(got, ref), (N, inverse)


def test_static_rejects_too_many_inclusions():
    torch, L, lib, api = _setup()
    c = homgen.Inclusions(d=2, Y=np.ones(2), A0=np.eye(2))
    for j in range(513):       # tiny disjoint squares on a 23 x 23 lattice
        c.add("rect", [(j % 23) / 23.0 - 0.5, (j // 23) / 23.0 - 0.5], [0.01, 0.01], 2.0 * np.eye(2))
    ds = api._desc(2, (13, 13), c.Y, "fp64", 1)
    A0, n, kind, cen, siz, Ain = api._incl_args(c)
    dbl = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    out = torch.zeros((1, 25, 25), dtype=torch.complex128, device="cuda")
    st = lib.hom_coef_inclusions_static(C.byref(ds), dbl(A0), n, kind, dbl(cen), dbl(siz), dbl(Ain), 0,
                                        C.c_void_p(out.data_ptr()), None)
    assert st == L.HOM_E_UNSUPPORTED_SIZE
    assert bool((out == 0).all())
