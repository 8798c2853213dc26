"""Python binding of libhom: device memory and streams from PyTorch, every
computation in the HIP library.  Names follow the C ABI (include/hom.h)."""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L

__all__ = ["Problem", "Batch", "Group", "coef_inclusions", "coef_pixels", "coef_from_cell", "problem_from_cell",
           "field_len", "workspace_bytes", "HomError"]

HomError = L.HomError


def _dev():
    if not torch.cuda.is_available():
        raise RuntimeError("libhom needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch.device("cuda", torch.cuda.current_device())


def _desc(d, N, Y, precision, ncoef, M=None):
    ds = L.Desc()
    ds.d = d
    for a in range(3):
        ds.N[a] = int(N[a]) if a < d else 1
        ds.Y[a] = float(Y[a]) if a < d else 1.0
        ds.M[a] = int(M[a]) if (M is not None and a < d) else 0
    ds.precision = {"fp64": L.HOM_FP64, "mixed": L.HOM_MIXED}.get(precision, precision)
    ds.ncoef = ncoef
    return ds


def quad_grid(N, M=None):
    """Quadrature grid per axis: M if given, else the doubled grid 2N - 1."""
    return tuple(int(m) for m in M) if M is not None else tuple(2 * int(n) - 1 for n in N)


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dptrs(tensors):
    arr = (C.c_void_p * len(tensors))()
    for i, t in enumerate(tensors):
        arr[i] = None if t is None else t.data_ptr()
    return arr


def field_len(d, N, dual, Y=(1, 1, 1)):
    n = C.c_size_t()
    ds = _desc(d, N, Y, "fp64", 1)
    L.check(L.load().hom_field_len(C.byref(ds), int(dual), C.byref(n)), "hom_field_len")
    return n.value


def workspace_bytes(d, N, Y, precision, ncoef, max_loads, M=None):
    n = C.c_size_t()
    ds = _desc(d, N, Y, precision, ncoef, M)
    L.check(L.load().hom_workspace_bytes(C.byref(ds), int(max_loads), C.byref(n)), "hom_workspace_bytes")
    return n.value


def _is_iso(A):
    A = np.asarray(A, float)
    return np.allclose(A, A[0, 0] * np.eye(A.shape[0]), rtol=0, atol=0)


def cell_ncoef(cell):
    """1 when every phase is a multiple of I, else d(d+1)/2."""
    d = cell.d
    mats = list(cell.phase_A) if hasattr(cell, "phase") else [cell.A0] + list(cell.A)
    return 1 if all(_is_iso(A) for A in mats) else d * (d + 1) // 2


def _dbl(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def cell_eig_range(cell):
    """Smallest and largest eigenvalue over the phases of a cell
    (hom_phase_eig_range): the a_min and a_max of the guaranteed stopping rule
    (set_stop)."""
    if hasattr(cell, "phase"):
        mats = [cell.phase_A[i] for i in np.unique(cell.phase)]
    else:
        mats = [cell.A0] + list(cell.A)
    A = np.ascontiguousarray(np.stack([np.asarray(m, float) for m in mats]).reshape(-1))
    out = (C.c_double * 2)()
    L.check(L.load().hom_phase_eig_range(cell.d, len(mats), _dbl(A), out), "hom_phase_eig_range")
    return float(out[0]), float(out[1])


def _scratch(ds, n_incl=0, P=None, stream=None):
    """Caller-owned device scratch of the coefficient helpers (hom_coef_scratch_bytes),
    kept alive until `stream` has passed the work that reads it."""
    n = C.c_size_t()
    Pc = None if P is None else (C.c_int32 * 3)(*(list(P) + [1] * (3 - len(P))))
    L.check(L.load().hom_coef_scratch_bytes(C.byref(ds), int(n_incl), Pc, C.byref(n)), "hom_coef_scratch_bytes")
    t = torch.empty(max(int(n.value), 1), dtype=torch.uint8, device=_dev())
    s = stream if stream is not None else torch.cuda.current_stream()
    if s != torch.cuda.current_stream():
        t.record_stream(s)
    return t


def _incl_args(cell):
    d, n = cell.d, cell.n
    kind = (C.c_int32 * max(n, 1))(*[0 if k == "rect" else 1 for k in cell.kind])
    cen = np.ascontiguousarray(np.array(cell.center, float).reshape(-1) if n else np.zeros(1))
    siz = np.zeros((max(n, 1), d))
    for j, s in enumerate(cell.size):
        siz[j, :len(s)] = s
    siz = np.ascontiguousarray(siz.reshape(-1))
    Ain = np.ascontiguousarray(np.array(cell.A, float).reshape(-1) if n else np.zeros(1))
    A0 = np.ascontiguousarray(np.asarray(cell.A0, float).reshape(-1))
    return A0, n, kind, cen, siz, Ain


def _pixel_args(cell):
    d = cell.d
    P = (C.c_int32 * 3)(*(list(cell.phase.shape) + [1] * (3 - d)))
    ph = np.ascontiguousarray(cell.phase.astype(np.int32).reshape(-1))
    pA = np.ascontiguousarray(np.asarray(cell.phase_A, float).reshape(-1))
    return P, ph, pA


def _wait(stream):
    if stream is not None:
        stream.wait_stream(torch.cuda.current_stream())


def coef_inclusions(cell, N, ncoef, inverse=False, stream=None, M=None):
    """Fourier coefficients on Z_M (default M = 2N - 1) of a matrix-inclusion cell, on the device."""
    d = cell.d
    ds = _desc(d, N, cell.Y, "fp64", ncoef, M)
    M = quad_grid(N[:d], M)
    out = torch.empty((ncoef,) + tuple(M), dtype=torch.complex128, device=_dev())
    A0, n, kind, cen, siz, Ain = _incl_args(cell)
    scr = _scratch(ds, n, None, stream)
    _wait(stream)
    st = L.load().hom_coef_inclusions(C.byref(ds), _dbl(A0), n, kind, _dbl(cen), _dbl(siz), _dbl(Ain), int(inverse),
                                      C.c_void_p(out.data_ptr()), C.c_void_p(scr.data_ptr()), scr.numel(),
                                      _stream_ptr(stream))
    L.check(st, "hom_coef_inclusions")
    return out


def coef_pixels(cell, N, ncoef, inverse=False, stream=None, M=None):
    """Fourier coefficients on Z_M (default M = 2N - 1) of a pixel/voxel image, on the device."""
    d = cell.d
    ds = _desc(d, N, cell.Y, "fp64", ncoef, M)
    M = quad_grid(N[:d], M)
    out = torch.empty((ncoef,) + tuple(M), dtype=torch.complex128, device=_dev())
    P, ph, pA = _pixel_args(cell)
    scr = _scratch(ds, 0, cell.phase.shape, stream)
    _wait(stream)
    st = L.load().hom_coef_pixels(C.byref(ds), P, ph.ctypes.data_as(C.POINTER(C.c_int32)), len(cell.phase_A),
                                  _dbl(pA), int(inverse), C.c_void_p(out.data_ptr()), C.c_void_p(scr.data_ptr()),
                                  scr.numel(), _stream_ptr(stream))
    L.check(st, "hom_coef_pixels")
    return out


def sample_cell(cell, N, ncoef=None, inverse=False, stream=None, closed=False):
    """Point values of A (or A^-1) at the points of the grid N (odd or even) of a
    cell, on the device (hom_sample_inclusions / hom_sample_pixels): float64
    [ncoef][*N]; closed: box faces belong to the inclusion."""
    d = cell.d
    N = tuple(int(n) for n in (N if np.iterable(N) else [N] * d))
    ncoef = cell_ncoef(cell) if ncoef is None else ncoef
    ds = _desc(d, N, cell.Y, "fp64", ncoef)
    out = torch.empty((ncoef,) + N, dtype=torch.float64, device=_dev())
    if hasattr(cell, "phase"):
        P, ph, pA = _pixel_args(cell)
        scr = _scratch(ds, 0, cell.phase.shape, stream)
        _wait(stream)
        st = L.load().hom_sample_pixels(C.byref(ds), P, ph.ctypes.data_as(C.POINTER(C.c_int32)), len(cell.phase_A),
                                        _dbl(pA), int(inverse), C.c_void_p(out.data_ptr()),
                                        C.c_void_p(scr.data_ptr()), scr.numel(), _stream_ptr(stream))
        L.check(st, "hom_sample_pixels")
        return out
    A0, n, kind, cen, siz, Ain = _incl_args(cell)
    scr = _scratch(ds, n, None, stream)
    _wait(stream)
    st = L.load().hom_sample_inclusions(C.byref(ds), _dbl(A0), n, kind, _dbl(cen), _dbl(siz), _dbl(Ain), int(inverse),
                                        int(bool(closed)), C.c_void_p(out.data_ptr()), C.c_void_p(scr.data_ptr()),
                                        scr.numel(), _stream_ptr(stream))
    L.check(st, "hom_sample_inclusions")
    return out


def probe_copy_gbs(nbytes=1 << 30, reps=10, stream=None):
    """Streaming rate of the device (hom_probe_copy): GB/s of bytes read plus written
    by a copy of nbytes, the measured peak for the HBM roofline."""
    n = (int(nbytes) // 16) * 16
    src = torch.ones(n // 4, dtype=torch.float32, device=_dev())
    dst = torch.empty_like(src)
    g = C.c_double()
    L.check(L.load().hom_probe_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), n, int(reps),
                                    _stream_ptr(stream), C.byref(g)), "hom_probe_copy")
    torch.cuda.synchronize()
    assert bool(torch.equal(src, dst)), "probe copy mismatch"
    del src, dst
    return g.value


def smooth_pixel_cell(cell, stream=None):
    """The smoothed medium of a two-phase 2D pixel cell (hom_smooth_pixels): a
    pixel cell with phases k = 0..16 of coefficient A0 + (k/16)(A1 - A0), k/16
    the smoothed characteristic function of phase 1."""
    import homgen
    assert cell.d == 2 and len(cell.phase_A) == 2, "two-phase 2D pixel cells"
    f = torch.as_tensor(np.ascontiguousarray(cell.phase == 1).astype(np.int32), device=_dev())
    out = torch.empty_like(f)
    _wait(stream)
    P = (C.c_int32 * 2)(*cell.phase.shape)
    A01 = np.ascontiguousarray(np.asarray(cell.phase_A, float).reshape(-1))
    table = np.zeros((17, 2, 2))
    L.check(L.load().hom_smooth_pixels(P, C.c_void_p(f.data_ptr()), C.c_void_p(out.data_ptr()), 2, _dbl(A01),
                                       _dbl(table), _stream_ptr(stream)), "hom_smooth_pixels")
    return homgen.Pixels(d=2, Y=np.asarray(cell.Y, float), phase=out.cpu().numpy().astype(np.int64), phase_A=table)


def coef_from_cell(cell, N, ncoef=None, stream=None, M=None):
    ncoef = cell_ncoef(cell) if ncoef is None else ncoef
    f = coef_pixels if hasattr(cell, "phase") else coef_inclusions
    return f(cell, N, ncoef, False, stream, M), f(cell, N, ncoef, True, stream, M), ncoef


class Problem:
    """One periodic cell on an odd grid N: the doubled-grid coefficients of A
    and A^{-1} live in a workspace tensor; solves return spectral fields."""

    def __init__(self, d, N, Y, Ahat, Bhat, precision="mixed", ncoef=1, max_loads=None, stream=None, M=None):
        lib = L.load()
        self.d = d
        self.N = tuple(int(n) for n in N[:d])
        self.Mq = quad_grid(self.N, None if M is None else tuple(M)[:d])
        self.Y = tuple(float(y) for y in Y[:d])
        self.precision = precision
        self.ncoef = ncoef
        self.max_loads = d if max_loads is None else max_loads
        # a dedicated stream (not the legacy default stream) so that the CG chunks are graph-captured
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.stream.wait_stream(torch.cuda.current_stream())
        self.desc = _desc(d, self.N, self.Y, precision, ncoef, self.Mq)
        nbytes = workspace_bytes(d, self.N, self.Y, precision, ncoef, self.max_loads, self.Mq)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=_dev())
        off = (-self.ws.data_ptr()) % 256
        self._ws_ptr = self.ws.data_ptr() + off
        h = C.c_void_p()
        st = lib.hom_setup(C.byref(self.desc), self.max_loads, C.c_void_p(Ahat.data_ptr()),
                           C.c_void_p(Bhat.data_ptr()), C.c_void_p(self._ws_ptr), nbytes,
                           C.c_void_p(self.stream.cuda_stream), C.byref(h))
        L.check(st, "hom_setup")
        self.h = h
        self._coef_refs = (Ahat, Bhat)   # the setup reads them asynchronously on self.stream
        self.flen = [field_len(d, self.N, 0, self.Y), field_len(d, self.N, 1, self.Y)]

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            try:
                L.load().hom_destroy(h)
            except Exception:
                pass
            self.h = None

    def update_coefficients(self, Ahat, Bhat):
        """New coefficient (same grid and layout) for this problem, keeping its workspace."""
        self.stream.wait_stream(torch.cuda.current_stream())
        L.check(L.load().hom_update_coefficients(self.h, C.c_void_p(Ahat.data_ptr()), C.c_void_p(Bhat.data_ptr())),
                "hom_update_coefficients")
        self._coef_refs = (Ahat, Bhat)
        _join(self.stream)

    def new_field(self, dual=False):
        t = torch.zeros(self.flen[int(dual)], dtype=torch.complex128, device=_dev())
        self.stream.wait_stream(torch.cuda.current_stream())
        return t

    def solve(self, dual=False, E=None, x0=None, tol=1e-6, maxit=10000, out=None, allow_not_converged=False):
        """Solve for loads E (nload x d; default the unit loads).  Returns
        (fields, infos) with fields a list of complex128 device tensors."""
        d = self.d
        E = np.eye(d) if E is None else np.atleast_2d(np.asarray(E, float))
        n = E.shape[0]
        fields = out if out is not None else [self.new_field(dual) for _ in range(n)]
        infos = (L.Info * n)()
        Ec = np.ascontiguousarray(E.reshape(-1))
        self.stream.wait_stream(torch.cuda.current_stream())
        x0p = _dptrs(x0) if x0 is not None else None
        f = L.load().hom_solve_dual if dual else L.load().hom_solve_primal
        st = f(self.h, n, Ec.ctypes.data_as(C.POINTER(C.c_double)), x0p, float(tol), int(maxit),
               _dptrs(fields), infos)
        L.check(st, "hom_solve_dual" if dual else "hom_solve_primal", allow_not_converged)
        info = [dict(iters=i.iters, status=i.status, rel_res_recur=i.rel_res_recur,
                     rel_res_true=i.rel_res_true, energy=i.energy) for i in infos]
        return fields, info

    def bounds(self, primal=None, dual=None):
        res = L.Result()
        self.stream.wait_stream(torch.cuda.current_stream())
        st = L.load().hom_bounds(self.h, _dptrs(primal) if primal is not None else None,
                                 _dptrs(dual) if dual is not None else None, C.byref(res))
        L.check(st, "hom_bounds")
        d = self.d
        g = lambda a: np.array(a[:d * d]).reshape(d, d)
        return dict(A_up=g(res.A_up), B_up=g(res.B_up), A_low=g(res.A_low), A_mean=g(res.A_mean), D=g(res.D))

    def apply(self, x, dual=False):
        y = self.new_field(dual)
        self.stream.wait_stream(torch.cuda.current_stream())
        L.check(L.load().hom_apply(self.h, int(dual), C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr())),
                "hom_apply")
        _join(self.stream)
        return y

    def dual_start(self, primal, Abar):
        """Dual start fields from the primal fields of the unit loads (hom_dual_start):
        J + j0 = A sum_a E_a (e_a + x^(a)) projected onto J_N, E = Abar^-1 J, for J = e_1..e_d."""
        d = self.d
        out = [self.new_field(True) for _ in range(d)]
        A = np.ascontiguousarray(np.asarray(Abar, float).reshape(d, d))
        self.stream.wait_stream(torch.cuda.current_stream())
        L.check(L.load().hom_dual_start(self.h, _dptrs(primal), A.ctypes.data_as(C.POINTER(C.c_double)),
                                        _dptrs(out)), "hom_dual_start")
        _join(self.stream)
        return out

    def profile_passes(self, dual=False, nload=None, reps=20):
        """Average per-launch milliseconds of the five operator passes (HIP events)."""
        ms = (C.c_double * 5)()
        n = self.d if nload is None else nload
        L.check(L.load().hom_profile_passes(self.h, int(dual), int(n), int(reps), ms), "hom_profile_passes")
        return dict(first=ms[0], mid_inv=ms[1], apply=ms[2], mid_fwd=ms[3], last=ms[4])

    @property
    def M(self):
        return self.Mq

    def field_to_grid(self, fields, dual=False):
        """Doubled-grid values (float32, [nload][d][*M]) of field vectors."""
        n = len(fields)
        out = torch.empty((n, self.d) + self.M, dtype=torch.float32, device=_dev())
        self.stream.wait_stream(torch.cuda.current_stream())
        L.check(L.load().hom_field_to_grid(self.h, int(dual), n, _dptrs(fields), C.c_void_p(out.data_ptr())),
                "hom_field_to_grid")
        _join(self.stream)
        return out

    def grid_to_field(self, grid, dual=False):
        """Admissible field vectors (projected on E_N / J_N) from doubled-grid fields [nload][d][*M]."""
        grid = grid.contiguous()
        n = grid.shape[0]
        out = [self.new_field(dual) for _ in range(n)]
        self.stream.wait_stream(torch.cuda.current_stream())
        L.check(L.load().hom_grid_to_field(self.h, int(dual), n, C.c_void_p(grid.data_ptr()), _dptrs(out)),
                "hom_grid_to_field")
        _join(self.stream)
        return out

    def net_input(self, out=None):
        """Network input channels [2][*M] (float32) of the coefficient of this problem."""
        if out is None:
            out = torch.empty((2,) + self.M, dtype=torch.float32, device=_dev())
        self.stream.wait_stream(torch.cuda.current_stream())
        L.check(L.load().hom_net_input(self.h, C.c_void_p(out.data_ptr())), "hom_net_input")
        _join(self.stream)
        return out

    def set_gani(self, AN, BN, grid=None):
        """GaNi mode (hom_set_gani) on the grid `grid` (default N; N + 1 per axis
        for the even grid whose reduced frequencies are Z_N): later solves use the
        point values AN, BN of A and A^-1 there (device float64 [ncoef][*grid])."""
        g = None if grid is None else (C.c_int32 * 3)(*(list(grid) + [1] * (3 - len(grid))))
        n = C.c_size_t()
        L.check(L.load().hom_gani_workspace_bytes(C.byref(self.desc), g, C.byref(n)), "hom_gani_workspace_bytes")
        self.gani_ws = torch.empty(n.value + 256, dtype=torch.uint8, device=_dev())
        off = (-self.gani_ws.data_ptr()) % 256
        self.stream.wait_stream(torch.cuda.current_stream())
        L.check(L.load().hom_set_gani(self.h, g, C.c_void_p(AN.data_ptr()), C.c_void_p(BN.data_ptr()),
                                      C.c_void_p(self.gani_ws.data_ptr() + off), n.value), "hom_set_gani")
        self.gani_grid = tuple(self.N if grid is None else grid)

    def set_gani_from_cell(self, cell, grid=None, closed=False):
        """GaNi mode with the point values of a cell on `grid` (sample_cell)."""
        grid = tuple(self.N if grid is None else grid)
        AN = sample_cell(cell, grid, self.ncoef, False, self.stream, closed)
        BN = sample_cell(cell, grid, self.ncoef, True, self.stream, closed)
        self.set_gani(AN, BN, grid)

    def clear_gani(self):
        L.check(L.load().hom_clear_gani(self.h), "hom_clear_gani")

    def gani_matrices(self, primal, dual=None):
        """A_{H,N} and B_{H,N} (hom_gani_matrices) of fields of the unit loads (either may be
        None: its matrix is NaN)."""
        A = (C.c_double * 9)()
        B = (C.c_double * 9)()
        self.stream.wait_stream(torch.cuda.current_stream())
        pp = _dptrs(primal) if primal is not None else None
        dp = _dptrs(dual) if dual is not None else None
        L.check(L.load().hom_gani_matrices(self.h, pp, dp, A, B), "hom_gani_matrices")
        d = self.d
        return np.array(A[:d * d]).reshape(d, d), np.array(B[:d * d]).reshape(d, d)

    def set_stop(self, rule="residual", etol=None, a_min=0.0, a_max=0.0):
        """Stopping rule of later solves (hom_problem_set_stop): "residual" (||r|| <= tol ||E||),
        "energy" (or an extrapolated energy tail below etol) or "guaranteed" (or the
        Gauss-Radau bound on the remaining energy below etol; a_min / a_max optionally
        bound the coefficient's eigenvalues)."""
        L.check(L.load().hom_problem_set_stop(self.h, _STOP_RULES[rule], float(etol or 0.0), float(a_min), float(a_max)),
                "hom_problem_set_stop")

    def tuning(self, dual=False, nload=None):
        """Tile shapes of this problem's FP32 solves (tuned now if not chosen yet)."""
        t = L.Tuning()
        n = self.d if nload is None else nload
        L.check(L.load().hom_problem_tuning(self.h, int(dual), int(n), C.byref(t)), "hom_problem_tuning")
        return _tuning_dict(t)

    def set_tiles(self, dual=False, nload=None, **shape):
        """Pin the tile shape of this problem's FP32 solves (keys as returned by tuning())."""
        n = self.d if nload is None else nload
        t = _tiles(**shape)
        L.check(L.load().hom_problem_set_tiles(self.h, int(dual), int(n), C.byref(t)), "hom_problem_set_tiles")

    def net_weights(self, out=None):
        """Energy weights [2][*M] (float32) of the primal and dual quadratures of this problem."""
        if out is None:
            out = torch.empty((2,) + self.M, dtype=torch.float32, device=_dev())
        self.stream.wait_stream(torch.cuda.current_stream())
        L.check(L.load().hom_net_weights(self.h, C.c_void_p(out.data_ptr())), "hom_net_weights")
        _join(self.stream)
        return out

    def solve_bounds(self, tol=1e-6, maxit=10000, allow_not_converged=False):
        xp, ip = self.solve(False, tol=tol, maxit=maxit, allow_not_converged=allow_not_converged)
        xd, idl = self.solve(True, tol=tol, maxit=maxit, allow_not_converged=allow_not_converged)
        b = self.bounds(xp, xd)
        b.update(info_primal=ip, info_dual=idl, fields_primal=xp, fields_dual=xd)
        return b


_STOP_RULES = {"residual": 0, "energy": 1, "guaranteed": 2, "gap": 3}


def set_tuning(on=True):
    """Tile tuning of the FP32 passes for geometries not seen yet (hom_set_tuning)."""
    L.check(L.load().hom_set_tuning(1 if on else 0), "hom_set_tuning")


def tune_cache_load(path, arch=None):
    """Merge the tuner choices of `arch` (default: the current device's) from a
    JSON-lines file into the process cache (hom_tune_cache_load); returns their count."""
    n = C.c_int32()
    L.check(L.load().hom_tune_cache_load(str(path).encode(), None if arch is None else arch.encode(), C.byref(n)),
            "hom_tune_cache_load")
    return n.value


def tune_cache_save(path, arch=None):
    """Write the process's tuner choices to a JSON-lines file (hom_tune_cache_save)."""
    L.check(L.load().hom_tune_cache_save(str(path).encode(), None if arch is None else arch.encode()),
            "hom_tune_cache_save")


def tune_cache_clear():
    L.check(L.load().hom_tune_cache_clear(), "hom_tune_cache_clear")


def _join(stream):
    """Order later work of the caller's current stream after what was queued on
    `stream`: outputs of an asynchronous call are then ready for it, and inputs
    it frees stay untouched until the call has read them."""
    torch.cuda.current_stream().wait_stream(stream)


def _tuning_dict(t):
    return dict(row_pairs=t.row_pairs, row_threads=t.row_threads, apply_points=t.apply_points,
                apply_half_exchange=t.apply_half_exchange, apply_all_packs=t.apply_all_packs,
                candidates=t.candidates, row_ms=t.row_ms, apply_ms=t.apply_ms)


def _tiles(row_pairs=0, row_threads=0, apply_points=0, apply_half_exchange=0, apply_all_packs=0, **_):
    t = L.Tuning()
    t.row_pairs, t.row_threads = int(row_pairs), int(row_threads)
    t.apply_points, t.apply_half_exchange = int(apply_points), int(apply_half_exchange)
    t.apply_all_packs = int(apply_all_packs)
    return t


def _result_dict(res, d):
    g = lambda a: np.array(a[:d * d]).reshape(d, d)
    return dict(A_up=g(res.A_up), B_up=g(res.B_up), A_low=g(res.A_low), A_mean=g(res.A_mean), D=g(res.D))


class Batch:
    """Problems of one size class (same d, N, Y, precision, ncoef, max_loads,
    stream) solved in lockstep: each CG kernel launch covers all of them."""

    def __init__(self, problems):
        lib = L.load()
        self.problems = list(problems)
        n = len(self.problems)
        p0 = self.problems[0]
        self.d, self.N, self.stream = p0.d, p0.N, p0.stream
        nb = C.c_size_t()
        L.check(lib.hom_batch_workspace_bytes(n, C.byref(nb)), "hom_batch_workspace_bytes")
        self.ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=_dev())
        ptr = self.ws.data_ptr() + ((-self.ws.data_ptr()) % 256)
        hs = (C.c_void_p * n)(*[p.h.value for p in self.problems])
        h = C.c_void_p()
        L.check(lib.hom_batch_create(hs, n, C.c_void_p(ptr), nb.value, C.byref(h)), "hom_batch_create")
        self.h = h

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            try:
                L.load().hom_batch_destroy(h)
            except Exception:
                pass
            self.h = None

    def new_fields(self, dual, nl):
        """Zero fields [[nl tensors] per problem]: views of one allocation."""
        p0 = self.problems[0]
        big = torch.zeros((len(self.problems) * nl, p0.flen[int(dual)]), dtype=torch.complex128, device=_dev())
        self.stream.wait_stream(torch.cuda.current_stream())
        return [[big[i * nl + l] for l in range(nl)] for i in range(len(self.problems))]

    def solve(self, dual=False, E=None, x0=None, tol=1e-6, maxit=10000, out=None, allow_not_converged=False):
        d, n = self.d, len(self.problems)
        E = np.eye(d) if E is None else np.atleast_2d(np.asarray(E, float))
        nl = E.shape[0]
        fields = out if out is not None else self.new_fields(dual, nl)
        flat = [f for fs in fields for f in fs]
        infos = (L.Info * (n * nl))()
        Ec = np.ascontiguousarray(E.reshape(-1))
        self.stream.wait_stream(torch.cuda.current_stream())
        x0p = _dptrs([t for ts in x0 for t in ts]) if x0 is not None else None
        st = L.load().hom_batch_solve(self.h, int(dual), nl, Ec.ctypes.data_as(C.POINTER(C.c_double)), x0p,
                                      float(tol), int(maxit), _dptrs(flat), infos)
        L.check(st, "hom_batch_solve", allow_not_converged)
        info = [[dict(iters=infos[i * nl + l].iters, status=infos[i * nl + l].status,
                      rel_res_recur=infos[i * nl + l].rel_res_recur, rel_res_true=infos[i * nl + l].rel_res_true,
                      energy=infos[i * nl + l].energy)
                 for l in range(nl)] for i in range(n)]
        return fields, info

    def bounds(self, primal=None, dual=None):
        n, d = len(self.problems), self.d
        res = (L.Result * n)()
        self.stream.wait_stream(torch.cuda.current_stream())
        pp = _dptrs([t for ts in primal for t in ts]) if primal is not None else None
        dp = _dptrs([t for ts in dual for t in ts]) if dual is not None else None
        L.check(L.load().hom_batch_bounds(self.h, pp, dp, res), "hom_batch_bounds")
        return [_result_dict(res[i], d) for i in range(n)]

    def set_stop(self, rule="residual", etol=None, a_min=0.0, a_max=0.0):
        """Stopping rule of later solves (hom_batch_set_stop): "residual" (||r|| <= tol ||E||),
        "energy" (or an extrapolated energy tail below etol), "guaranteed" (or the
        Gauss-Radau bound on the remaining energy below etol) or "gap" (solve_pair /
        solve_bounds only: or each side's remaining error below etol times a
        guaranteed lower bound on the converged gap of its bound); a_min / a_max
        optionally bound the coefficient's eigenvalues."""
        L.check(L.load().hom_batch_set_stop(self.h, _STOP_RULES[rule], float(etol or 0.0), float(a_min), float(a_max)),
                "hom_batch_set_stop")

    def tuning(self, dual=False, nload=None):
        """Tile shapes of this batch's FP32 solves (tuned now if not chosen yet)."""
        t = L.Tuning()
        n = self.d if nload is None else nload
        L.check(L.load().hom_batch_tuning(self.h, int(dual), int(n), C.byref(t)), "hom_batch_tuning")
        return _tuning_dict(t)

    def set_tiles(self, dual=False, nload=None, **shape):
        """Pin the tile shape of this batch's FP32 solves (keys as returned by tuning())."""
        n = self.d if nload is None else nload
        t = _tiles(**shape)
        L.check(L.load().hom_batch_set_tiles(self.h, int(dual), int(n), C.byref(t)), "hom_batch_set_tiles")

    def set_timing(self, on=True):
        L.check(L.load().hom_batch_set_timing(self.h, int(bool(on))), "hom_batch_set_timing")

    def get_timing(self):
        """Average milliseconds per launch of each pass over the timed solves, and launch counts."""
        ms = (C.c_double * 5)()
        cnt = (C.c_int64 * 5)()
        L.check(L.load().hom_batch_get_timing(self.h, ms, cnt), "hom_batch_get_timing")
        names = ["first", "mid_inv", "apply", "mid_fwd", "last"]
        return {n: (ms[i] / cnt[i] if cnt[i] else 0.0) for i, n in enumerate(names)}, \
            {n: int(cnt[i]) for i, n in enumerate(names)}

    def profile_passes(self, dual=False, nload=None, reps=20):
        ms = (C.c_double * 5)()
        n = self.d if nload is None else nload
        L.check(L.load().hom_batch_profile_passes(self.h, int(dual), int(n), int(reps), ms),
                "hom_batch_profile_passes")
        return dict(first=ms[0], mid_inv=ms[1], apply=ms[2], mid_fwd=ms[3], last=ms[4])

    def _check_span(self, t, stride, block):
        """The n strided blocks of `block` floats from t's first element stay inside t's storage."""
        need = (len(self.problems) - 1) * stride + block
        end = t.untyped_storage().data_ptr() + t.untyped_storage().nbytes()
        if t.dtype != torch.float32 or t.data_ptr() + 4 * need > end:
            raise ValueError(f"tensor too small for {len(self.problems)} blocks of {block} floats at stride {stride}")

    def field_to_grid(self, fields, dual, out, stride=None):
        """Doubled-grid values (FP32) of fields [[d tensors] per problem] into out, cell i's
        [nload][d][*M] block at float offset i * stride (hom_batch_field_to_grid)."""
        nl = len(fields[0])
        Mt = int(np.prod(self.problems[0].M))
        stride = nl * self.d * Mt if stride is None else int(stride)
        self._check_span(out, stride, nl * self.d * Mt)
        flat = [t for ts in fields for t in ts]
        self.stream.wait_stream(torch.cuda.current_stream())
        L.check(L.load().hom_batch_field_to_grid(self.h, int(dual), nl, _dptrs(flat), C.c_void_p(out.data_ptr()),
                                                 stride), "hom_batch_field_to_grid")
        _join(self.stream)
        return out

    def grid_to_field(self, grids, dual, nload=None, stride=None):
        """Admissible fields (projected on E_N / J_N) of every problem from doubled-grid
        fields, cell i's [nload][d][*M] block at float offset i * stride of the tensor
        `grids` (hom_batch_grid_to_field); returns [[nload tensors] per problem]."""
        nl = self.d if nload is None else nload
        Mt = int(np.prod(self.problems[0].M))
        stride = nl * self.d * Mt if stride is None else int(stride)
        self._check_span(grids, stride, nl * self.d * Mt)
        out = self.new_fields(dual, nl)
        flat = [t for ts in out for t in ts]
        self.stream.wait_stream(torch.cuda.current_stream())
        L.check(L.load().hom_batch_grid_to_field(self.h, int(dual), nl, C.c_void_p(grids.data_ptr()), stride,
                                                 _dptrs(flat)), "hom_batch_grid_to_field")
        _join(self.stream)
        return out

    def net_input(self, out, stride=None, weights=False):
        """Network input channels (or energy weights) [2][*M] of every problem into out,
        cell i's block at float offset i * stride (hom_batch_net_input)."""
        Mt = int(np.prod(self.problems[0].M))
        stride = 2 * Mt if stride is None else int(stride)
        self._check_span(out, stride, 2 * Mt)
        self.stream.wait_stream(torch.cuda.current_stream())
        L.check(L.load().hom_batch_net_input(self.h, C.c_void_p(out.data_ptr()), stride, int(bool(weights))),
                "hom_batch_net_input")
        _join(self.stream)
        return out

    def update_coefficients(self, coefs):
        """New coefficients [(Ahat, Bhat)] for every problem of the batch (hom_batch_update_coefficients)."""
        n = len(self.problems)
        assert len(coefs) == n
        A = (C.c_void_p * n)(*[c[0].data_ptr() for c in coefs])
        B = (C.c_void_p * n)(*[c[1].data_ptr() for c in coefs])
        self.stream.wait_stream(torch.cuda.current_stream())
        L.check(L.load().hom_batch_update_coefficients(self.h, A, B), "hom_batch_update_coefficients")
        for p, c in zip(self.problems, coefs):
            p._coef_refs = (c[0], c[1])   # the setup reads them asynchronously
        _join(self.stream)

    def _fields(self, dual, nl):
        """Output fields of solve_bounds, allocated once per (dual, loads) and reused."""
        key = (bool(dual), nl)
        cache = self.__dict__.setdefault("_field_cache", {})
        if key not in cache:
            cache[key] = self.new_fields(dual, nl)
        return cache[key]

    def solve_pair(self, E=None, tol=1e-6, maxit=10000, out_primal=None, out_dual=None, allow_not_converged=False,
                   x0_primal=None, x0_dual=None):
        """Primal and dual solves of the same loads side by side (hom_batch_solve_pair);
        x0_primal / x0_dual: optional starting fields [[nload tensors] per problem]."""
        d, n = self.d, len(self.problems)
        E = np.eye(d) if E is None else np.atleast_2d(np.asarray(E, float))
        nl = E.shape[0]
        fp = out_primal if out_primal is not None else self.new_fields(False, nl)
        fd = out_dual if out_dual is not None else self.new_fields(True, nl)
        ip, idl = (L.Info * (n * nl))(), (L.Info * (n * nl))()
        Ec = np.ascontiguousarray(E.reshape(-1))
        self.stream.wait_stream(torch.cuda.current_stream())
        x0p = _dptrs([t for ts in x0_primal for t in ts]) if x0_primal is not None else None
        x0d = _dptrs([t for ts in x0_dual for t in ts]) if x0_dual is not None else None
        st = L.load().hom_batch_solve_pair(self.h, nl, Ec.ctypes.data_as(C.POINTER(C.c_double)), x0p, x0d,
                                           float(tol), int(maxit), _dptrs([t for ts in fp for t in ts]),
                                           _dptrs([t for ts in fd for t in ts]), ip, idl)
        L.check(st, "hom_batch_solve_pair", allow_not_converged)
        conv = lambda infos: [[dict(iters=infos[i * nl + l].iters, status=infos[i * nl + l].status,
                                    rel_res_recur=infos[i * nl + l].rel_res_recur,
                                    rel_res_true=infos[i * nl + l].rel_res_true,
                                    energy=infos[i * nl + l].energy) for l in range(nl)]
                              for i in range(n)]
        return fp, conv(ip), fd, conv(idl)

    def solve_bounds(self, tol=1e-6, maxit=10000, allow_not_converged=False, x0_primal=None, x0_dual=None):
        """Primal and dual solves of the unit loads (side by side, optionally from starting
        fields) and the bounds of every problem.  The fields live in buffers owned by the
        batch and are overwritten by the next call."""
        d, n = self.d, len(self.problems)
        fp, fd = self._fields(False, d), self._fields(True, d)
        ip, idl = (L.Info * (n * d))(), (L.Info * (n * d))()
        res = (L.Result * n)()
        self.stream.wait_stream(torch.cuda.current_stream())
        x0p = _dptrs([t for ts in x0_primal for t in ts]) if x0_primal is not None else None
        x0d = _dptrs([t for ts in x0_dual for t in ts]) if x0_dual is not None else None
        st = L.load().hom_batch_solve_bounds(self.h, x0p, x0d, float(tol), int(maxit),
                                             _dptrs([t for ts in fp for t in ts]), _dptrs([t for ts in fd for t in ts]),
                                             ip, idl, res)
        L.check(st, "hom_batch_solve_bounds", allow_not_converged)
        conv = lambda infos, i: [dict(iters=infos[i * d + l].iters, status=infos[i * d + l].status,
                                      rel_res_recur=infos[i * d + l].rel_res_recur,
                                      rel_res_true=infos[i * d + l].rel_res_true,
                                      energy=infos[i * d + l].energy) for l in range(d)]
        out = [_result_dict(res[i], d) for i in range(n)]
        for i, r in enumerate(out):
            r.update(info_primal=conv(ip, i), info_dual=conv(idl, i))
        return out


class Group:
    """Batches (size classes) whose primal and dual solves of the unit loads run
    together from one captured HIP graph (hom_group_solve_pair)."""

    def __init__(self, batches):
        self.batches = list(batches)
        hs = (C.c_void_p * len(self.batches))(*[b.h.value for b in self.batches])
        h = C.c_void_p()
        L.check(L.load().hom_group_create(hs, len(self.batches), C.byref(h)), "hom_group_create")
        self.h = h

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            try:
                L.load().hom_group_destroy(h)
            except Exception:
                pass
            self.h = None

    def set_launch(self, mode):
        """"graph": one captured graph advances every solve per launch; "streams": every
        solve replays its own chunk graph, one host loop polls them all (hom_group_set_launch)."""
        L.check(L.load().hom_group_set_launch(self.h, {"graph": 0, "streams": 1}[mode]), "hom_group_set_launch")

    def solve_bounds(self, tol=1e-6, maxit=10000, allow_not_converged=False, fused=True):
        """Bounds of every problem of every batch (a list per batch), fields in the batches' buffers.
        fused: one call (hom_group_solve_bounds: each side's bound passes start when that side
        stops); else hom_group_solve_pair followed by hom_batch_bounds per batch (same results)."""
        fp, fd, counts = [], [], []
        for b in self.batches:
            xp, xd = b._fields(False, b.d), b._fields(True, b.d)
            fp += [t for ts in xp for t in ts]
            fd += [t for ts in xd for t in ts]
            counts.append(len(b.problems) * b.d)
        n = sum(counts)
        ip, idl = (L.Info * n)(), (L.Info * n)()
        for b in self.batches:
            b.stream.wait_stream(torch.cuda.current_stream())
        if fused:
            res_all = (L.Result * sum(len(b.problems) for b in self.batches))()
            st = L.load().hom_group_solve_bounds(self.h, float(tol), int(maxit), _dptrs(fp), _dptrs(fd),
                                                 C.cast(ip, C.c_void_p), C.cast(idl, C.c_void_p), res_all)
            L.check(st, "hom_group_solve_bounds", allow_not_converged)
        else:
            st = L.load().hom_group_solve_pair(self.h, float(tol), int(maxit), _dptrs(fp), _dptrs(fd),
                                               C.cast(ip, C.c_void_p), C.cast(idl, C.c_void_p))
            L.check(st, "hom_group_solve_pair", allow_not_converged)
        out, off, roff = [], 0, 0
        for b, cnt in zip(self.batches, counts):
            d = b.d
            conv = lambda infos: [[dict(iters=infos[off + i * d + l].iters, status=infos[off + i * d + l].status,
                                        rel_res_recur=infos[off + i * d + l].rel_res_recur,
                                        rel_res_true=infos[off + i * d + l].rel_res_true,
                                        energy=infos[off + i * d + l].energy) for l in range(d)]
                                  for i in range(len(b.problems))]
            if fused:
                res = [_result_dict(res_all[roff + i], d) for i in range(len(b.problems))]
            else:
                res = b.bounds(b._fields(False, d), b._fields(True, d))
            for r, a, c in zip(res, conv(ip), conv(idl)):
                r.update(info_primal=a, info_dual=c)
            out.append(res)
            off += cnt
            roff += len(b.problems)
        return out


def problem_from_cell(cell, N, precision="mixed", max_loads=None, stream=None, M=None):
    """Problem of a cell on the grid N; M: quadrature grid (default 2N - 1)."""
    N = tuple(int(n) for n in (N if np.iterable(N) else [N] * cell.d))
    if M is not None:
        M = tuple(int(m) for m in (M if np.iterable(M) else [M] * cell.d))
    Ah, Bh, nc = coef_from_cell(cell, N, stream=stream, M=M)
    pb = Problem(cell.d, N, cell.Y, Ah, Bh, precision=precision, ncoef=nc, max_loads=max_loads, stream=stream, M=M)
    return pb
