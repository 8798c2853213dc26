"""Learned initial guess for the CG solves (binding of hom_unet_* and the
grid transfers of include/hom.h).

A periodic U-Net maps the doubled-grid coefficient of a cell (two channels:
a/<a> and a clipped log) to the primal and dual fluctuation fields of the d
unit loads on the doubled grid (2 d^2 channels, field component gamma of load
alpha).  The solver turns a prediction into an admissible starting field with
hom_grid_to_field (truncation to Z_N and projection onto E_N or J_N), so the
bounds stay guaranteed whatever the network outputs; the network only changes
the number of CG iterations.

Training data are solver fields: the converged primal/dual fields of
generated cells, brought to the doubled grid with hom_field_to_grid.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np
import torch

from . import _lib as L
from . import api


def layer_shapes(d, levels, base, cin, cout):
    """(cin, cout, kernel) of every conv layer, in the order of the flat parameter array."""
    out, prev = [], cin
    for l in range(levels):
        c = base << l
        out += [(prev, c, 3), (c, c, 3)]
        prev = c
    for l in range(levels - 2, -1, -1):
        c, cu = base << l, base << (l + 1)
        out += [(cu, c, 3), (2 * c, c, 3), (c, c, 3)]
    out.append((base, cout, 1))
    return out


class UNet:
    def __init__(self, d, size, levels=4, base=32, cin=2, cout=None, batch=16, stream=None):
        lib = L.load()
        self.d, self.levels, self.base, self.cin = d, levels, base, cin
        self.cout = 2 * d * d if cout is None else cout
        self.size = tuple(int(s) for s in size)
        self.batch = batch
        self.stream = stream if stream is not None else torch.cuda.Stream()
        ds = L.UNetDesc()
        ds.d, ds.levels, ds.base, ds.cin, ds.cout, ds.batch = d, levels, base, cin, self.cout, batch
        for a in range(3):
            ds.size[a] = self.size[a] if a < len(self.size) else 1
        self.desc = ds
        npar, work = C.c_size_t(), C.c_size_t()
        L.check(lib.hom_unet_sizes(C.byref(ds), C.byref(npar), C.byref(work)), "hom_unet_sizes")
        self.nparams = npar.value
        dev = api._dev()
        self.params = torch.zeros(self.nparams, dtype=torch.float32, device=dev)
        self.grads = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.work = torch.empty(work.value + 256, dtype=torch.uint8, device=dev)
        ptr = self.work.data_ptr() + ((-self.work.data_ptr()) % 256)
        h = C.c_void_p()
        self.stream.wait_stream(torch.cuda.current_stream())
        L.check(lib.hom_unet_create(C.byref(ds), C.c_void_p(self.params.data_ptr()),
                                    C.c_void_p(self.grads.data_ptr()), C.c_void_p(self.m.data_ptr()),
                                    C.c_void_p(self.v.data_ptr()), C.c_void_p(ptr), work.value,
                                    C.c_void_p(self.stream.cuda_stream), C.byref(h)), "hom_unet_create")
        self.h = h
        self.step = 0
        self.out = torch.empty((batch, self.cout) + self.size, dtype=torch.float32, device=dev)

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            try:
                L.load().hom_unet_destroy(h)
            except Exception:
                pass
            self.h = None

    def init_params(self, seed=0):
        """He-normal weights, zero biases (host RNG, then copied to the device)."""
        rng = np.random.default_rng(seed)
        chunks = []
        for ci, co, ks in layer_shapes(self.d, self.levels, self.base, self.cin, self.cout):
            fan_in = ci * ks ** self.d
            std = math.sqrt(2.0 / fan_in) if ks == 3 else math.sqrt(1.0 / fan_in)
            chunks.append(rng.standard_normal(co * ci * ks ** self.d) * std)
            chunks.append(np.zeros(co))
        theta = np.concatenate(chunks).astype(np.float32)
        assert theta.size == self.nparams
        self.set_params(torch.from_numpy(theta))
        self.m.zero_()
        self.v.zero_()
        self.step = 0

    def set_params(self, theta):
        self.params.copy_(theta.to(self.params.device, torch.float32))

    def forward(self, x, out=None):
        """x: [batch, cin, *size] float32 on the device -> [batch, cout, *size] (out, or the
        network's output tensor)."""
        x = x.contiguous()
        assert tuple(x.shape) == (self.batch, self.cin) + self.size
        o = self.out if out is None else out
        self.stream.wait_stream(torch.cuda.current_stream())
        L.check(L.load().hom_unet_forward(self.h, C.c_void_p(x.data_ptr()), C.c_void_p(o.data_ptr())),
                "hom_unet_forward")
        torch.cuda.current_stream().wait_stream(self.stream)
        return o

    def forward_samples(self, X, idx, out=None):
        """Forward of the samples X[idx] (X: [n, cin, *size], contiguous) without a
        separate gather (hom_unet_forward_samples)."""
        o = self.out if out is None else out
        assert tuple(X.shape[1:]) == (self.cin,) + self.size and len(idx) == self.batch
        assert 0 <= min(idx) and max(idx) < X.shape[0]
        self.stream.wait_stream(torch.cuda.current_stream())
        L.check(L.load().hom_unet_forward_samples(self.h, sample_ptrs(X, idx), C.c_void_p(o.data_ptr())),
                "hom_unet_forward_samples")
        torch.cuda.current_stream().wait_stream(self.stream)
        return o

    def loss(self, target, weight=None):
        """(Weighted) mean squared error of the last output; weight [batch][wch][*size] or None."""
        target = target.contiguous()
        val = C.c_double()
        self.stream.wait_stream(torch.cuda.current_stream())
        if weight is None:
            L.check(L.load().hom_unet_loss(self.h, C.c_void_p(target.data_ptr()), C.byref(val)), "hom_unet_loss")
        else:
            weight = weight.contiguous()
            L.check(L.load().hom_unet_loss_weighted(self.h, C.c_void_p(target.data_ptr()),
                                                    C.c_void_p(weight.data_ptr()), int(weight.shape[1]),
                                                    C.byref(val)), "hom_unet_loss_weighted")
        return val.value

    def loss_samples(self, Y, idx, W=None):
        """Loss of the last output against the samples Y[idx] (and weights W[idx])
        without a separate gather (hom_unet_loss_samples)."""
        val = C.c_double()
        assert tuple(Y.shape[1:]) == (self.cout,) + self.size and len(idx) == self.batch
        assert 0 <= min(idx) and max(idx) < Y.shape[0]
        assert W is None or (tuple(W.shape[2:]) == self.size and W.shape[0] == Y.shape[0])
        self.stream.wait_stream(torch.cuda.current_stream())
        wp = sample_ptrs(W, idx) if W is not None else None
        L.check(L.load().hom_unet_loss_samples(self.h, sample_ptrs(Y, idx), wp, 1 if W is None else int(W.shape[1]),
                                               C.byref(val)), "hom_unet_loss_samples")
        return val.value

    def backward(self, gout=None):
        ptr = C.c_void_p(gout.contiguous().data_ptr()) if gout is not None else None
        self.stream.wait_stream(torch.cuda.current_stream())
        L.check(L.load().hom_unet_backward(self.h, ptr), "hom_unet_backward")
        torch.cuda.current_stream().wait_stream(self.stream)
        return self.grads

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step += 1
        L.check(L.load().hom_unet_adam(self.h, float(lr), float(beta1), float(beta2), float(eps), self.step),
                "hom_unet_adam")

    def state(self):
        return dict(params=self.params.cpu(), m=self.m.cpu(), v=self.v.cpu(), step=self.step,
                    arch=dict(d=self.d, levels=self.levels, base=self.base, cin=self.cin, cout=self.cout))

    def load_state(self, st):
        self.params.copy_(st["params"])
        self.m.copy_(st["m"])
        self.v.copy_(st["v"])
        self.step = int(st["step"])


# ---------------------------------------------------------------- data and training
def sample_ptrs(T, idx):
    """Device pointers of the samples T[i], i in idx (T contiguous, sample-major)."""
    assert T.is_contiguous()
    step = T[0].numel() * T.element_size()
    base = T.data_ptr()
    return (C.c_void_p * len(idx))(*[base + int(i) * step for i in idx])


def _class_batch(cells, N, precision, stream):
    d = cells[0].d
    nc = max(api.cell_ncoef(c) for c in cells)
    coefs = [api.coef_from_cell(c, N, ncoef=nc, stream=stream)[:2] for c in cells]
    probs = [api.Problem(d, N, cells[0].Y, Ah, Bh, precision=precision, ncoef=nc, stream=stream)
             for Ah, Bh in coefs]
    return probs, api.Batch(probs), nc


def solver_samples(cells, N, tol=1e-6, precision="mixed", chunk=64, stream=None, targets="grid"):
    """Network inputs and targets from solver fields for cells of one size class
    (same d, N and cell size).

    The cells are solved in lockstep batches of up to `chunk` (primal and dual side
    by side), the problem handles of a batch being re-used through new
    coefficients; inputs and targets of a batch are written by one call each.
    Returns (inputs [n, 2, *M], targets, energy weights [n, 2, *M], iterations
    [n, 2 d]).  targets = "grid": the fields on the doubled grid [n, 2 d^2, *M]
    (primal loads then dual loads); targets = "spectra": the solver fields
    themselves, a pair of complex tensors [n, d, len] (primal, dual), to be
    brought to the grid per minibatch (grid_targets) where the grids of every
    sample would not fit."""
    d = cells[0].d
    N = tuple(int(n) for n in (N if np.iterable(N) else [N] * d))
    M = tuple(2 * n - 1 for n in N)
    Mt = int(np.prod(M))
    stream = stream if stream is not None else torch.cuda.Stream()
    n = len(cells)
    dev = api._dev()
    X = torch.empty((n, 2) + M, dtype=torch.float32, device=dev)
    W = torch.empty((n, 2) + M, dtype=torch.float32, device=dev)
    if targets == "grid":
        Yt = torch.empty((n, 2 * d * d) + M, dtype=torch.float32, device=dev)
    else:
        fl = [api.field_len(d, N, k, cells[0].Y) for k in (0, 1)]
        Yt = (torch.empty((n, d, fl[0]), dtype=torch.complex128, device=dev),
              torch.empty((n, d, fl[1]), dtype=torch.complex128, device=dev))
    iters = np.zeros((n, 2 * d), dtype=np.int64)
    probs = batch = None
    nc0 = None
    for i0 in range(0, n, chunk):
        part = cells[i0:i0 + chunk]
        nc = max(api.cell_ncoef(c) for c in part)
        if probs is None or len(probs) != len(part) or nc != nc0:
            probs, batch, nc0 = _class_batch(part, N, precision, stream)
        else:
            batch.update_coefficients([api.coef_from_cell(c, N, ncoef=nc, stream=stream)[:2] for c in part])
        if targets == "grid":
            xp, ip, xd, idl = batch.solve_pair(tol=tol)
        else:
            m = len(part)
            out_p = [[Yt[0][i0 + j, a] for a in range(d)] for j in range(m)]
            out_d = [[Yt[1][i0 + j, a] for a in range(d)] for j in range(m)]
            xp, ip, xd, idl = batch.solve_pair(tol=tol, out_primal=out_p, out_dual=out_d)
        batch.net_input(X[i0:])
        batch.net_input(W[i0:], weights=True)
        if targets == "grid":
            stride = 2 * d * d * Mt
            batch.field_to_grid(xp, False, Yt[i0:], stride)
            batch.field_to_grid(xd, True, Yt[i0:, d * d:], stride)
        iters[i0:i0 + len(part)] = [[r["iters"] for r in a + b] for a, b in zip(ip, idl)]
    torch.cuda.synchronize()
    return X, Yt, W, iters


def grid_targets(geo, spectra, idx, out):
    """Targets [len(idx), 2 d^2, *M] of stored solver fields (solver_samples with
    targets="spectra") on the doubled grid; geo: a Batch of len(idx) problems of
    the class (only its geometry is used)."""
    d = geo.d
    Mt = int(np.prod(geo.problems[0].M))
    stride = 2 * d * d * Mt
    P, D = spectra
    geo.field_to_grid([[P[i, a] for a in range(d)] for i in idx], False, out, stride)
    geo.field_to_grid([[D[i, a] for a in range(d)] for i in idx], True, out[:, d * d:], stride)
    return out


def train(net, X, Y, steps, lr=1e-3, seed=0, log_every=0, lr_final=None, W=None, geo=None, warmup=0):
    """Adam on random minibatches of (X, Y) (linear warm-up over `warmup` steps, then
    cosine decay to lr_final); returns the loss history.
    Minibatches are read through sample pointers (no gather).  Y: target grids, or
    stored solver fields (a pair of spectra tensors) with geo, a Batch of net.batch
    problems of the class, bringing them to the grid per step.  With W (energy
    weights, one channel per half of the outputs) the loss is the weighted squared
    error, an approximation of the energy norms of the errors."""
    rng = np.random.default_rng(seed)
    n = X.shape[0]
    hist = []
    lr_final = lr if lr_final is None else lr_final
    tgt = None
    if isinstance(Y, tuple):
        assert geo is not None and len(geo.problems) == net.batch
        tgt = torch.empty((net.batch, net.cout) + net.size, dtype=torch.float32, device=X.device)
    for s in range(steps):
        idx = rng.integers(0, n, net.batch)
        net.forward_samples(X, idx)
        if tgt is None:
            loss = net.loss_samples(Y, idx, W)
        else:
            grid_targets(geo, Y, idx, tgt)
            loss = net.loss(tgt)
        net.backward()
        t = s / max(steps - 1, 1)
        rate = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * t))
        if s < warmup:
            rate *= (s + 1) / warmup
        net.adam(lr=rate)
        hist.append(loss)
        if log_every and (s % log_every == 0 or s == steps - 1):
            print(f"[train] step {s} loss {loss:.5g}", flush=True)
    return hist


def predict_x0(net, batch):
    """Admissible initial fields, primal and dual, d unit loads each, for every
    problem of a batch: the network inputs of all cells in one call, the network
    (a captured graph) over minibatches without host synchronisation, and the
    projection of all predictions onto E_N / J_N by one call per side
    (hom_batch_grid_to_field).  Returns (primal, dual): [[d fields] per problem]."""
    d, M = batch.d, batch.problems[0].M
    Mt = int(np.prod(M))
    n, B = len(batch.problems), net.batch
    npad = -(-n // B) * B
    dev = api._dev()
    X = torch.zeros((npad, 2) + M, dtype=torch.float32, device=dev)
    G = torch.empty((npad, net.cout) + M, dtype=torch.float32, device=dev)
    batch.net_input(X)
    for i0 in range(0, npad, B):
        net.forward(X[i0:i0 + B], out=G[i0:i0 + B])
    stride = net.cout * Mt
    x0p = batch.grid_to_field(G, False, stride=stride)
    x0d = batch.grid_to_field(G[:, d * d:], True, stride=stride)
    return x0p, x0d
