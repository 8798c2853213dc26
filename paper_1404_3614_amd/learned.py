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

    def forward(self, x):
        """x: [batch, cin, *size] float32 on the device -> [batch, cout, *size]."""
        x = x.contiguous()
        assert tuple(x.shape) == (self.batch, self.cin) + self.size
        self.stream.wait_stream(torch.cuda.current_stream())
        L.check(L.load().hom_unet_forward(self.h, C.c_void_p(x.data_ptr()), C.c_void_p(self.out.data_ptr())),
                "hom_unet_forward")
        torch.cuda.current_stream().wait_stream(self.stream)
        return self.out

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
def solver_samples(cells, N, tol=1e-6, precision="mixed", chunk=64, stream=None):
    """Network inputs and targets from solver fields for cells of one size class
    (same d, N and cell size, isotropic or not alike).

    The cells are solved in lockstep batches of up to `chunk`, the problem
    handles of a batch being re-used through new coefficients.  Returns
    (inputs [n, 2, *M], targets [n, 2 d^2, *M], energy weights [n, 2, *M],
    iterations [n, 2 d])."""
    d = cells[0].d
    N = tuple(int(n) for n in (N if np.iterable(N) else [N] * d))
    M = tuple(2 * n - 1 for n in N)
    stream = stream if stream is not None else torch.cuda.Stream()
    n = len(cells)
    X = torch.empty((n, 2) + M, dtype=torch.float32, device=api._dev())
    Yt = torch.empty((n, 2 * d * d) + M, dtype=torch.float32, device=api._dev())
    W = torch.empty((n, 2) + M, dtype=torch.float32, device=api._dev())
    iters = np.zeros((n, 2 * d), dtype=np.int64)
    probs, batch, nc0 = None, None, None
    for i0 in range(0, n, chunk):
        part = cells[i0:i0 + chunk]
        nc = max(api.cell_ncoef(c) for c in part)
        coefs = [api.coef_from_cell(c, N, ncoef=nc, stream=stream)[:2] for c in part]
        if probs is None or len(probs) != len(part) or nc != nc0:
            probs = [api.Problem(d, N, part[0].Y, Ah, Bh, precision=precision, ncoef=nc, stream=stream)
                     for Ah, Bh in coefs]
            batch, nc0 = api.Batch(probs), nc
        else:
            for p, (Ah, Bh) in zip(probs, coefs):
                p.update_coefficients(Ah, Bh)
        xp, ip = batch.solve(False, tol=tol)
        xd, idl = batch.solve(True, tol=tol)
        for j, p in enumerate(probs):
            p.net_input(out=X[i0 + j])
            p.net_weights(out=W[i0 + j])
            Yt[i0 + j, :d * d] = p.field_to_grid(xp[j], dual=False).reshape((d * d,) + M)
            Yt[i0 + j, d * d:] = p.field_to_grid(xd[j], dual=True).reshape((d * d,) + M)
            iters[i0 + j] = [r["iters"] for r in ip[j] + idl[j]]
        torch.cuda.synchronize()
    return X, Yt, W, iters


def train(net, X, Y, steps, lr=1e-3, seed=0, log_every=0, lr_final=None, W=None):
    """Adam on random minibatches of (X, Y) (cosine decay to lr_final); returns the loss history.
    With W (energy weights, one channel per half of the outputs) the loss is the
    weighted squared error, an approximation of the energy norms of the errors."""
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    n = X.shape[0]
    hist = []
    lr_final = lr if lr_final is None else lr_final
    for s in range(steps):
        idx = torch.randint(0, n, (net.batch,), generator=g).to(X.device)
        net.forward(X[idx])
        loss = net.loss(Y[idx], None if W is None else W[idx])
        net.backward()
        t = s / max(steps - 1, 1)
        net.adam(lr=lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * t)))
        hist.append(loss)
        if log_every and (s % log_every == 0 or s == steps - 1):
            print(f"[train] step {s} loss {loss:.5g}", flush=True)
    return hist


def predict_grids(net, problems):
    """Network outputs [n, 2 d^2, *M] for problems of one class (batches of net.batch)."""
    M = problems[0].M
    out = torch.empty((len(problems), net.cout) + M, dtype=torch.float32, device=api._dev())
    X = torch.zeros((net.batch, 2) + M, dtype=torch.float32, device=api._dev())
    for i0 in range(0, len(problems), net.batch):
        chunk = problems[i0:i0 + net.batch]
        for j, p in enumerate(chunk):
            p.net_input(out=X[j])
        torch.cuda.synchronize()
        y = net.forward(X)
        out[i0:i0 + len(chunk)] = y[:len(chunk)]
    torch.cuda.synchronize()
    return out


def predict_x0(net, problems):
    """Admissible initial fields, primal and dual, d unit loads each, for problems of one class:
    the network output projected by the solver (hom_grid_to_field)."""
    d, M = problems[0].d, problems[0].M
    grids = predict_grids(net, problems)
    xs_p, xs_d = [], []
    for j, p in enumerate(problems):
        xs_p.append(p.grid_to_field(grids[j, :d * d].reshape((d, d) + M), dual=False))
        xs_d.append(p.grid_to_field(grids[j, d * d:].reshape((d, d) + M), dual=True))
    return xs_p, xs_d
