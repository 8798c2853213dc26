"""GPU: the surrogate network kernels against the FP64 oracle network, the
grid transfers against the oracle's trigonometric interpolation, and the
learned initial guess (admissible start, unchanged bounds, fewer iterations).

Tolerances:
  * network output and loss: 1e-5 relative (FP32 sums of at most 64*27 terms);
  * parameter gradients, per layer: 1e-3 relative in the 2-norm (FP32 forward
    and backward against FP64; a ReLU whose pre-activation lies within FP32
    rounding of zero may switch, which moves single terms only);
  * field_to_grid: 1e-6 of the field's max (the grid is stored in FP32);
  * grid_to_field: 1e-12 relative (FP64 arithmetic on FP32-exact input).
"""
import math
import zlib

import numpy as np
import pytest

import homgen
from oracle import galerkin as ga, spectral as sp, unet as ou

pytestmark = pytest.mark.gpu


def _H():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1404_3614_amd as H
    from paper_1404_3614_amd import _lib
    _lib.load()
    return H


def he_theta(d, levels, base, cin, cout, rng):
    parts = []
    for ci, co, ks in ou.layer_shapes(d, levels, base, cin, cout):
        parts.append(rng.standard_normal(co * ci * ks ** d) * math.sqrt(2.0 / (ci * ks ** d)))
        parts.append(rng.standard_normal(co) * 0.1)
    return np.concatenate(parts)


NET_CASES = [
    # name, d, levels, base, size, batch, cout
    ("2d_l2_b4", 2, 2, 4, (9, 11), 2, 3),
    ("2d_l3_b32", 2, 3, 32, (25, 19), 2, 8),
    ("2d_l4_b8", 2, 4, 8, (27, 27), 1, 8),
    ("3d_l2_b4", 3, 2, 4, (5, 7, 6), 2, 18),
    ("3d_l3_b8", 3, 3, 8, (9, 11, 9), 1, 5),
]


@pytest.mark.parametrize("name,d,levels,base,size,batch,cout", NET_CASES, ids=[c[0] for c in NET_CASES])
def test_unet_forward_backward_match_oracle(name, d, levels, base, size, batch, cout):
    _H()
    import torch
    from paper_1404_3614_amd.learned import UNet
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    cin = 2
    theta = he_theta(d, levels, base, cin, cout, rng).astype(np.float32)
    x = rng.standard_normal((batch, cin) + size).astype(np.float32)
    tgt = rng.standard_normal((batch, cout) + size).astype(np.float32)
    print(f"[unet] {name} params {theta.size}", flush=True)
    net = UNet(d, size, levels=levels, base=base, cin=cin, cout=cout, batch=batch)
    assert net.nparams == theta.size == ou.n_params(d, levels, base, cin, cout)
    net.set_params(torch.from_numpy(theta))
    out = net.forward(torch.from_numpy(x).cuda()).cpu().numpy().astype(np.float64)
    loss = net.loss(torch.from_numpy(tgt).cuda())
    g = net.backward().cpu().numpy().astype(np.float64)

    th64, x64, t64 = theta.astype(np.float64), x.astype(np.float64), tgt.astype(np.float64)
    out_ref = ou.forward(th64, x64, levels, base, cout)
    loss_ref, g_ref = ou.loss_and_grad(th64, x64, t64, levels, base)
    assert np.abs(out - out_ref).max() <= 1e-5 * np.abs(out_ref).max()
    assert abs(loss - loss_ref) <= 1e-5 * loss_ref
    off = 0
    for k, (ci, co, ks) in enumerate(ou.layer_shapes(d, levels, base, cin, cout)):
        nw = co * ci * ks ** d
        for what, n in (("w", nw), ("b", co)):
            a, r = g[off:off + n], g_ref[off:off + n]
            rel = np.linalg.norm(a - r) / max(np.linalg.norm(r), 1e-30)
            assert rel <= 1e-3, f"layer {k} {what}: rel {rel:.3g}"
            off += n
    assert off == g.size


def test_unet_external_output_gradient_and_adam():
    """hom_unet_backward with a caller gradient, then one Adam step, against the FP64 formulas."""
    _H()
    import torch
    from paper_1404_3614_amd.learned import UNet
    d, levels, base, cin, cout, size, batch = 2, 2, 8, 2, 4, (13, 13), 2
    rng = np.random.default_rng(7)
    theta = he_theta(d, levels, base, cin, cout, rng).astype(np.float32)
    x = rng.standard_normal((batch, cin) + size).astype(np.float32)
    gout = rng.standard_normal((batch, cout) + size).astype(np.float32)
    net = UNet(d, size, levels=levels, base=base, cin=cin, cout=cout, batch=batch)
    net.set_params(torch.from_numpy(theta))
    net.forward(torch.from_numpy(x).cuda())
    g = net.backward(torch.from_numpy(gout).cuda()).cpu().numpy().astype(np.float64)
    _, tape, ws = ou.forward(theta.astype(np.float64), x.astype(np.float64), levels, base, cout, keep=True)
    g_ref = ou.backward(theta.astype(np.float64), x.astype(np.float64), tape, ws, gout.astype(np.float64), levels)
    assert np.linalg.norm(g - g_ref) <= 1e-4 * np.linalg.norm(g_ref)
    gg = net.grads.cpu().numpy().astype(np.float64)
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    for step in (1, 2):
        before = net.params.cpu().numpy().astype(np.float64)
        m_prev = net.m.cpu().numpy().astype(np.float64)
        v_prev = net.v.cpu().numpy().astype(np.float64)
        net.adam(lr=lr, beta1=b1, beta2=b2, eps=eps)
        torch.cuda.synchronize()
        m = b1 * m_prev + (1 - b1) * gg
        v = b2 * v_prev + (1 - b2) * gg * gg
        upd = lr * (m / (1 - b1 ** step)) / (np.sqrt(v / (1 - b2 ** step)) + eps)
        after = net.params.cpu().numpy().astype(np.float64)
        assert np.abs((before - after) - upd).max() <= 1e-5 * lr + 1e-6 * np.abs(before).max()
        assert np.allclose(net.m.cpu().numpy(), m, rtol=1e-5, atol=1e-9)


def test_unet_weighted_loss_matches_oracle():
    """Weighted squared error (one weight channel per half of the outputs) and its gradient."""
    _H()
    import torch
    from paper_1404_3614_amd.learned import UNet
    d, levels, base, cin, cout, size, batch = 2, 3, 8, 2, 8, (15, 13), 2
    rng = np.random.default_rng(11)
    theta = he_theta(d, levels, base, cin, cout, rng).astype(np.float32)
    x = rng.standard_normal((batch, cin) + size).astype(np.float32)
    tgt = rng.standard_normal((batch, cout) + size).astype(np.float32)
    w = rng.uniform(0.1, 3.0, (batch, 2) + size).astype(np.float32)
    net = UNet(d, size, levels=levels, base=base, cin=cin, cout=cout, batch=batch)
    net.set_params(torch.from_numpy(theta))
    net.forward(torch.from_numpy(x).cuda())
    loss = net.loss(torch.from_numpy(tgt).cuda(), torch.from_numpy(w).cuda())
    g = net.backward().cpu().numpy().astype(np.float64)
    th, x64 = theta.astype(np.float64), x.astype(np.float64)
    out, tape, ws = ou.forward(th, x64, levels, base, cout, keep=True)
    wfull = np.repeat(w.astype(np.float64), cout // 2, axis=1)
    diff = out - tgt.astype(np.float64)
    loss_ref = float(np.sum(wfull * diff ** 2) / out.size)
    g_ref = ou.backward(th, x64, tape, ws, 2.0 * wfull * diff / out.size, levels)
    assert abs(loss - loss_ref) <= 1e-5 * loss_ref
    assert np.linalg.norm(g - g_ref) <= 1e-4 * np.linalg.norm(g_ref)


def test_unet_invalid_desc():
    H = _H()
    from paper_1404_3614_amd.learned import UNet
    with pytest.raises(H.HomError):
        UNet(2, (1, 9), levels=2, base=4, batch=1)
    with pytest.raises(H.HomError):
        UNet(4, (9, 9), levels=2, base=4, batch=1)


# ---------------------------------------------------------------- grid transfers
GRID_CASES = [
    ("c1", lambda: homgen.square_inclusion_cell(), (13, 13)),
    ("rect_aniso", lambda: homgen.square_inclusion_cell(Y=np.array([1.0, 1.7])), (13, 41)),
    ("sph3d", lambda: homgen.sphere_cell(seed=3, n=4, anisotropic=True), (5, 13, 5)),
]


def _rand_spectrum(d, N, Y, dual, rng):
    u = rng.standard_normal((d,) + tuple(N))
    G = sp.proj_J(N, np.array(Y)) if dual else sp.proj_E(N, np.array(Y))
    return sp.apply_blockdiag(G, sp.dft_nd(u, d))


@pytest.mark.parametrize("name,mk,N", GRID_CASES, ids=[c[0] for c in GRID_CASES])
@pytest.mark.parametrize("dual", [False, True], ids=["primal", "dual"])
def test_field_to_grid_matches_oracle(name, mk, N, dual):
    H = _H()
    import torch
    from layout import field_from_spectrum
    cell = mk()
    d = cell.d
    pb = H.problem_from_cell(cell, N, precision="fp64")
    rng = np.random.default_rng(23)
    M = tuple(2 * n - 1 for n in N)
    specs = [_rand_spectrum(d, N, cell.Y, dual, rng) for _ in range(d)]
    fields = [torch.tensor(field_from_spectrum(s, d, N, cell.Y, dual), dtype=torch.complex128, device="cuda")
              for s in specs]
    out = pb.field_to_grid(fields, dual=dual).cpu().numpy()
    assert out.shape == (d, d) + M
    for l, s in enumerate(specs):
        ref = ga.to_grid(s, M)
        assert np.abs(out[l] - ref).max() <= 1e-6 * np.abs(ref).max()


@pytest.mark.parametrize("name,mk,N", GRID_CASES, ids=[c[0] for c in GRID_CASES])
@pytest.mark.parametrize("dual", [False, True], ids=["primal", "dual"])
def test_grid_to_field_matches_oracle(name, mk, N, dual):
    H = _H()
    import torch
    from layout import spectrum_from_field
    cell = mk()
    d = cell.d
    pb = H.problem_from_cell(cell, N, precision="mixed")
    rng = np.random.default_rng(29)
    M = tuple(2 * n - 1 for n in N)
    grid = rng.standard_normal((d, d) + M).astype(np.float32)
    fields = pb.grid_to_field(torch.from_numpy(grid).cuda(), dual=dual)
    G = sp.proj_J(N, np.array(cell.Y)) if dual else sp.proj_E(N, np.array(cell.Y))
    for l in range(d):
        ref = sp.apply_blockdiag(G, sp.trunc(sp.dft_nd(grid[l].astype(np.float64), d), N))
        got = spectrum_from_field(fields[l].cpu().numpy(), d, N, cell.Y, dual)
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    # a projection: grid -> field -> grid -> field is the identity on its image
    again = pb.grid_to_field(pb.field_to_grid(fields, dual=dual), dual=dual)
    for a, b in zip(fields, again):
        a, b = a.cpu().numpy(), b.cpu().numpy()
        assert np.abs(a - b).max() <= 1e-6 * np.abs(a).max()


def test_net_input_channels_and_weights():
    H = _H()
    cell = homgen.square_inclusion_cell(rho_in=300.0)
    N = (13, 13)
    pb = H.problem_from_cell(cell, N, precision="mixed")
    x = pb.net_input().cpu().numpy().astype(np.float64)
    w = pb.net_weights().cpu().numpy().astype(np.float64)
    op = ga.make_problem(cell, N)
    a = np.einsum("aa...->...", op.Atil) / 2
    b = np.einsum("aa...->...", op.Btil) / 2
    assert np.abs(x[0] - a / a.mean()).max() <= 1e-6 * np.abs(a / a.mean()).max()
    assert np.abs(x[1] - np.log(np.maximum(a, 1e-3 * a.mean()) / a.mean())).max() <= 1e-5
    for k, c in enumerate((a, b)):
        ref = np.maximum(c, 1e-3 * c.mean()) / c.mean()
        assert np.abs(w[k] - ref).max() <= 1e-6 * ref.max()
        assert w[k].min() > 0.0


# ---------------------------------------------------------------- learned initial guess
def _cells(seed0, n, logrho):
    return [homgen.random_squares_cell(seed0 + i, logrho=logrho)[0] for i in range(n)]


def test_learned_x0_tighter_start_same_bounds():
    """Train a small surrogate on solver fields (2D, N = 41), then solve held-out
    high-contrast cells from x0 = 0 and from the projected prediction.

    What the network gains: its projected output is an admissible field, so it
    already gives guaranteed bounds (Def. upper_lower_bounds: any field of E_N /
    J_N does), much closer to the converged ones than those of the zero field
    (the Voigt / Reuss bounds): the energy error Abar(x0) - Abar(x*) is a
    fraction of Abar(0) - Abar(x*).  CG from that start reaches the same bounds.
    Under the gap rule, which stops on the bounds' own error, the start saves
    iterations; under the residual rule it does not (the stopping test is
    governed by the interface content of the residual, which the prediction
    does not remove), and that count is only bounded here."""
    H = _H()
    import torch
    from paper_1404_3614_amd import learned as lr_
    N = (41, 41)
    M = (81, 81)
    train_cells = _cells(7_000_000, 512, (math.log10(2.0), 3.0))
    print("[learned] generating training fields", flush=True)
    X, Y, W, it_train = lr_.solver_samples(train_cells, N, tol=1e-6)
    net = lr_.UNet(2, M, levels=3, base=16, batch=16)
    net.init_params(seed=1)
    print("[learned] training", flush=True)
    hist = lr_.train(net, X, Y, steps=600, lr=2e-3, lr_final=1e-4, seed=3)
    assert np.mean(hist[-50:]) < 0.1 * np.mean(hist[:10])

    test_cells = _cells(8_000_000, 32, (2.0, 3.0))
    st = torch.cuda.Stream()
    probs = [H.problem_from_cell(c, N, precision="mixed", stream=st) for c in test_cells]
    batch = H.Batch(probs)
    rng = [H.cell_eig_range(c) for c in test_cells]
    a_min, a_max = min(r[0] for r in rng), max(r[1] for r in rng)
    plain = batch.solve_bounds(tol=1e-6)
    zero = batch.bounds([[p.new_field(False) for _ in range(2)] for p in probs],
                        [[p.new_field(True) for _ in range(2)] for p in probs])
    x0p, x0d = lr_.predict_x0(net, batch)
    start = batch.bounds(x0p, x0d)
    learned = batch.solve_bounds(tol=1e-6, x0_primal=x0p, x0_dual=x0d)
    its = lambda res: np.array([[r["iters"] for r in b["info_primal"] + b["info_dual"]] for b in res])
    it_plain, it_learn = its(plain), its(learned)
    ep, ed = [], []
    for b0, z, s, b1 in zip(plain, zero, start, learned):
        scale = np.linalg.norm(b0["A_up"], 2)
        # same bounds to the solver tolerance
        assert np.abs(b1["A_up"] - b0["A_up"]).max() <= 1e-6 * scale
        assert np.abs(b1["A_low"] - b0["A_low"]).max() <= 1e-6 * scale
        # the start is admissible: its bounds are guaranteed, only looser
        assert np.linalg.eigvalsh(s["A_up"] - b1["A_up"]).min() >= -1e-9 * scale
        assert np.linalg.eigvalsh(b1["A_low"] - s["A_low"]).min() >= -1e-9 * scale
        ep.append((np.diag(s["A_up"]) - np.diag(b0["A_up"])) / (np.diag(z["A_up"]) - np.diag(b0["A_up"])))
        ed.append((np.diag(s["B_up"]) - np.diag(b0["B_up"])) / (np.diag(z["B_up"]) - np.diag(b0["B_up"])))
    ep, ed = float(np.mean(ep)), float(np.mean(ed))
    # the gap rule (each bound within 1 % of the discretisation gap) from both starts
    batch.set_stop("gap", 1e-2, a_min, a_max)
    gap_plain = batch.solve_bounds(tol=1e-12)
    gap_learn = batch.solve_bounds(tol=1e-12, x0_primal=x0p, x0_dual=x0d)
    batch.set_stop("residual")
    g_plain, g_learn = its(gap_plain), its(gap_learn)
    print(f"[learned] energy error of the start vs zero start: primal {ep:.3f} dual {ed:.3f}; "
          f"iterations residual rule plain {it_plain.mean():.1f} learned {it_learn.mean():.1f}; "
          f"gap rule plain {g_plain.mean():.1f} learned {g_learn.mean():.1f}", flush=True)
    assert ep < 0.5 and ed < 0.8
    assert g_learn.mean() < g_plain.mean()
    for b0, b1 in zip(gap_plain, gap_learn):
        n = np.linalg.norm(b0["A_up"], 2)
        for key in ("A_up", "A_low"):
            assert np.abs(b1[key] - b0[key]).max() <= 0.02 * n      # both within 1 % of the gap of the same bounds
    assert it_learn.mean() <= 1.25 * it_plain.mean()


@pytest.mark.parametrize("d,N", [(2, (41, 41)), (3, (13, 13, 13))], ids=["2d", "3d"])
def test_batched_transfers_equal_per_problem(d, N):
    """hom_batch_field_to_grid / hom_batch_grid_to_field / hom_batch_net_input
    (one launch per pass for every cell) against the per-problem calls: the same
    kernels on the same data, so equal bit for bit; strided blocks land where
    the stride says."""
    H = _H()
    import torch
    cells = ([homgen.random_squares_cell(900 + i)[0] for i in range(3)] if d == 2 else
             [homgen.random_spheres_cell(900 + i, kmin=3, kmax=5)[0] for i in range(3)])
    st = torch.cuda.Stream()
    probs = [H.problem_from_cell(c, N, precision="mixed", stream=st) for c in cells]
    b = H.Batch(probs)
    xp, _, xd, _ = b.solve_pair(tol=1e-6)
    M = probs[0].M
    Mt = int(np.prod(M))
    stride = 2 * d * d * Mt + 7 * Mt          # room for a record larger than one block
    G = torch.full((len(probs), stride // Mt) + M, float("nan"), dtype=torch.float32, device="cuda")
    b.field_to_grid(xp, False, G, stride)
    b.field_to_grid(xd, True, G[:, d * d:], stride)
    X = torch.empty((len(probs), 2) + M, dtype=torch.float32, device="cuda")
    Wt = torch.empty_like(X)
    b.net_input(X)
    b.net_input(Wt, weights=True)
    torch.cuda.synchronize()
    for i, p in enumerate(probs):
        gp = p.field_to_grid(xp[i], dual=False).reshape((d * d,) + M)
        gd = p.field_to_grid(xd[i], dual=True).reshape((d * d,) + M)
        assert torch.equal(G[i, :d * d], gp) and torch.equal(G[i, d * d:2 * d * d], gd)
        assert torch.isnan(G[i, 2 * d * d:]).all()
        assert torch.equal(X[i], p.net_input()) and torch.equal(Wt[i], p.net_weights())
    back_p = b.grid_to_field(G, False, stride=stride)
    back_d = b.grid_to_field(G[:, d * d:], True, stride=stride)
    for i, p in enumerate(probs):
        ref_p = p.grid_to_field(G[i, :d * d].reshape((d, d) + M).contiguous(), dual=False)
        ref_d = p.grid_to_field(G[i, d * d:2 * d * d].reshape((d, d) + M).contiguous(), dual=True)
        for a in range(d):
            assert torch.equal(back_p[i][a], ref_p[a]) and torch.equal(back_d[i][a], ref_d[a])


def test_pair_solve_from_starting_fields_equals_separate_solves():
    """hom_batch_solve_pair with starting fields: the same iterations and fields as
    the primal and dual solves from those fields one after the other."""
    H = _H()
    import torch
    cells = [homgen.random_squares_cell(950 + i)[0] for i in range(3)]
    st = torch.cuda.Stream()
    probs = [H.problem_from_cell(c, (41, 41), precision="mixed", stream=st) for c in cells]
    b = H.Batch(probs)
    coarse_p, _, coarse_d, _ = b.solve_pair(tol=1e-2)
    x0p = [[t.clone() for t in ts] for ts in coarse_p]
    x0d = [[t.clone() for t in ts] for ts in coarse_d]
    fp, ip, fd, idl = b.solve_pair(tol=1e-8, x0_primal=x0p, x0_dual=x0d)
    sp, isp = b.solve(False, x0=x0p, tol=1e-8)
    sd, isd = b.solve(True, x0=x0d, tol=1e-8)
    for i in range(len(probs)):
        assert [r["iters"] for r in ip[i] + idl[i]] == [r["iters"] for r in isp[i] + isd[i]]
        for a in range(2):
            assert torch.equal(fp[i][a], sp[i][a]) and torch.equal(fd[i][a], sd[i][a])
    # and fewer iterations than from zero
    _, iz, _, idz = b.solve_pair(tol=1e-8)
    assert sum(r["iters"] for c in ip for r in c) < sum(r["iters"] for c in iz for r in c)
