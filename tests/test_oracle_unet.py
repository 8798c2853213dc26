"""Pins for oracle.unet: explicit backpropagation against central finite
differences (FP64), and the adjoint identities of pooling and upsampling."""
import numpy as np
import pytest

from oracle import unet


@pytest.mark.parametrize("d,size,levels", [(2, (5, 7), 2), (2, (9, 9), 3), (3, (3, 5, 3), 2)])
def test_gradient_matches_finite_differences(d, size, levels):
    rng = np.random.default_rng(3)
    base, cin, cout, B = 2, 2, 3, 2
    npar = unet.n_params(d, levels, base, cin, cout)
    theta = rng.standard_normal(npar) * 0.5
    x = rng.standard_normal((B, cin) + size)
    t = rng.standard_normal((B, cout) + size)
    loss, g = unet.loss_and_grad(theta, x, t, levels, base)
    h = 1e-6
    for i in rng.choice(npar, size=min(40, npar), replace=False):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        lp = unet.loss_and_grad(tp, x, t, levels, base)[0]
        lm = unet.loss_and_grad(tm, x, t, levels, base)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


@pytest.mark.parametrize("S", [(6, 7), (5, 5), (3, 4, 5)])
def test_pool_and_upsample_adjoints(S):
    rng = np.random.default_rng(4)
    x = rng.standard_normal((2, 3) + S)
    y = rng.standard_normal((2, 3) + tuple((n + 1) // 2 for n in S))
    # <pool x, y> = <x, pool^T y>
    assert abs(np.sum(unet.pool(x) * y) - np.sum(x * unet.pool_backward(y, S))) < 1e-12
    # <up y, x> = <y, up^T x>
    assert abs(np.sum(unet.up(y, S) * x) - np.sum(y * unet.up_backward(x, y.shape[2:]))) < 1e-12


def test_layer_count_and_parameter_layout():
    shapes = unet.layer_shapes(2, 4, 32, 2, 8)
    assert len(shapes) == 4 * 2 + 3 * 3 + 1
    assert shapes[0] == (2, 32, 3) and shapes[7] == (256, 256, 3) and shapes[-1] == (32, 8, 1)
    assert unet.n_params(2, 4, 32, 2, 8) == sum(co * ci * k * k + co for ci, co, k in shapes)
