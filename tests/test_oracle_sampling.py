"""Pins of the oracle's point values A(x_N^k) (GaNi, Def. GaNi / eq. FD_A_GaNi).

The grid points are x^k = Y k / N, k in Z_N, stored at index k mod N (eq.
grid_points, Sec. 4.2).  Pixel p along an axis covers [-Y/2 + p Y/P,
-Y/2 + (p + 1) Y/P); inclusions are open sets, periodic by the minimum image
(eq. S); the closed square of eq. S2 includes its faces.  Every expected value
below is derived by hand from these definitions, so that an off-by-one pixel
index, a missing periodic wrap, a wrong storage order or a closed/open mix-up
fails here, independently of the implementation under test.
"""
import numpy as np
import pytest

import homgen
from oracle import coefficients as co, even as ev

SAMPLERS = [("odd", lambda cell, shape, inverse=False: co.point_values(cell, shape, inverse)),
            ("general", lambda cell, shape, inverse=False: ev.point_values(cell, shape, inverse))]


def ids_image(shape):
    """Pixel cell whose phase id is the flat pixel index, phase q = (q + 1) I."""
    d = len(shape)
    P = int(np.prod(shape))
    phase = np.arange(P, dtype=np.int32).reshape(shape)
    phase_A = np.stack([np.eye(d) * (q + 1.0) for q in range(P)])
    return homgen.Pixels(d=d, Y=np.ones(d), phase=phase, phase_A=phase_A)


@pytest.mark.parametrize("name,pv", SAMPLERS, ids=[s[0] for s in SAMPLERS])
@pytest.mark.parametrize("N", [3, 5, 7])
def test_pixel_centres_on_grid_points(name, pv, N):
    """P = N (odd): pixel p has its centre at -1/2 + (p + 1/2)/N = k/N with
    k = p - (N - 1)/2, so the value at grid index k mod N is that of pixel
    k + (N - 1)/2: the image rolled by (N - 1)/2, i.e. ifftshift."""
    cell = ids_image((N, N))
    vals = pv(cell, (N, N))[0, 0]
    ids = np.arange(N * N).reshape(N, N)
    assert np.array_equal(vals, np.fft.ifftshift(ids) + 1.0)
    assert vals[0, 0] == ids[(N - 1) // 2, (N - 1) // 2] + 1.0        # the origin sits in the centre pixel


@pytest.mark.parametrize("name,pv", SAMPLERS, ids=[s[0] for s in SAMPLERS])
def test_pixel_left_edges_belong_to_the_pixel(name, pv):
    """N = 3, P = 6 per axis: the points -1/3, 0, 1/3 are the left edges of
    pixels 1, 3, 5 (x + 1/2 = 1/6, 3/6, 5/6 of the cell); stored in the order
    k = 0, 1, -1 that is pixels 3, 5, 1.  The same along the second axis."""
    cell = ids_image((6, 6))
    vals = pv(cell, (3, 3))[0, 0]
    order = [3, 5, 1]
    want = np.array([[6 * i + j + 1.0 for j in order] for i in order])
    assert np.array_equal(vals, want)


@pytest.mark.parametrize("name,pv", SAMPLERS, ids=[s[0] for s in SAMPLERS])
def test_pixel_coarse_image_and_inverse(name, pv):
    """N = 5, P = 2 (two pixels per axis, each of width 1/2): the points
    k/5 with k = -2, -1 lie in pixel 0 and k = 0, 1, 2 in pixel 1 (x = 0 is the
    left edge of pixel 1).  The inverse samples hold the inverse matrices."""
    phase = np.array([[0, 1], [1, 0]], dtype=np.int32)
    A = [np.array([[2.0, 0.5], [0.5, 1.0]]), np.array([[7.0, -1.0], [-1.0, 3.0]])]
    cell = homgen.Pixels(d=2, Y=np.ones(2), phase=phase, phase_A=np.stack(A))
    pix_of_k = {0: 1, 1: 1, 2: 1, 3: 0, 4: 0}           # index k mod 5 -> pixel
    for inverse in (False, True):
        vals = pv(cell, (5, 5), inverse)
        for i in range(5):
            for j in range(5):
                want = A[phase[pix_of_k[i], pix_of_k[j]]]
                want = np.linalg.inv(want) if inverse else want
                assert np.allclose(vals[:, :, i, j], want, rtol=1e-15, atol=0)


def _ball(center, R):
    c = homgen.Inclusions(d=3, Y=np.ones(3), A0=np.eye(3))
    c.add("ball", center, [R], 5.0 * np.eye(3))
    return c


@pytest.mark.parametrize("name,pv", SAMPLERS, ids=[s[0] for s in SAMPLERS])
def test_ball_counted_by_hand(name, pv):
    """N = 5 (points k/5, k = -2..2 per axis).

    Centre 0, R = 0.3: |x|^2 = (i^2 + j^2 + l^2)/25 < 0.09 iff i^2 + j^2 + l^2 <= 2:
    1 + 6 + 12 = 19 points, and (1, 1, 1) is outside (3/25 = 0.12).

    Centre (1/2, 1/2, 1/2), R = 0.35 (periodic wrap): the per-axis distances to
    1/2 are 0.1 (k = +-2, the k = -2 side across the cell boundary), 0.3
    (k = +-1), 0.5 (k = 0); sums of squares below 0.1225 are 0.03 (2^3 = 8
    points) and 0.11 (3 * 2 * 2^2 = 24 points): 32 points, none with k = 0."""
    vals = pv(_ball([0.0, 0.0, 0.0], 0.3), (5, 5, 5))[0, 0]
    inside = vals == 5.0
    assert int(inside.sum()) == 19
    k = np.array([0, 1, 2, -2, -1])
    K2 = k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2
    assert np.array_equal(inside, K2 <= 2)
    vals = pv(_ball([0.5, 0.5, 0.5], 0.35), (5, 5, 5))[0, 0]
    inside = vals == 5.0
    assert int(inside.sum()) == 32
    assert not inside[0].any() and not inside[:, 0].any() and not inside[:, :, 0].any()
    assert inside[2, 2, 2] and inside[3, 3, 3] and inside[2, 3, 1]     # (2,2,2), (-2,-2,-2), (2,-2,1)
    assert not inside[1, 1, 1]                                         # 0.09 * 3 = 0.27


def test_box_open_and_closed_on_an_even_grid():
    """N = 4 (points -1/2, -1/4, 0, 1/4 per axis), centred square of side 1/2:
    the open square holds only x = 0 per axis (1 point), the closed one also the
    faces x = +-1/4 (3 per axis, 9 points); a box across the cell boundary
    (centre (1/2, 0)) holds x_0 = -1/2 and is cut by the open rule at +-1/4."""
    c = homgen.Inclusions(d=2, Y=np.ones(2), A0=np.eye(2))
    c.add("rect", [0.0, 0.0], [0.5, 0.5], 3.0 * np.eye(2))
    op = ev.point_values(c, (4, 4))[0, 0] == 3.0
    cl = ev.point_values(c, (4, 4), closed=True)[0, 0] == 3.0
    assert int(op.sum()) == 1 and op[0, 0]
    assert int(cl.sum()) == 9
    k = np.array([0, 1, -2, -1])          # even.freqs_general(4): 0, 1, -2, -1
    want = (np.abs(k)[:, None] <= 1) & (np.abs(k)[None, :] <= 1)
    assert np.array_equal(cl, want)
    c2 = homgen.Inclusions(d=2, Y=np.ones(2), A0=np.eye(2))
    c2.add("rect", [0.5, 0.0], [0.5, 0.5], 3.0 * np.eye(2))
    op2 = ev.point_values(c2, (4, 4))[0, 0] == 3.0
    assert int(op2.sum()) == 1 and op2[2, 0]          # x = (-1/2, 0): distance 0 to the centre by the wrap
    cl2 = ev.point_values(c2, (4, 4), closed=True)[0, 0] == 3.0
    assert int(cl2.sum()) == 9 and cl2[1, 0] and cl2[3, 0] and cl2[2, 1] and cl2[2, 3]


def test_box_on_an_odd_grid_and_non_unit_cell():
    """N = 5 on the cell Y = (2, 1): points x = (2k/5, k/5).  A box of sides
    (1.0, 0.5) centred at (0.4, 0): |x_0 - 0.4| < 0.5 holds for k_0 = 0, 1, 2
    (0.4, 0, 0.4 away) and |x_1| < 0.25 for k_1 = -1, 0, 1: 9 points."""
    c = homgen.Inclusions(d=2, Y=np.array([2.0, 1.0]), A0=np.eye(2))
    c.add("rect", [0.4, 0.0], [1.0, 0.5], 4.0 * np.eye(2))
    for name, pv in SAMPLERS:
        inside = pv(c, (5, 5))[0, 0] == 4.0
        want = np.zeros((5, 5), bool)
        for i in (0, 1, 2):
            for j in (0, 1, 4):
                want[i, j] = True
        assert np.array_equal(inside, want), name
