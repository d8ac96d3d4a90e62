"""Pins of the oracle's kernel and tap rule against closed forms, power
series, numerical quadrature and the published I0 table."""
import math
import os

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import grid, kernel

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _i0_series(x, terms=60):
    # I0(x) = sum_k (x^2/4)^k / (k!)^2
    s, t = 0.0, 1.0
    q = x * x / 4.0
    for k in range(terms):
        if k:
            t *= q / (k * k)
        s += t
    return s


def test_beta_and_peak():
    # beta from the width/oversampling rule; c(0) = I0(beta) by the series.
    b = kernel.BETA
    assert abs(b - math.pi * math.sqrt(4 * 1.5 ** 2 - 0.8)) < 1e-15
    assert abs(kernel.kb(np.array([0.0]))[0] - _i0_series(b)) < 1e-9 * _i0_series(b)


def test_i0_against_published_table():
    # Values of I0 and I1 from the standard tables (Abramowitz & Stegun 9.8).
    rows = np.loadtxt(os.path.join(GOLDEN, "bessel_i0_i1.txt"))
    for x, i0v, i1v in rows:
        assert abs(_i0_series(x) - i0v) < 2e-9 * i0v
        # c(u) at the u where beta*sqrt(1-(u/2)^2) == x
        if x < kernel.BETA:
            u = 2.0 * math.sqrt(1.0 - (x / kernel.BETA) ** 2)
            assert abs(kernel.kb(np.array([u]))[0] - i0v) < 2e-9 * i0v
            # c'(u) = -(beta u / 4) I1(x) / s with s = x / beta (W = 4)
            want = -(kernel.BETA * u / 4.0) * i1v * kernel.BETA / x
            assert abs(kernel.kb_deriv(np.array([u]))[0] - want) < 2e-9 * abs(want)


def test_open_support():
    u = np.array([-2.0, -1.999999, 0.0, 1.999999, 2.0, 2.5])
    c = kernel.kb(u)
    assert c[0] == 0.0 and c[4] == 0.0 and c[5] == 0.0
    assert c[1] > 0 and c[3] > 0
    # edge/peak ratio ~ 9.2e-4 (the kernel's pedestal)
    assert abs(kernel.kb(np.array([1.9999999]))[0] / c[2] - 1.0 / kernel.kb(np.array([0.0]))[0]) < 1e-6


@pytest.mark.parametrize("f", [0.0, 0.05, 0.125, 0.2, 0.25, 0.3])
def test_kb_ft_against_quadrature(f):
    # C(f) = int_{-W/2}^{W/2} c(u) cos(2 pi f u) du (c is even)
    val, _ = quad(lambda u: kernel.kb(np.array([u]))[0] * math.cos(2 * math.pi * f * u),
                  -2.0, 2.0, epsabs=1e-12, epsrel=1e-12, limit=200)
    assert abs(kernel.kb_ft(np.array([f]))[0] - val) < 1e-9 * abs(val)


def test_kb_ft_negative_radicand_branch():
    # beyond pi W f > beta the transform continues as W sin(z)/z
    f = 1.2 * kernel.BETA / (math.pi * 4)
    val, _ = quad(lambda u: kernel.kb(np.array([u]))[0] * math.cos(2 * math.pi * f * u),
                  -2.0, 2.0, epsabs=1e-12, epsrel=1e-12, limit=400)
    assert abs(kernel.kb_ft(np.array([f]))[0] - val) < 1e-7 * kernel.kb_ft(np.array([0.0]))[0]


def test_kb_deriv_against_finite_difference():
    u = np.linspace(-1.95, 1.95, 41)
    h = 1e-6
    fd = (kernel.kb(u + h) - kernel.kb(u - h)) / (2 * h)
    assert np.max(np.abs(kernel.kb_deriv(u) - fd)) < 1e-6 * kernel.kb(np.array([0.0]))[0]


def test_tap_rule():
    idx, off = grid.taps_1d(np.array([5.3, 4.0, -0.5, 31.9]), 32)
    # y = 5.3: taps 4,5,6,7 with offsets 1.3, 0.3, -0.7, -1.7
    assert list(idx[:, 0]) == [4, 5, 6, 7]
    assert np.allclose(off[:, 0], [1.3, 0.3, -0.7, -1.7])
    # integer y: taps y-1..y+2, the last at offset -2 has weight 0
    assert list(idx[:, 1]) == [3, 4, 5, 6]
    assert kernel.kb(off[3, 1:2])[0] == 0.0
    # floor, not truncation, for negative coordinates; periodic wrap
    assert list(idx[:, 2]) == [30, 31, 0, 1]
    assert list(idx[:, 3]) == [30, 31, 0, 1]


def test_spread_is_adjoint_of_gather_and_sums_duplicates():
    g = np.random.default_rng(1)
    G = (12, 10)
    coords = g.uniform(-3, 14, (50, 2))
    coords[10] = coords[3]  # duplicate point: both contributions must land
    grid_ = g.standard_normal(G) + 1j * g.standard_normal(G)
    v = g.standard_normal(50) + 1j * g.standard_normal(50)
    lhs = np.vdot(grid.spread(v, coords, G), grid_)
    rhs = np.vdot(v, grid.gather(grid_, coords))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # a fancy-index += would drop the duplicate; bincount does not
    one = np.zeros(50, dtype=complex)
    one[3] = one[10] = 1.0
    s = grid.spread(one, coords, G)
    two = np.zeros(50, dtype=complex)
    two[3] = 2.0
    assert np.allclose(s, grid.spread(two, coords, G))
