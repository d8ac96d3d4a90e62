"""Pins of the oracle's image-space gridding T_d / T_d^H (Eq. 5, 7-9).

* brute force: the FFT-based T and T^H equal the dense matrix built from the
  explicit double sum with no FFT (catches scale, pad/crop index and sign
  slips);
* exact special case: an integer displacement s moves every tap by alpha*s
  on the periodic grid, so T_s x == roll(T_0 x, -s) (pins the pull sign and
  the wrap);
* the method's claim of an exact forward-adjoint pair;
* d = 0 gives the identity, and a constant fractional d gives the textbook
  Fourier shift, both up to the kernel's approximation error.
"""
import numpy as np
import pytest

from oracle import dense, warp
from synth import bump_displacement, ellipsoid_phantom, rng


def _rand_c(g, shape):
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


@pytest.mark.parametrize("shape", [(8, 8), (4, 6, 8)])
def test_warp_equals_dense_brute_force(shape, rel):
    g = np.random.default_rng(7)
    d = g.uniform(-2.5, 2.5, (len(shape),) + shape).astype(np.float32)
    x = _rand_c(g, shape)
    T = dense.warp_matrix(d)
    assert rel(warp.warp(x, d), (T @ x.reshape(-1)).reshape(shape)) < 1e-12
    v = _rand_c(g, shape)
    assert rel(warp.warp_adjoint(v, d), (T.conj().T @ v.reshape(-1)).reshape(shape)) < 1e-12


@pytest.mark.parametrize("shape", [(10, 12), (6, 8, 10)])
def test_adjoint_identity(shape):
    g = np.random.default_rng(3)
    d = g.uniform(-4, 4, (len(shape),) + shape).astype(np.float32)
    x, y = _rand_c(g, shape), _rand_c(g, shape)
    lhs = np.vdot(y, warp.warp(x, d))
    rhs = np.vdot(warp.warp_adjoint(y, d), x)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("shift", [(1, 0), (0, -3), (2, 5), (-1, 2, 3)])
def test_integer_shift_is_circular_roll(shift):
    ndim = len(shift)
    shape = (16, 12) if ndim == 2 else (8, 10, 12)
    g = np.random.default_rng(11)
    x = _rand_c(g, shape)
    d0 = np.zeros((ndim,) + shape, dtype=np.float32)
    ds = np.stack([np.full(shape, s, dtype=np.float32) for s in shift])
    want = np.roll(warp.warp(x, d0), [-s for s in shift], axis=tuple(range(ndim)))
    got = warp.warp(x, ds)
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))


def test_identity_at_zero_displacement_2d(rel):
    # the 2D warp workload's phantom; kernel error band of W=4, alpha=2 KB
    x = ellipsoid_phantom((64, 64), 10, rng(1, 0))
    d0 = np.zeros((2, 64, 64), dtype=np.float32)
    e = rel(warp.warp(x, d0), x)
    # frozen band: 1.65e-3 for this phantom
    assert 1.5e-3 < e < 1.8e-3


def test_identity_at_zero_displacement_3d(rel):
    x = ellipsoid_phantom((24, 24, 24), 10, rng(9, 0))
    d0 = np.zeros((3, 24, 24, 24), dtype=np.float32)
    e = rel(warp.warp(x, d0), x)
    # frozen band: 2.2e-3 for this phantom
    assert 1.9e-3 < e < 2.5e-3


@pytest.mark.parametrize("t", [(0.37,), (0.25, -0.6), (0.5, 0.13, -0.71)])
def test_constant_shift_matches_fourier_shift(t, rel):
    ndim = len(t)
    shape = {1: (64,), 2: (32, 40), 3: (16, 20, 24)}[ndim]
    g = np.random.default_rng(5)
    # smooth (band-limited) test image: low frequencies only
    X = np.zeros(shape, dtype=complex)
    sl = tuple(slice(0, n // 4) for n in shape)
    X[sl] = _rand_c(g, tuple(n // 4 for n in shape))
    x = np.fft.ifftn(X)
    d = np.stack([np.full(shape, ti, dtype=np.float32) for ti in t])
    phase = np.ones(shape, dtype=complex)
    for i, (n, ti) in enumerate(zip(shape, np.float32(t))):
        k = np.fft.fftfreq(n, 1.0 / n)
        sh = [1] * ndim
        sh[i] = n
        phase = phase * np.exp(2j * np.pi * k * float(ti) / n).reshape(sh)
    want = np.fft.ifftn(np.fft.fftn(x) * phase)   # x(r + t)
    # observed 3.6e-4 (1D), 4.1e-4 (2D), 9.2e-4 (3D)
    assert rel(warp.warp(x, d), want) < 1.2e-3


def test_warp_at_matches_full(rel):
    shape = (12, 10, 8)
    g = np.random.default_rng(2)
    x = _rand_c(g, shape)
    d = bump_displacement(shape, 3, 3.0, 2.0, g)
    vox = np.array([0, 5, 77, 500, 959])
    assert rel(warp.warp_at(x, d, vox), warp.warp(x, d).reshape(-1)[vox]) < 1e-14


def test_multi_adjoint_is_sum():
    shape = (8, 8)
    g = np.random.default_rng(4)
    ds = [g.uniform(-2, 2, (2,) + shape).astype(np.float32) for _ in range(3)]
    vs = [_rand_c(g, shape) for _ in range(3)]
    s = warp.warp_multi_adjoint(vs, ds)
    T = [dense.warp_matrix(d) for d in ds]
    want = sum(Ti.conj().T @ v.reshape(-1) for Ti, v in zip(T, vs)).reshape(shape)
    assert np.allclose(s, want, rtol=0, atol=1e-12 * np.abs(want).max())
