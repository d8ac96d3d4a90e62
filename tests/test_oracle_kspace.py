"""Pins of the oracle's k-space pair G / G^H (Eq. 1-3).

* brute force: the FFT-based G and G^H equal the dense matrix built from the
  explicit sum with no FFT;
* the approximated definition: G is the direct NDFT up to the kernel's
  approximation error (pins the exponent sign, the centring and the scale);
* the forward-adjoint pair.
"""
import numpy as np
import pytest

from oracle import dense, kspace
from synth import radial_spokes_2d, radial_spokes_3d, uniform_samples


def _rand_c(g, shape):
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


@pytest.mark.parametrize("shape", [(8, 6), (4, 6, 8)])
def test_nufft_equals_dense_brute_force(shape, rel):
    g = np.random.default_rng(1)
    k = uniform_samples(40, len(shape), g)
    z = _rand_c(g, shape)
    A = dense.nufft_matrix(k, shape)
    assert rel(kspace.nufft_forward(z, k), A @ z.reshape(-1)) < 1e-12
    y = _rand_c(g, 40)
    assert rel(kspace.nufft_adjoint(y, k, shape), (A.conj().T @ y).reshape(shape)) < 1e-12


def test_nufft_approximates_ndft_2d(rel):
    g = np.random.default_rng(2)
    shape = (32, 32)
    k = uniform_samples(3000, 2, g)
    z = _rand_c(g, shape)
    e = rel(kspace.nufft_forward(z, k), kspace.ndft(z, k))
    # W=4, alpha=2 Kaiser-Bessel: ~6e-4
    assert 3e-4 < e < 1e-3
    y = _rand_c(g, 3000)
    e2 = rel(kspace.nufft_adjoint(y, k, shape), kspace.ndft_adjoint(y, k, shape))
    assert e2 < 1e-3


def test_nufft_approximates_ndft_3d_radial(rel):
    g = np.random.default_rng(3)
    shape = (12, 16, 10)
    k = radial_spokes_3d(0, 30, 16)
    z = _rand_c(g, shape)
    assert rel(kspace.nufft_forward(z, k), kspace.ndft(z, k)) < 2e-3


def test_ndft_scale_is_orthonormal():
    # with every grid frequency sampled once, the NDFT is a unitary DFT
    shape = (6, 4)
    kk = np.stack(np.meshgrid(*[np.fft.fftfreq(n) for n in shape], indexing="ij"), -1).reshape(-1, 2)
    A = np.stack([kspace.ndft(e.reshape(shape), kk) for e in np.eye(24)], axis=1)
    assert np.allclose(A.conj().T @ A, np.eye(24), atol=1e-12)


@pytest.mark.parametrize("shape", [(16, 12), (8, 10, 6)])
def test_adjoint_identity(shape):
    g = np.random.default_rng(4)
    k = radial_spokes_2d(0, 13, 16) if len(shape) == 2 else radial_spokes_3d(0, 13, 8)
    z = _rand_c(g, shape)
    y = _rand_c(g, k.shape[0])
    lhs = np.vdot(y, kspace.nufft_forward(z, k))
    rhs = np.vdot(kspace.nufft_adjoint(y, k, shape), z)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_edge_samples_wrap():
    # k = -0.5 sits on the grid edge: kappa = -G/2, taps wrap periodically
    shape = (8, 8)
    k = np.array([[-0.5, -0.5], [-0.5, 0.49], [0.0, 0.0]], dtype=np.float32)
    g = np.random.default_rng(5)
    z = _rand_c(g, shape)
    A = dense.nufft_matrix(k, shape)
    assert np.allclose(kspace.nufft_forward(z, k), A @ z.reshape(-1), atol=1e-12)
