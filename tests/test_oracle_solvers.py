"""Pins of the oracle's wavelet transform, soft threshold, FISTA, power
iteration (Eq. 11, Eq. 13), registration energy (the gradient-based
alternative to the demons step) and the bulk-translation / gridding
reconstruction pieces (section "Motion Capturing for Segmented Data
Acquisitions"), each against something other than itself:

* Haar: a hand-computed 1D example at one and three levels, orthonormality
  of the dense matrix, perfect reconstruction, a constant image;
* soft threshold: hand cases;
* FISTA: the subgradient optimality conditions of its limit, the normal
  equations when lambda = 0, the O(1/k^2) bound of Beck and Teboulle and a
  clear lead over ISTA (the momentum steps);
* power iteration: numpy.linalg.eigvalsh;
* registration: the energy gradient against central finite differences,
  summation by parts of the smoothness term;
* linear phase: the direct NDFT of a shifted compact image (exact sign and
  scale); Pipe-Menon weights: constant on a Cartesian sampling, where
  P w = 1 exactly, and P w -> 1 for most of a random sampling; the
  coil-combined gridding reconstruction returns the image from full Cartesian
  sampling (G^H G = I within the kernel error, sum_c |S_c|^2 = 1);
* Appendix-1 inversion: integer translations (whole-sample rolls, where the
  naive inverse is exact up to the zero-field warp and the normal operator
  does not depend on the shift), and CG on the l2 form well ahead of the
  negated field for a nonrigid one.
"""
import numpy as np
import pytest

from oracle import fista, gridrecon, inversion, kspace, register, wavelet, warp
from synth import bump_displacement, ellipsoid_phantom, rng

R2 = np.sqrt(2.0)


def _rand_c(g, shape):
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


# --------------------------------------------------------------------------
# wavelet
# --------------------------------------------------------------------------
def test_haar_1d_hand_example():
    x = np.arange(1.0, 9.0)  # 1..8
    w1 = wavelet.forward(x, 1).real
    assert np.allclose(w1, [3 / R2, 7 / R2, 11 / R2, 15 / R2, -1 / R2, -1 / R2, -1 / R2, -1 / R2], atol=1e-14)
    w3 = wavelet.forward(x, 3).real
    # level 2 on (3, 7, 11, 15)/sqrt2: (10, 26)/2, (-4, -4)/2; level 3: 36/(2 sqrt2), -16/(2 sqrt2)
    assert np.allclose(w3, [36 / (2 * R2), -16 / (2 * R2), -2, -2, -1 / R2, -1 / R2, -1 / R2, -1 / R2],
                       atol=1e-13)


@pytest.mark.parametrize("shape,levels", [((4, 8), 1), ((8, 8), 2), ((4, 4, 8), 2)])
def test_haar_dense_matrix_is_orthonormal(shape, levels):
    n = int(np.prod(shape))
    Wm = np.stack([wavelet.forward(np.eye(n)[j].reshape(shape), levels).reshape(-1) for j in range(n)], axis=1)
    assert np.allclose(Wm.conj().T @ Wm, np.eye(n), atol=1e-12)
    assert np.allclose(Wm @ Wm.conj().T, np.eye(n), atol=1e-12)


@pytest.mark.parametrize("shape,levels", [((16, 24), 3), ((8, 16, 8), 3), ((32,), 5)])
def test_haar_perfect_reconstruction(shape, levels):
    x = _rand_c(np.random.default_rng(1), shape)
    w = wavelet.forward(x, levels)
    assert np.linalg.norm(wavelet.inverse(w, levels) - x) < 1e-12 * np.linalg.norm(x)
    assert abs(np.linalg.norm(w) - np.linalg.norm(x)) < 1e-12 * np.linalg.norm(x)


def test_haar_constant_image():
    shape, levels = (8, 16, 8), 3
    w = wavelet.forward(np.full(shape, 2.5 + 1j), levels)
    keep = wavelet.approximation_mask(shape, levels)
    assert keep.sum() == 1 * 2 * 1
    assert np.allclose(w[keep], (2.5 + 1j) * 2 ** (levels * 3 / 2), atol=1e-12)
    assert np.max(np.abs(w[~keep])) < 1e-12


def test_haar_refuses_indivisible_lengths():
    with pytest.raises(ValueError):
        wavelet.forward(np.zeros((12, 8)), 3)


# --------------------------------------------------------------------------
# soft threshold, FISTA, power iteration
# --------------------------------------------------------------------------
def test_soft_threshold_hand_cases():
    c = np.array([3 + 4j, 3 + 4j, 3 + 4j, 0j, -2.0 + 0j])
    tau = np.array([1.0, 5.0, 7.0, 1.0, 0.5])
    got = np.array([fista.soft_threshold(ci, ti) for ci, ti in zip(c, tau)])
    assert np.allclose(got, [2.4 + 3.2j, 0, 0, 0, -1.5], atol=1e-15)


def _problem(seed, shape=(4, 4), m=24, cond=None):
    g = np.random.default_rng(seed)
    n = int(np.prod(shape))
    A = _rand_c(g, (m, n)) / np.sqrt(m)
    if cond is not None:  # singular values spread over [1/cond, 1]
        U, _, Vh = np.linalg.svd(A, full_matrices=False)
        A = U @ np.diag(np.geomspace(1.0, 1.0 / cond, n)) @ Vh
    y = _rand_c(g, m)
    AhA = A.conj().T @ A
    b = (A.conj().T @ y).reshape(shape)
    L = 2.0 * np.linalg.eigvalsh(AhA)[-1]
    return A, y, AhA, b, L


def _apply(AhA, shape):
    return lambda v: (AhA @ v.reshape(-1)).reshape(shape)


def _F(A, y, x, lam, levels):
    r = A @ x.reshape(-1) - y
    return fista.objective(float(np.vdot(r, r).real), x, lam, levels)


def test_fista_limit_satisfies_optimality_conditions():
    shape, levels, lam = (4, 4), 1, 2.0
    A, y, AhA, b, L = _problem(0, shape)
    x = fista.fista(_apply(AhA, shape), b, lam, L, 4000, levels)
    u = wavelet.forward(x, levels)
    g = wavelet.forward(2.0 * (_apply(AhA, shape)(x) - b), levels)  # gradient in coefficient space
    keep = wavelet.approximation_mask(shape, levels)
    assert np.max(np.abs(g[keep])) < 1e-8
    nz = (~keep) & (np.abs(u) > 1e-9)
    z = (~keep) & ~nz
    assert nz.any() and z.any()  # both cases occur
    assert np.max(np.abs(g[nz] + lam * u[nz] / np.abs(u[nz]))) < 1e-7
    assert np.max(np.abs(g[z])) <= lam * (1 + 1e-9)


def test_fista_without_penalty_solves_the_normal_equations():
    shape = (4, 4)
    A, y, AhA, b, L = _problem(1, shape)
    x = fista.fista(_apply(AhA, shape), b, 0.0, L, 3000, 1)
    want = np.linalg.solve(AhA, b.reshape(-1)).reshape(shape)
    assert np.linalg.norm(x - want) < 1e-9 * np.linalg.norm(want)


def test_fista_rate_and_lead_over_ista():
    """F(x_k) - F* <= 2 L ||x0 - x*||^2 / (k + 1)^2 (Beck and Teboulle), and
    after 40 iterations on an ill-conditioned problem FISTA's gap is well
    below plain ISTA's (no momentum)"""
    shape, levels, lam = (4, 4), 1, 0.05
    A, y, AhA, b, L = _problem(2, shape, m=32, cond=300.0)
    ap = _apply(AhA, shape)
    xs = fista.fista(ap, b, lam, L, 20000, levels)
    Fs = _F(A, y, xs, lam, levels)
    for k in (5, 20, 40, 100):
        gap = _F(A, y, fista.fista(ap, b, lam, L, k, levels), lam, levels) - Fs
        assert gap <= 2 * L * np.linalg.norm(xs) ** 2 / (k + 1) ** 2
    x = np.zeros(shape, dtype=np.complex128)
    for _ in range(40):  # ISTA
        x = fista.prox(x - 2.0 * (ap(x) - b) / L, lam / L, levels)
    gap_ista = _F(A, y, x, lam, levels) - Fs
    gap_fista = _F(A, y, fista.fista(ap, b, lam, L, 40, levels), lam, levels) - Fs
    assert gap_fista < 0.5 * gap_ista


def test_power_iteration_matches_eigvalsh():
    g = np.random.default_rng(3)
    B = _rand_c(g, (12, 12))
    N = B.conj().T @ B + np.diag(np.linspace(0, 30, 12))
    lam, v = fista.power_iteration(lambda u: (N @ u.reshape(-1)).reshape(3, 4), np.ones((3, 4)), 300)
    want = np.linalg.eigvalsh(N)[-1]
    assert abs(lam - want) < 1e-10 * want
    assert abs(np.linalg.norm(v) - 1.0) < 1e-12


# --------------------------------------------------------------------------
# registration energy
# --------------------------------------------------------------------------
def _safe(d, h, alpha=2):
    f = np.mod(alpha * (np.indices(d.shape[1:]) + d), 1.0)
    return (f > alpha * h * 1.5) & (f < 1 - alpha * h * 1.5)


def test_registration_gradient_matches_finite_differences():
    shape, mu, h = (16, 20), 0.3, 1e-4
    ref = ellipsoid_phantom(shape, 6, rng(70, 0))
    d_true = bump_displacement(shape, 3, 4.0, 2.0, rng(70, 1)).astype(np.float64)
    mov = warp.warp(ref, d_true)
    d = 0.6 * d_true + 0.1
    grad = register.energy_grad(d, ref, mov, mu)
    g = np.random.default_rng(4)
    v = g.standard_normal(d.shape) * _safe(d, h)
    fd = (register.energy(d + h * v, ref, mov, mu) - register.energy(d - h * v, ref, mov, mu)) / (2 * h)
    assert abs(fd - np.sum(grad * v)) < 1e-6 * abs(fd)


def test_smoothness_summation_by_parts():
    g = np.random.default_rng(5)
    d = g.standard_normal((3, 6, 5, 8))
    lhs = register.smoothness(d)
    rhs = sum(np.sum(d[i] * register.neg_laplacian(d[i])) for i in range(3))
    assert abs(lhs - rhs) < 1e-10 * lhs


def test_gradient_descent_lowers_the_energy():
    shape = (16, 16)
    ref = ellipsoid_phantom(shape, 6, rng(71, 0))
    d_true = bump_displacement(shape, 2, 4.0, 1.5, rng(71, 1)).astype(np.float64)
    mov = warp.warp(ref, d_true)
    d, hist = register.gradient_descent(ref, mov, np.zeros_like(d_true), 0.05, 0.02, 15)
    assert hist[-1] < 0.5 * hist[0]
    assert np.linalg.norm(d - d_true) < np.linalg.norm(d_true)


# --------------------------------------------------------------------------
# linear phase, density compensation
# --------------------------------------------------------------------------
def test_linear_phase_is_the_ndft_of_the_shifted_object():
    shape = (12, 10)
    g = np.random.default_rng(6)
    z = np.zeros(shape, dtype=np.complex128)
    z[3:7, 2:6] = _rand_c(g, (4, 4))  # compact support: a shift by (2, -1) does not wrap
    t = np.array([2.0, -1.0])
    zs = np.roll(z, (2, -1), axis=(0, 1))  # z[x - t]
    k = g.uniform(-0.5, 0.5, (40, 2))
    assert np.allclose(kspace.ndft(zs, k), gridrecon.phase(k, t) * kspace.ndft(z, k), atol=1e-12)


def test_dcf_is_uniform_on_cartesian_samples_and_a_fixed_point():
    n = 16
    ax = (np.arange(n) - n // 2) / n
    k = np.stack(np.meshgrid(ax, ax, indexing="ij"), axis=-1).reshape(-1, 2)
    w = gridrecon.dcf(k, (n, n), 12)
    assert np.std(w) < 1e-10 * np.mean(w)
    pw = gridrecon.dcf_apply(w, k, (n, n))
    assert np.max(np.abs(pw - 1.0)) < 1e-10  # the fixed point: P w = 1
    # random samples: the iteration drives P w towards 1 for all but a few
    # isolated samples (the median deviation falls by 100x from 2 to 40
    # iterations)
    g = np.random.default_rng(7)
    kr = g.uniform(-0.5, 0.5, (300, 2))
    med = []
    for it in (2, 10, 40):
        wr = gridrecon.dcf(kr, (n, n), it)
        pw = gridrecon.dcf_apply(wr, kr, (n, n))
        med.append(np.median(np.abs(pw - 1.0)))
    assert med[0] > med[1] > med[2] and med[2] < 1e-3


# --------------------------------------------------------------------------
# Appendix 1: inverting a nonrigid transform
# --------------------------------------------------------------------------
def test_inversion_exact_for_integer_translations():
    """an integer constant field s moves whole samples: T_s x = roll(T_0 x,
    -s) with T_0 the (nearly identity) zero-field warp, which commutes with
    integer rolls.  So the naive inverse T_{-s} T_s x is T_0 T_0 x (with the
    wrong sign it would be rolled by 2s), and the normal operator does not
    depend on s"""
    shape = (12, 10)
    g = np.random.default_rng(8)
    p = _rand_c(g, shape)
    d = np.stack([np.full(shape, 3.0), np.full(shape, -2.0)])
    zero = np.zeros_like(d)
    q = warp.warp(p, d)
    assert np.allclose(q, np.roll(warp.warp(p, zero), (-3, 2), axis=(0, 1)), atol=1e-12)
    assert np.allclose(inversion.naive(q, d), warp.warp(warp.warp(p, zero), zero), atol=1e-12)
    assert np.linalg.norm(inversion.naive(q, d) - p) < 5e-3 * np.linalg.norm(p)
    assert np.allclose(inversion.normal(p, d, 0.25), inversion.normal(p, zero, 0.25), atol=1e-12)
    assert np.linalg.norm(inversion.normal(p, d, 0.25) - 1.25 * p) < 5e-3 * np.linalg.norm(p)


def test_iterative_inverse_beats_the_negated_field():
    """for a nonrigid field the negated field is only a first-order inverse;
    CG on the l2 form recovers the image several times better"""
    from oracle import cg
    shape = (32, 32)
    p = ellipsoid_phantom(shape, 6, rng(75, 0))
    d = bump_displacement(shape, 3, 5.0, 2.5, rng(75, 1)).astype(np.float64)
    q = warp.warp(p, d)
    err_naive = np.linalg.norm(inversion.naive(q, d) - p)
    x, hist = cg.cg(lambda v: inversion.normal(v, d, 1e-4), warp.warp_adjoint(q, d), 30)
    assert hist[-1] < 1e-3 * hist[0]
    assert np.linalg.norm(x - p) < 0.3 * err_naive


def test_grid_recon_inverts_full_cartesian_sampling():
    """with every Cartesian frequency sampled once, G^H G is the identity
    within the kernel's approximation error, so the coil-combined gridding
    reconstruction of noiseless multi-coil data (coil maps with
    sum_c |S_c|^2 = 1) returns the image; a wrong conjugate on S, a dropped
    coil or a phase of the wrong sign fails it by far more"""
    from synth import coil_maps
    n = 16
    shape = (n, n)
    ax = (np.arange(n) - n // 2) / n
    k = np.stack(np.meshgrid(ax, ax, indexing="ij"), axis=-1).reshape(-1, 2)
    g = np.random.default_rng(9)
    x = _rand_c(g, shape)
    S = coil_maps(shape, 3, rng(76, 0)).astype(np.complex128)
    assert np.allclose(np.sum(np.abs(S) ** 2, axis=0), 1.0, atol=1e-6)
    y = np.stack([kspace.nufft_forward(S[c] * x, k) for c in range(3)])
    rec = gridrecon.grid_recon(y, k, S, shape)
    assert np.linalg.norm(rec - x) < 5e-3 * np.linalg.norm(x)
    # translated data corrected by the matching phase gives the same image
    t = np.array([1.5, -0.75])
    yt = gridrecon.phase(k, t)[None] * y
    assert np.allclose(gridrecon.grid_recon(yt, k, S, shape, t=t), rec, atol=1e-10)
    assert np.linalg.norm(gridrecon.grid_recon(yt, k, S, shape) - x) > 0.1 * np.linalg.norm(x)
    # density weights scale sample by sample: w = 2 doubles the image
    assert np.allclose(gridrecon.grid_recon(y, k, S, shape, w=2.0 * np.ones(k.shape[0])), 2.0 * rec, atol=1e-10)
