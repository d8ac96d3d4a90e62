"""Pins of the oracle's nonrigid SENSE operators (Eq. 10), the l2 normal
operator of Eq. 11, conjugate gradients and the loss gradients.

* A_p equals the product of the brute-force dense matrices G_p diag(S_c) T_p;
* the stacked forward-adjoint pair and a Hermitian, lambda-bounded normal
  operator;
* sum_c |S_c|^2 = 1 makes S an isometry;
* CG iterates equal the Galerkin (Krylov-optimal) solutions computed with
  dense linear algebra, and converge to numpy.linalg.solve;
* gradients equal central finite differences (grad_d only on components
  whose taps do not cross the kernel's support edge within the step).
"""
import numpy as np
import pytest

from oracle import cg, dense, sense, warp
from synth import bump_displacement, coil_maps, radial_spokes_3d, rng, uniform_samples


def _rand_c(g, shape):
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


def _problem(shape=(6, 4, 8), C=2, P=2, M=(30, 45), seed=0):
    g = np.random.default_rng(seed)
    ds = [bump_displacement(shape, 2, 2.0, 1.7, g) for _ in range(P)]
    S = coil_maps(shape, C, g, dtype=np.complex128)
    ks = [uniform_samples(m, len(shape), g) for m in M]
    return g, ds, S, ks


def test_coil_maps_are_isometry():
    S = coil_maps((10, 12, 8), 5, rng(0, 2), dtype=np.complex128)
    assert np.max(np.abs(np.sum(np.abs(S) ** 2, axis=0) - 1.0)) < 1e-12
    g = np.random.default_rng(0)
    x = _rand_c(g, (10, 12, 8))
    assert abs(np.linalg.norm(S * x) - np.linalg.norm(x)) < 1e-12 * np.linalg.norm(x)


def test_sense_equals_dense_product(rel):
    shape = (4, 6, 4)
    g, ds, S, ks = _problem(shape, C=2, P=2, M=(20, 25))
    x = _rand_c(g, shape)
    ys = sense.sense_forward(x, ds, S, ks)
    for p in range(2):
        T = dense.warp_matrix(ds[p])
        Gm = dense.nufft_matrix(ks[p], shape)
        for c in range(2):
            want = Gm @ (S[c].reshape(-1) * (T @ x.reshape(-1)))
            assert rel(ys[p][c], want) < 1e-12


def test_stacked_adjoint_identity():
    shape = (6, 4, 8)
    g, ds, S, ks = _problem(shape)
    x = _rand_c(g, shape)
    ys = [_rand_c(g, (2, m)) for m in (30, 45)]
    Ax = sense.sense_forward(x, ds, S, ks)
    lhs = sum(np.vdot(y, a) for y, a in zip(ys, Ax))
    rhs = np.vdot(sense.sense_adjoint(ys, ds, S, ks, shape), x)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_normal_operator_hermitian_and_bounded():
    shape = (6, 4, 8)
    g, ds, S, ks = _problem(shape)
    lam = 0.3
    x, z = _rand_c(g, shape), _rand_c(g, shape)
    Nx, Nz = sense.normal(x, lam, ds, S, ks), sense.normal(z, lam, ds, S, ks)
    a, b = np.vdot(z, Nx), np.conj(np.vdot(x, Nz))
    assert abs(a - b) <= 1e-12 * abs(a)
    q = np.vdot(x, Nx)
    assert abs(q.imag) <= 1e-12 * abs(q)
    assert q.real >= lam * np.vdot(x, x).real * (1 - 1e-12)


def _dense_normal(shape, lam, ds, S, ks):
    n = int(np.prod(shape))
    cols = [sense.normal(e.reshape(shape), lam, ds, S, ks).reshape(-1) for e in np.eye(n)]
    return np.stack(cols, axis=1)


def test_cg_iterates_are_krylov_galerkin_solutions():
    shape = (4, 4, 4)
    g, ds, S, ks = _problem(shape, C=2, P=2, M=(20, 30), seed=3)
    lam = 0.05
    Nd = _dense_normal(shape, lam, ds, S, ks)
    b = _rand_c(g, shape).reshape(-1)
    for iters in (1, 3, 6):
        x, _ = cg.cg(lambda v: Nd @ v, b, iters)
        # K = span{b, Nb, ..., N^{iters-1} b}; x = V (V^H N V)^{-1} V^H b
        K = [b]
        for _ in range(iters - 1):
            K.append(Nd @ K[-1])
        V, _ = np.linalg.qr(np.stack(K, axis=1))
        want = V @ np.linalg.solve(V.conj().T @ Nd @ V, V.conj().T @ b)
        assert np.linalg.norm(x - want) <= 1e-8 * np.linalg.norm(want)


def test_cg_from_nonzero_start_is_shifted_galerkin_solution():
    """from x0 != 0 the iterates are x0 plus the Galerkin solution of
    N e = r0 = b - N x0 over the Krylov space of r0 (a dropped or sign-flipped
    N x0 term in r0 fails this), and they still converge to the direct solve"""
    shape = (4, 4, 4)
    g, ds, S, ks = _problem(shape, C=2, P=2, M=(20, 30), seed=5)
    lam = 0.05
    Nd = _dense_normal(shape, lam, ds, S, ks)
    b = _rand_c(g, shape).reshape(-1)
    x0 = 0.7 * _rand_c(g, shape).reshape(-1)
    r0 = b - Nd @ x0
    for iters in (1, 3, 6):
        x, hist = cg.cg(lambda v: Nd @ v, b, iters, x0=x0)
        K = [r0]
        for _ in range(iters - 1):
            K.append(Nd @ K[-1])
        V, _ = np.linalg.qr(np.stack(K, axis=1))
        want = x0 + V @ np.linalg.solve(V.conj().T @ Nd @ V, V.conj().T @ r0)
        assert np.linalg.norm(x - want) <= 1e-8 * np.linalg.norm(want)
        assert abs(hist[0] - np.linalg.norm(r0)) <= 1e-12 * np.linalg.norm(r0)
    x, _ = cg.cg(lambda v: Nd @ v, b, 200, x0=x0)
    want = np.linalg.solve(Nd, b)
    assert np.linalg.norm(x - want) <= 1e-8 * np.linalg.norm(want)


def test_cg_converges_to_direct_solve():
    shape = (4, 4, 2)
    g, ds, S, ks = _problem(shape, C=2, P=2, M=(20, 30), seed=4)
    lam = 0.5
    Nd = _dense_normal(shape, lam, ds, S, ks)
    b = _rand_c(g, shape)
    x, hist = cg.cg(lambda v: sense.normal(v, lam, ds, S, ks), b, 40)
    want = np.linalg.solve(Nd, b.reshape(-1)).reshape(shape)
    assert np.linalg.norm(x - want) <= 1e-8 * np.linalg.norm(want)
    assert hist[-1] < 1e-8 * hist[0]


def test_grad_x_finite_difference():
    shape = (6, 4, 8)
    g, ds, S, ks = _problem(shape)
    x = _rand_c(g, shape)
    ys = [_rand_c(g, (2, m)) for m in (30, 45)]
    gx, _ = sense.loss_grads(x, ds, S, ks, ys)
    v = _rand_c(g, shape)
    h = 1e-6
    fd = (sense.loss(x + h * v, ds, S, ks, ys) - sense.loss(x - h * v, ds, S, ks, ys)) / (2 * h)
    assert abs(fd - np.vdot(gx, v).real) <= 1e-6 * abs(fd)


def _safe_mask(d, h, alpha=2):
    f = np.mod(alpha * d.astype(np.float64), 1.0)
    return (f > alpha * h * 1.5) & (f < 1 - alpha * h * 1.5)


def test_grad_d_finite_difference():
    shape = (6, 4, 8)
    g, ds, S, ks = _problem(shape, seed=6)
    x = _rand_c(g, shape)
    ys = [_rand_c(g, (2, m)) for m in (30, 45)]
    _, gds = sense.loss_grads(x, ds, S, ks, ys)
    h = 1e-3
    # componentwise on a few safe components
    for p in range(2):
        safe = np.argwhere(_safe_mask(ds[p], h))
        for idx in safe[:: max(1, len(safe) // 6)][:6]:
            idx = tuple(idx)
            dp, dm = [d.astype(np.float64) for d in ds], [d.astype(np.float64) for d in ds]
            dp[p][idx] += h
            dm[p][idx] -= h
            fd = (sense.loss(x, dp, S, ks, ys) - sense.loss(x, dm, S, ks, ys)) / (2 * h)
            # O(h^2) truncation is absolute: scale by the gradient's magnitude
            assert abs(fd - gds[p][idx]) <= 1e-5 * max(abs(fd), 0.1 * np.abs(gds[p]).max())
    # directional derivative along a random direction on safe components
    # |direction| <= 1 so that no perturbed tap moves past the safe margin
    dirs = [np.where(_safe_mask(d, h), g.uniform(-1.0, 1.0, d.shape), 0.0) for d in ds]
    dp = [d.astype(np.float64) + h * e for d, e in zip(ds, dirs)]
    dm = [d.astype(np.float64) - h * e for d, e in zip(ds, dirs)]
    fd = (sense.loss(x, dp, S, ks, ys) - sense.loss(x, dm, S, ks, ys)) / (2 * h)
    an = sum(np.sum(gd * e) for gd, e in zip(gds, dirs))
    assert abs(fd - an) <= 1e-5 * abs(fd)


def test_warp_grad_d_matches_jacobian_fd():
    shape = (8, 6)
    g = np.random.default_rng(8)
    x = _rand_c(g, shape)
    d = g.uniform(-2, 2, (2,) + shape)
    v = _rand_c(g, shape)
    gd = warp.warp_grad_d(x, d, v)
    h = 1e-4
    safe = np.argwhere(_safe_mask(d, h))
    for idx in safe[:10]:
        idx = tuple(idx)
        dp, dm = d.copy(), d.copy()
        dp[idx] += h
        dm[idx] -= h
        fd = (np.vdot(v, warp.warp(x, dp)).real - np.vdot(v, warp.warp(x, dm)).real) / (2 * h)
        assert abs(fd - gd[idx]) <= 1e-6 * max(abs(fd), np.abs(gd).max())
