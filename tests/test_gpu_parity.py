"""GPU parity of every operator against the FP64 oracle, through the C ABI,
on seeded inputs at sizes the oracle finishes in seconds.  Shapes are chosen
so that the spread tiles and FFT line tiles have ragged tails.

Tolerance: 1e-5 relative L2 for FP32 operators against FP64."""
import numpy as np
import pytest

import oracle
from synth import (bump_displacement, coil_maps, ellipsoid_phantom, make_inputs, radial_spokes_2d,
                   radial_spokes_3d, rng, small_workload, WORKLOADS, uniform_samples)

from gpu_util import pack, rel, say, to_dev, unpack

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def isg():
    import torch
    assert torch.cuda.is_available()
    import paper_2501_16713_amd as isg
    return isg


def _rand_c(g, shape):
    return (g.standard_normal(shape) + 1j * g.standard_normal(shape)).astype(np.complex64)


# --------------------------------------------------------------------------
# image-space gridding
# --------------------------------------------------------------------------
def test_warp_2d_workload(isg):
    """the 2D warp workload: 64x64 ellipses, 4 bumps sigma 8, max |d| 3"""
    w = WORKLOADS["warp2d_64"]
    inp = make_inputs(w, with_traj=False)
    x, d = inp["x"], inp["d"][0]
    say("warp2d_64: forward + adjoint")
    plan = isg.Plan(w.shape)
    mo = plan.motion(to_dev(d))
    got = plan.warp(to_dev(x), mo).cpu().numpy()
    assert rel(got, oracle.warp.warp(x, d)) < TOL
    v = _rand_c(np.random.default_rng(1), w.shape)
    got_a = plan.warp_adjoint(to_dev(v), mo).cpu().numpy()
    assert rel(got_a, oracle.warp.warp_adjoint(v, d)) < TOL


@pytest.mark.parametrize("shape,dmax", [((24, 20, 36), 4.0), ((16, 16, 16), 0.0), ((40, 32, 24), 9.0)])
def test_warp_3d(isg, shape, dmax):
    say(f"warp3d {shape} dmax {dmax}")
    g = rng(11, 1)
    x = ellipsoid_phantom(shape, 10, rng(11, 0)).astype(np.complex64)
    d = bump_displacement(shape, 4, shape[0] / 5, dmax, g) if dmax > 0 else \
        np.zeros((3,) + shape, dtype=np.float32)
    plan = isg.Plan(shape)
    mo = plan.motion(to_dev(d))
    assert rel(plan.warp(to_dev(x), mo).cpu().numpy(), oracle.warp.warp(x, d)) < TOL
    v = _rand_c(g, shape)
    assert rel(plan.warp_adjoint(to_dev(v), mo).cpu().numpy(), oracle.warp.warp_adjoint(v, d)) < TOL


def test_warp_integer_shift_and_wrap(isg):
    """integer d moves whole taps; large d wraps around the periodic grid"""
    shape = (16, 24, 20)
    g = np.random.default_rng(3)
    x = _rand_c(g, shape)
    d = np.stack([np.full(shape, s, np.float32) for s in (3.0, -17.0, 41.5)])
    plan = isg.Plan(shape)
    mo = plan.motion(to_dev(d))
    assert rel(plan.warp(to_dev(x), mo).cpu().numpy(), oracle.warp.warp(x, d)) < TOL


def test_warp_adjoint_identity(isg):
    shape = (32, 24, 40)
    g = np.random.default_rng(4)
    d = bump_displacement(shape, 5, 6.0, 6.0, g)
    x, y = _rand_c(g, shape), _rand_c(g, shape)
    plan = isg.Plan(shape)
    mo = plan.motion(to_dev(d))
    Tx = plan.warp(to_dev(x), mo).cpu().numpy().astype(np.complex128)
    THy = plan.warp_adjoint(to_dev(y), mo).cpu().numpy().astype(np.complex128)
    lhs, rhs = np.vdot(y, Tx), np.vdot(THy, x)
    assert abs(lhs - rhs) < 1e-5 * abs(lhs)


@pytest.mark.parametrize("shape", [(40, 36), (16, 20, 24)])
def test_warp_grad_d(isg, shape):
    say(f"grad_d {shape}")
    g = np.random.default_rng(5)
    x = ellipsoid_phantom(shape, 10, rng(12, 0)).astype(np.complex64)
    d = bump_displacement(shape, 3, shape[0] / 4, 3.0, g)
    v = _rand_c(g, shape)
    plan = isg.Plan(shape)
    mo = plan.motion(to_dev(d))
    got = plan.warp_grad_d(to_dev(x), to_dev(v), mo).cpu().numpy()
    want = oracle.warp.warp_grad_d(x, d, v)
    assert np.linalg.norm(got - want) < TOL * np.linalg.norm(want)


# --------------------------------------------------------------------------
# nonrigid SENSE
# --------------------------------------------------------------------------
def _small_sense(shape=(16, 20, 24), C=3, P=2):
    ndim = len(shape)
    w = small_workload(shape=shape, ncoils=C, nphases=P, spokes=(30, 45, 20)[:P], readout=max(shape))
    if ndim == 3:
        return w, make_inputs(w)
    inp = make_inputs(w, with_traj=False)
    inp["k"] = [radial_spokes_2d(0, 25, 48), uniform_samples(700, 2, np.random.default_rng(9))][:P]
    return w, inp


@pytest.mark.parametrize("shape,C,P", [((16, 20, 24), 3, 2), ((24, 18, 20), 5, 3), ((32, 40), 4, 2)])
def test_sense_forward_adjoint(isg, shape, C, P):
    say(f"sense {shape} C={C} P={P}")
    w, inp = _small_sense(shape, C, P)
    plan = isg.Plan(shape, ncoils=C, nphases=P)
    S = to_dev(inp["S"])
    mots = [plan.motion(to_dev(d)) for d in inp["d"]]
    trs = [plan.traj(to_dev(k)) for k in inp["k"]]
    y = plan.sense_forward(to_dev(inp["x"]), mots, S, trs).cpu().numpy()
    want = oracle.sense.sense_forward(inp["x"], inp["d"], inp["S"], inp["k"])
    assert rel(y, pack(want)) < TOL
    g = np.random.default_rng(2)
    yr = _rand_c(g, y.shape)
    xa = plan.sense_adjoint(to_dev(yr), mots, S, trs).cpu().numpy()
    want_a = oracle.sense.sense_adjoint(unpack(yr, inp["k"]), inp["d"], inp["S"], inp["k"], shape)
    assert rel(xa, want_a) < TOL


def test_samples_on_grid_lines(isg):
    """Readouts along the array axes at (j - L/2)/L: in FP64 some grid
    coordinates G k fall a few 1e-8 below an integer, so their FP32 fraction
    rounds to 1.  The taps must stay those of the FP64 cell (the first tap
    keeps the kernel's non-zero edge value), sample by sample."""
    shape, C = (36, 40, 48), 2
    G = [2 * n for n in shape]
    ks = []
    for a, L in ((0, 36), (1, 40), (2, 48)):
        k = np.zeros((L, 3), dtype=np.float32)
        k[:, a] = (np.arange(-L // 2, L // 2) / L).astype(np.float32)
        ks.append(k)
    k = np.concatenate(ks)
    kap = k.astype(np.float64) * np.array(G)
    assert ((kap - np.floor(kap)).astype(np.float32) >= 1.0).any()  # the case is exercised
    x = ellipsoid_phantom(shape, 10, rng(41, 0)).astype(np.complex64)
    S = coil_maps(shape, C, rng(41, 2))
    d = np.zeros((3,) + shape, dtype=np.float32)
    say("samples on grid lines")
    plan = isg.Plan(shape, ncoils=C)
    mo, tr = plan.motion(to_dev(d)), plan.traj(to_dev(k))
    y = plan.sense_forward(to_dev(x), [mo], to_dev(S), [tr]).cpu().numpy()
    want = pack(oracle.sense.sense_forward(x, [d], S, [k]))
    per_sample = np.linalg.norm(y - want, axis=1) / np.linalg.norm(want, axis=1).max()
    assert per_sample.max() < TOL
    yr = _rand_c(np.random.default_rng(5), y.shape)
    xa = plan.sense_adjoint(to_dev(yr), [mo], to_dev(S), [tr]).cpu().numpy()
    assert rel(xa, oracle.sense.sense_adjoint(unpack(yr, [k]), [d], S, [k], shape)) < TOL


def test_normal_operator(isg):
    shape, C, P = (16, 20, 24), 3, 2
    say("normal small")
    w, inp = _small_sense(shape, C, P)
    plan = isg.Plan(shape, ncoils=C, nphases=P)
    S = to_dev(inp["S"])
    mots = [plan.motion(to_dev(d)) for d in inp["d"]]
    trs = [plan.traj(to_dev(k)) for k in inp["k"]]
    lam = 0.05
    got = plan.normal(to_dev(inp["x"]), lam, mots, S, trs).cpu().numpy()
    want = oracle.sense.normal(inp["x"], lam, inp["d"], inp["S"], inp["k"])
    e = rel(got, want)
    say(f"  normal rel err {e:.2e}")
    assert e < TOL


def _cg_problem(isg):
    shape, C, P = (16, 16, 16), 3, 2
    w, inp = _small_sense(shape, C, P)
    plan = isg.Plan(shape, ncoils=C, nphases=P)
    S = to_dev(inp["S"])
    mots = [plan.motion(to_dev(d)) for d in inp["d"]]
    trs = [plan.traj(to_dev(k)) for k in inp["k"]]
    ys = oracle.sense.sense_forward(inp["x"], inp["d"], inp["S"], inp["k"])
    y = pack(ys).astype(np.complex64)
    return shape, inp, plan, S, mots, trs, y


# Bounds on the FP32 CG iterate's relative distance from the FP64 oracle's
# after 8 iterations.  lambda_max of this problem's normal operator is about
# 52 (power iteration on the oracle), so kappa = (52 + lambda)/lambda is 11.4,
# 105 and 5200; CG amplifies the FP32 operator's ~1e-6 relative error (and
# the FP32 rounding of its vectors) by up to about k kappa, and how much of
# that bound is reached depends on the rounding pattern.  Measured on MI355X
# with two image-space spreads that sum in different orders: 9.8e-6 and
# 1.8e-5, 6.0e-5 and 3.3e-4, 5.3e-4 and 4.8e-4 (x0 = 0), and 1.3e-6 (x0 != 0,
# lambda 0.5, 5 iterations).  Each bound is about 3x the larger measured
# value, far below k kappa 1e-6 for the small lambdas, so a defect of about
# 1e-3 relative in one iteration fails.
_CG_TOL = {5.0: 6e-5, 0.5: 1e-3, 1e-2: 2e-3}
_CG_TOL_X0 = 1e-5


def _cg_tol(lam):
    return _CG_TOL[lam]


@pytest.mark.parametrize("lam", [5.0, 0.5, 1e-2])
def test_cg_solve(isg, lam):
    tol = _cg_tol(lam)
    say(f"cg small lam={lam} tol={tol:.1e}")
    shape, inp, plan, S, mots, trs, y = _cg_problem(isg)
    iters = 8
    x, hist = plan.cg_solve(to_dev(y), mots, S, trs, lam, iters)
    yo = unpack(y.astype(np.complex128), inp["k"])
    b = oracle.sense.sense_adjoint(yo, inp["d"], inp["S"], inp["k"], shape)
    xo, ho = oracle.cg.cg(lambda v: oracle.sense.normal(v, lam, inp["d"], inp["S"], inp["k"]), b, iters)
    e = rel(x.cpu().numpy(), xo)
    eh = float(np.max(np.abs(np.array(hist) - ho)) / ho[0])
    say(f"  iterate rel err {e:.2e}; residual history rel err "
        f"{np.max(np.abs(np.array(hist) - ho) / np.array(ho)):.2e}, against ||r_0|| {eh:.2e}")
    assert e < tol
    # the recursively updated residual norms, against the initial residual
    # (FP64 inner products of FP32 vectors: about 1e-6 per iteration)
    assert eh < max(tol, 1e-4)


def test_cg_from_nonzero_start(isg):
    """CG from x0 != 0 (r0 = b - N x0 needs an application of N; from x0 = 0
    the solver skips it) against the oracle's CG from the same x0"""
    lam, iters = 0.5, 5
    tol = _CG_TOL_X0
    shape, inp, plan, S, mots, trs, y = _cg_problem(isg)
    g = np.random.default_rng(11)
    x0 = 0.1 * _rand_c(g, shape)
    x, hist = plan.cg_solve(to_dev(y), mots, S, trs, lam, iters, x0=to_dev(x0))
    yo = unpack(y.astype(np.complex128), inp["k"])
    b = oracle.sense.sense_adjoint(yo, inp["d"], inp["S"], inp["k"], shape)
    xo, ho = oracle.cg.cg(lambda v: oracle.sense.normal(v, lam, inp["d"], inp["S"], inp["k"]), b, iters,
                          x0=x0.astype(np.complex128))
    e = rel(x.cpu().numpy(), xo)
    say(f"  x0 != 0: iterate rel err {e:.2e}, initial residual {hist[0]:.6e} vs {ho[0]:.6e}")
    assert e < tol
    assert abs(hist[0] - ho[0]) < 1e-5 * ho[0]


def test_cg_graph_replay_matches_eager(isg, monkeypatch):
    """the HIP-graph replay of a CG iteration equals eager launches"""
    import torch
    shape, inp, plan, S, mots, trs, y = _cg_problem(isg)
    xg, hg = plan.cg_solve(to_dev(y), mots, S, trs, 0.1, 6)
    monkeypatch.setenv("ISG_NO_GRAPH", "1")
    xe, he = plan.cg_solve(to_dev(y), mots, S, trs, 0.1, 6)
    # the same kernels in the same order with fixed-order reductions (the
    # spreads use no atomics): replay and eager launches agree bit for bit
    assert torch.equal(xg, xe)
    assert hg == he


def test_cg_breakdown_is_reported(isg):
    """a negative lambda larger than the spectrum makes Re<p, N p> < 0"""
    shape, inp, plan, S, mots, trs, y = _cg_problem(isg)
    with pytest.raises(isg.IsgError, match="BREAKDOWN"):
        plan.cg_solve(to_dev(y), mots, S, trs, -1e3, 3)
