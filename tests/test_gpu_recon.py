"""GPU parity of the reconstruction layer against the FP64 oracle, through the
C ABI: the Haar wavelet, wavelet-FISTA and the power iteration (Eq. 11,
Eq. 13), the inversion of a nonrigid transform (Appendix 1), gradient-descent
registration with T_d as the warp, the linear-phase translation correction,
Pipe-Menon density compensation and direct gridding reconstruction (section
"Motion Capturing for Segmented Data Acquisitions").

Tolerances (relative L2 against FP64): 1e-6 for the wavelet (two FP32
roundings per level and axis); 1e-5 for single applications of the FP32
operators; 1e-4 after a few solver iterations (each iteration adds the
operator's ~1e-6 and the iterations are contractions or normalised); the
half-precision storage forms of the gridding reconstruction at the bars of
their adjoints."""
import numpy as np
import pytest

import oracle
from synth import (bump_displacement, coil_maps, ellipsoid_phantom, make_inputs, radial_spokes_2d,
                   radial_spokes_3d, rng, small_workload, WORKLOADS)

from gpu_util import pack, rel, say, to_dev, unpack

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def isg():
    import torch
    assert torch.cuda.is_available()
    import paper_2501_16713_amd as isg
    return isg


def _rand_c(g, shape):
    return (g.standard_normal(shape) + 1j * g.standard_normal(shape)).astype(np.complex64)


# --------------------------------------------------------------------------
# wavelet
# --------------------------------------------------------------------------
@pytest.mark.parametrize("shape,levels", [((64, 48), 1), ((64, 48), 3), ((16, 24, 40), 1), ((16, 24, 40), 3),
                                          ((32, 32, 32), 5)])
def test_wavelet_forward_inverse(isg, shape, levels):
    say(f"wavelet {shape} levels {levels}")
    x = _rand_c(np.random.default_rng(levels), shape)
    plan = isg.Plan(shape)
    w = plan.wavelet_forward(to_dev(x), levels).cpu().numpy()
    assert rel(w, oracle.wavelet.forward(x, levels)) < 1e-6
    v = _rand_c(np.random.default_rng(levels + 10), shape)
    xi = plan.wavelet_inverse(to_dev(v), levels).cpu().numpy()
    assert rel(xi, oracle.wavelet.inverse(v, levels)) < 1e-6
    back = plan.wavelet_inverse(to_dev(w), levels).cpu().numpy()
    assert rel(back, x) < 1e-6


def test_wavelet_refuses_indivisible_levels(isg):
    plan = isg.Plan((16, 24, 40))
    x = to_dev(np.zeros((16, 24, 40), np.complex64))
    with pytest.raises(isg.IsgError):
        plan.wavelet_forward(x, 4)  # 24 is not divisible by 16
    with pytest.raises(isg.IsgError):
        plan.wavelet_inverse(x, 0)


# --------------------------------------------------------------------------
# Appendix 1: inverting a nonrigid transform
# --------------------------------------------------------------------------
def _warp_problem():
    w = WORKLOADS["warp2d_64"]
    inp = make_inputs(w, with_traj=False)
    x, d = inp["x"], inp["d"][0]
    return x, d, oracle.warp.warp(x, d).astype(np.complex64)


def test_warp_cg_matches_oracle_and_beats_naive(isg):
    x, d, q = _warp_problem()
    lam, iters = 1e-3, 12
    say("warp CG 64x64")
    plan = isg.Plan(x.shape)
    mo = plan.motion(to_dev(d))
    p, hist = plan.warp_cg_solve(to_dev(q), mo, lam, iters)
    p = p.cpu().numpy()
    b = oracle.warp.warp_adjoint(q, d)
    want, whist = oracle.cg.cg(lambda v: oracle.inversion.normal(v, d, lam), b, iters)
    assert rel(p, want) < 1e-4
    assert np.allclose(hist, whist, rtol=1e-3, atol=1e-4 * whist[0])
    # the Appendix-1 comparison: the iterative inverse recovers the image far
    # better than the naive one (the negated field)
    naive = plan.warp(to_dev(q), plan.motion(to_dev(-d))).cpu().numpy()
    assert rel(naive, oracle.inversion.naive(q, d)) < 1e-5
    assert rel(p, x) < 0.5 * rel(naive, x)


def test_warp_power_and_fista_match_oracle(isg):
    x, d, q = _warp_problem()
    say("warp power iteration + FISTA 64x64")
    plan = isg.Plan(x.shape)
    mo = plan.motion(to_dev(d))
    v0 = _rand_c(np.random.default_rng(5), x.shape)
    lmax, v = plan.warp_power_iteration(mo, 12, to_dev(v0))
    wl, wv = oracle.fista.power_iteration(lambda u: oracle.inversion.normal(u, d, 0.0), v0, 12)
    assert abs(lmax - wl) < 1e-5 * wl
    assert rel(v.cpu().numpy(), wv) < 1e-4
    L, lam, levels, iters = 2.2 * wl, 1e-3, 3, 10
    p, change = plan.warp_fista_solve(to_dev(q), mo, lam, L, levels, iters)
    b = oracle.warp.warp_adjoint(q, d)
    want = oracle.fista.fista(lambda u: oracle.inversion.normal(u, d, 0.0), b, lam, L, iters, levels)
    assert rel(p.cpu().numpy(), want) < 1e-4
    assert len(change) == iters and all(np.isfinite(change)) and change[-1] < change[0]


# --------------------------------------------------------------------------
# Eq. 11: nonrigid motion-corrected reconstruction with the wavelet penalty
# --------------------------------------------------------------------------
def _sense_problem():
    w = small_workload((16, 16, 16), ncoils=3, nphases=2, spokes=(40, 60))
    inp = make_inputs(w)
    x, ds, S, ks = inp["x"], inp["d"], inp["S"], inp["k"]
    ys = oracle.sense.sense_forward(x, ds, S, ks)
    g = np.random.default_rng(9)
    ys = [y + 0.01 * np.abs(y).max() * _rand_c(g, y.shape) for y in ys]
    return x, ds, S, ks, ys


def test_sense_power_and_fista_match_oracle(isg):
    x, ds, S, ks, ys = _sense_problem()
    say("SENSE power iteration + FISTA 16^3")
    plan = isg.Plan(x.shape, ncoils=S.shape[0], nphases=len(ds))
    mos = [plan.motion(to_dev(d)) for d in ds]
    trs = [plan.traj(to_dev(k)) for k in ks]
    Sd = to_dev(S)
    v0 = _rand_c(np.random.default_rng(6), x.shape)
    apply_n = lambda u: oracle.sense.normal(u, 0.0, ds, S, ks)  # noqa: E731
    lmax, v = plan.power_iteration(mos, Sd, trs, 10, to_dev(v0))
    wl, wv = oracle.fista.power_iteration(apply_n, v0, 10)
    assert abs(lmax - wl) < 1e-5 * wl
    assert rel(v.cpu().numpy(), wv) < 1e-4
    L, lam, levels, iters = 2.2 * wl, 0.02 * wl, 2, 8
    xg, change = plan.fista_solve(to_dev(pack(ys).astype(np.complex64)), mos, Sd, trs, lam, L, levels, iters)
    b = oracle.sense.sense_adjoint(ys, ds, S, ks, x.shape)
    want = oracle.fista.fista(apply_n, b, lam, L, iters, levels)
    assert rel(xg.cpu().numpy(), want) < 1e-4
    # a warm start continues the same iteration count from x0
    x0 = _rand_c(np.random.default_rng(7), x.shape)
    xg2, _ = plan.fista_solve(to_dev(pack(ys).astype(np.complex64)), mos, Sd, trs, lam, L, levels, 3,
                              x0=to_dev(x0))
    assert rel(xg2.cpu().numpy(), oracle.fista.fista(apply_n, b, lam, L, 3, levels, x0=x0)) < 1e-4


# --------------------------------------------------------------------------
# registration
# --------------------------------------------------------------------------
@pytest.mark.parametrize("shape,iters", [((32, 32), 10), ((12, 16, 12), 4)])
def test_registration_matches_oracle(isg, shape, iters):
    say(f"registration {shape} x {iters}")
    ref = ellipsoid_phantom(shape, 6, rng(72, 0)).astype(np.complex64)
    d_true = bump_displacement(shape, 2, shape[0] / 4, 1.5, rng(72, 1))
    mov = oracle.warp.warp(ref, d_true).astype(np.complex64)
    mu, step = 0.05, 0.02
    plan = isg.Plan(shape)
    d, hist = plan.register(to_dev(ref), to_dev(mov), mu, step, iters)
    want, whist = oracle.register.gradient_descent(ref, mov, np.zeros(d_true.shape), mu, step, iters)
    assert rel(d.cpu().numpy(), want) < 1e-4
    assert np.allclose(hist, whist, rtol=1e-4)
    assert hist[-1] < hist[0]


# --------------------------------------------------------------------------
# translation phase, density compensation, gridding reconstruction
# --------------------------------------------------------------------------
def test_shift_phase_in_the_sense_models(isg):
    x, ds, S, ks, ys = _sense_problem()
    say("translation phase 16^3")
    g = np.random.default_rng(8)
    ts = [np.repeat(g.uniform(-2.0, 2.0, (k.shape[0] // 16, 3)), 16, axis=0).astype(np.float32) for k in ks]
    plan = isg.Plan(x.shape, ncoils=S.shape[0], nphases=len(ds))
    mos = [plan.motion(to_dev(d)) for d in ds]
    trs = [plan.traj(to_dev(k)) for k in ks]
    Sd = to_dev(S)
    base = plan.normal(to_dev(x), 0.0, mos, Sd, trs).cpu().numpy()
    for tr, t in zip(trs, ts):
        tr.set_shift(to_dev(t))
    phs = [oracle.gridrecon.phase(k, t) for k, t in zip(ks, ts)]
    got = unpack(plan.sense_forward(to_dev(x), mos, Sd, trs).cpu().numpy(), ks)
    want = [ph[None] * y for ph, y in zip(phs, oracle.sense.sense_forward(x, ds, S, ks))]
    assert rel(np.concatenate([a.ravel() for a in got]), np.concatenate([a.ravel() for a in want])) < 1e-5
    ya = pack(ys).astype(np.complex64)
    got_a = plan.sense_adjoint(to_dev(ya), mos, Sd, trs).cpu().numpy()
    want_a = oracle.sense.sense_adjoint([np.conj(ph)[None] * y for ph, y in zip(phs, ys)], ds, S, ks, x.shape)
    assert rel(got_a, want_a) < 1e-5
    # the phases cancel in the normal operator
    assert rel(plan.normal(to_dev(x), 0.0, mos, Sd, trs).cpu().numpy(), base) < 1e-6
    for tr in trs:
        tr.set_shift(None)
    got0 = plan.sense_adjoint(to_dev(ya), mos, Sd, trs).cpu().numpy()
    assert rel(got0, oracle.sense.sense_adjoint(ys, ds, S, ks, x.shape)) < 1e-5


@pytest.mark.parametrize("case", ["2d", "3d"])
def test_dcf_matches_oracle(isg, case):
    if case == "2d":
        shape, k, iters = (32, 32), radial_spokes_2d(0, 48, 32), 6
    else:
        shape, k, iters = (16, 16, 16), radial_spokes_3d(0, 60, 16), 4
    say(f"dcf {case}")
    plan = isg.Plan(shape)
    tr = plan.traj(to_dev(k))
    w = plan.dcf(tr, iters).cpu().numpy()
    want = oracle.gridrecon.dcf(k, shape, iters)
    assert np.linalg.norm(w - want) < 1e-5 * np.linalg.norm(want)
    assert np.all(plan.dcf(tr, 0).cpu().numpy() == 1.0)


@pytest.mark.parametrize("storage,tol", [("fp32", 1e-5), ("fp16", 5e-4), ("bf16", 4e-3)])
def test_grid_recon_matches_oracle(isg, storage, tol):
    shape, C = (24, 20, 16), 3
    say(f"grid recon {shape} {storage}")
    k = radial_spokes_3d(0, 90, 24)
    S = coil_maps(shape, C, rng(73, 0))
    g = np.random.default_rng(10)
    y = _rand_c(g, (k.shape[0], C))
    t = g.uniform(-1.5, 1.5, (k.shape[0], 3)).astype(np.float32)
    w = oracle.gridrecon.dcf(k, shape, 3).astype(np.float32)
    plan = isg.Plan(shape, ncoils=C, storage=storage)
    tr = plan.traj(to_dev(k))
    got = plan.grid_recon(tr, to_dev(y), to_dev(S)).cpu().numpy()
    assert rel(got, oracle.gridrecon.grid_recon(y.T, k, S, shape)) < tol
    got_w = plan.grid_recon(tr, to_dev(y), to_dev(S), w=to_dev(w)).cpu().numpy()
    assert rel(got_w, oracle.gridrecon.grid_recon(y.T, k, S, shape, w=w)) < tol
    tr.set_shift(to_dev(t))
    got_t = plan.grid_recon(tr, to_dev(y), to_dev(S), w=to_dev(w)).cpu().numpy()
    assert rel(got_t, oracle.gridrecon.grid_recon(y.T, k, S, shape, w=w, t=t)) < tol


def test_low_resolution_navigator(isg):
    """the low-resolution image navigator: the samples near the k-space
    origin of a full-resolution trajectory, re-expressed in cycles/voxel of a
    coarser grid, gridded there"""
    full, low, C = 48, 16, 4
    k = radial_spokes_3d(0, 200, full)
    near = np.all(np.abs(k) * full < low / 2, axis=1)
    kl = (k[near] * (full / low)).astype(np.float32)
    shape = (low,) * 3
    S = coil_maps(shape, C, rng(74, 0))
    y = _rand_c(np.random.default_rng(11), (kl.shape[0], C))
    say(f"iNAV {shape} from {kl.shape[0]} of {k.shape[0]} samples")
    plan = isg.Plan(shape, ncoils=C)
    tr = plan.traj(to_dev(kl))
    w = plan.dcf(tr, 4)
    got = plan.grid_recon(tr, to_dev(y), to_dev(S), w=w).cpu().numpy()
    want = oracle.gridrecon.grid_recon(y.T, kl, S, shape, w=oracle.gridrecon.dcf(kl, shape, 4))
    assert rel(got, want) < 1e-5
