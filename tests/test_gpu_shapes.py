"""GPU parity at the edges of the accepted shapes, against the FP64 oracle:

* 2D axes of 8, 10 and 12 voxels (oversampled 16, 20, 24 cells), where the
  spread tile extents are capped at half the axis, and a 3D axis of 8 voxels
  with the k-space tile extent along axis 1 asked for 16;
* lengths with a prime factor 7 (the general Stockham passes with a
  radix-7 stage), 2D and 3D.

Tolerance 1e-5 relative L2 (FP32 against FP64)."""
import numpy as np
import pytest

import oracle
from synth import bump_displacement, coil_maps, ellipsoid_phantom, rng, uniform_samples

from gpu_util import rel, say, to_dev, unpack

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _rand_c(g, shape):
    return (g.standard_normal(shape) + 1j * g.standard_normal(shape)).astype(np.complex64)


def _inputs(shape, C, M, seed):
    g = np.random.default_rng(seed)
    x = ellipsoid_phantom(shape, 6, rng(50 + seed, 0)).astype(np.complex64)
    d = bump_displacement(shape, 3, max(shape) / 4, 2.5, g)
    S = coil_maps(shape, C, rng(50 + seed, 2))
    k = uniform_samples(M, len(shape), g)
    return g, x, d, S, k


@pytest.mark.parametrize("shape", [(8, 12), (10, 16), (12, 8), (8, 8), (14, 28), (28, 10)])
def test_small_and_radix7_2d(shape):
    import paper_2501_16713_amd as isg
    say(f"2D shape {shape}")
    g, x, d, S, k = _inputs(shape, 3, 400, sum(shape))
    plan = isg.Plan(shape, ncoils=3)
    mo, tr = plan.motion(to_dev(d)), plan.traj(to_dev(k))
    assert rel(plan.warp(to_dev(x), mo).cpu().numpy(), oracle.warp.warp(x, d)) < TOL
    v = _rand_c(g, shape)
    assert rel(plan.warp_adjoint(to_dev(v), mo).cpu().numpy(), oracle.warp.warp_adjoint(v, d)) < TOL
    Sd = to_dev(S)
    y = plan.sense_forward(to_dev(x), [mo], Sd, [tr]).cpu().numpy()
    assert rel(y, oracle.sense.sense_forward(x, [d], S, [k])[0].T) < TOL
    yr = _rand_c(g, y.shape)
    xa = plan.sense_adjoint(to_dev(yr), [mo], Sd, [tr]).cpu().numpy()
    assert rel(xa, oracle.sense.sense_adjoint(unpack(yr, [k]), [d], S, [k], shape)) < TOL


@pytest.mark.parametrize("shape,t1", [((8, 8, 12), 16), ((16, 8, 10), 16), ((14, 12, 16), 8), ((10, 14, 8), 4)])
def test_small_and_radix7_3d(shape, t1):
    import paper_2501_16713_amd as isg
    say(f"3D shape {shape}, k-space tile extent {t1}")
    g, x, d, S, k = _inputs(shape, 2, 500, sum(shape))
    plan = isg.Plan(shape, ncoils=2)
    plan.set_option("ktile_t1", t1)
    mo, tr = plan.motion(to_dev(d)), plan.traj(to_dev(k))
    assert rel(plan.warp(to_dev(x), mo).cpu().numpy(), oracle.warp.warp(x, d)) < TOL
    v = _rand_c(g, shape)
    assert rel(plan.warp_adjoint(to_dev(v), mo).cpu().numpy(), oracle.warp.warp_adjoint(v, d)) < TOL
    Sd = to_dev(S)
    y = plan.sense_forward(to_dev(x), [mo], Sd, [tr]).cpu().numpy()
    assert rel(y, oracle.sense.sense_forward(x, [d], S, [k])[0].T) < TOL
    yr = _rand_c(g, y.shape)
    xa = plan.sense_adjoint(to_dev(yr), [mo], Sd, [tr]).cpu().numpy()
    assert rel(xa, oracle.sense.sense_adjoint(unpack(yr, [k]), [d], S, [k], shape)) < TOL


def test_handles_outlive_their_plan():
    """destroying the plan first detaches its motions and trajectories: their
    destroy calls afterwards free only their own memory, and an apply call
    with a detached handle fails cleanly"""
    import ctypes as C
    import paper_2501_16713_amd as isg
    from paper_2501_16713_amd import _lib
    shape = (16, 16, 16)
    g, x, d, S, k = _inputs(shape, 2, 200, 3)
    lib = _lib.load()
    plan = isg.Plan(shape, ncoils=2)
    mo, tr = plan.motion(to_dev(d)), plan.traj(to_dev(k))
    before = plan.device_bytes()
    mh, th = mo.handle, tr.handle
    mo.handle = tr.handle = None  # take the raw handles over from the wrappers
    assert lib.isg_plan_destroy(plan.handle) == 0
    plan.handle = None
    M = C.c_int64(0)
    assert lib.isg_traj_count(th, C.byref(M)) == 0 and M.value == 200
    a, b, c = C.c_int64(0), C.c_int64(0), C.c_int64(0)
    assert lib.isg_traj_info(th, C.byref(a), C.byref(b), C.byref(c)) == 0 and c.value > 0
    assert lib.isg_motion_destroy(mh) == 0
    assert lib.isg_traj_destroy(th) == 0
    assert before > 0
    # the Python wrappers close dependants first
    plan = isg.Plan(shape, ncoils=2)
    mo, tr = plan.motion(to_dev(d)), plan.traj(to_dev(k))
    plan.close()
    assert mo.handle is None and tr.handle is None


@pytest.mark.parametrize("shape,C", [((16, 20, 24), 1), ((24, 16, 20), 3), ((20, 24, 16), 5), ((16, 16, 32), 12),
                                     ((16, 16, 160), 1)])
def test_register_spread_coil_counts(shape, C):
    """k-space tiles of 8 x 4 x 8 (the register-accumulating spread) with odd
    and even coil counts, one of them a single coil, against the oracle's
    adjoint; several states so the tile-major output holds split tiles too.
    One coil along a last axis of 160 (lines of 320 = 16 x 20) gives the
    coil-reduction epilogue its most outputs per thread (8)."""
    import paper_2501_16713_amd as isg
    say(f"register spread {shape} C={C}")
    g = np.random.default_rng(C)
    S = coil_maps(shape, C, rng(60 + C, 2))
    ds = [bump_displacement(shape, 3, max(shape) / 4, 2.0, g) for _ in range(2)]
    ks = [uniform_samples(1500, 3, g), uniform_samples(300, 3, g) * np.float32(0.25)]
    plan = isg.Plan(shape, ncoils=C, nphases=2)
    plan.set_option("ktile_t1", 4)
    plan.set_option("spread_chunk", 64)
    mots = [plan.motion(to_dev(d)) for d in ds]
    trs = [plan.traj(to_dev(k)) for k in ks]
    y = _rand_c(g, (sum(k.shape[0] for k in ks), C))
    xa = plan.sense_adjoint(to_dev(y), mots, to_dev(S), trs).cpu().numpy()
    want = oracle.sense.sense_adjoint(unpack(y, ks), ds, S, ks, shape)
    assert rel(xa, want) < TOL
