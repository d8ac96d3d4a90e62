"""GPU parity at the full workload sizes, in the launch configuration the
benchmark uses (one plan for all states, library-owned scratch, FP32).

* 96^3, 8 coils, 1 state, 192k radial samples: A and A^H against the FP64
  oracle element by element.
* 160^3, 12 coils, 6 states, 80k..600k samples per state (the benchmark
  workload): the oracle's T_d x at sampled voxels, and properties that hold
  at any size: the adjoint identity of T and of the stacked A, a Hermitian
  normal operator bounded below by lambda, and N = A^H A + lambda I.
"""
import numpy as np
import pytest

import oracle
from synth import WORKLOADS, complex_noise, make_inputs, rng

from gpu_util import pack, rel, say, to_dev, unpack

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def isg():
    import torch
    assert torch.cuda.is_available()
    import paper_2501_16713_amd as isg
    return isg


def _setup(isg, name):
    w = WORKLOADS[name]
    inp = make_inputs(w)
    plan = isg.Plan(w.shape, ncoils=w.ncoils, nphases=w.nphases)
    S = to_dev(inp["S"])
    mots = [plan.motion(to_dev(d)) for d in inp["d"]]
    trs = [plan.traj(to_dev(k)) for k in inp["k"]]
    return w, inp, plan, S, mots, trs


@pytest.fixture(scope="module")
def c2(isg):
    say("setting up sense3d_96")
    return _setup(isg, "sense3d_96")


@pytest.fixture(scope="module")
def c3(isg):
    say("setting up batched_160")
    return _setup(isg, "batched_160")


def test_sense3d_96_forward(c2):
    w, inp, plan, S, mots, trs = c2
    say("sense3d_96 forward vs oracle")
    got = plan.sense_forward(to_dev(inp["x"]), mots, S, trs).cpu().numpy()
    want = pack(oracle.sense.sense_forward(inp["x"], inp["d"], inp["S"], inp["k"]))
    e = rel(got, want)
    say(f"  rel err {e:.2e}")
    assert e < TOL


def test_sense3d_96_adjoint(c2):
    w, inp, plan, S, mots, trs = c2
    say("sense3d_96 adjoint vs oracle")
    M = sum(k.shape[0] for k in inp["k"])
    y = complex_noise((M, w.ncoils), rng(w.cfg, 3))
    got = plan.sense_adjoint(to_dev(y), mots, S, trs).cpu().numpy()
    want = oracle.sense.sense_adjoint(unpack(y, inp["k"]), inp["d"], inp["S"], inp["k"], w.shape)
    e = rel(got, want)
    say(f"  rel err {e:.2e}")
    assert e < TOL


def test_batched_160_warp_sampled(c3):
    """T_{d_p} x at 3000 voxels per state for two states, against the oracle"""
    w, inp, plan, S, mots, trs = c3
    g = np.random.default_rng(160)
    x = to_dev(inp["x"])
    u = oracle.warp.upsample(inp["x"])  # shared by the states
    for p in (0, 5):
        vox = g.choice(int(np.prod(w.shape)), 3000, replace=False)
        got = plan.warp(x, mots[p]).cpu().numpy().reshape(-1)[vox]
        want = oracle.grid.gather(u, oracle.warp.warp_coords(inp["d"][p])[vox])
        e = rel(got, want)
        say(f"  state {p}: sampled warp rel err {e:.2e}")
        assert e < TOL


def test_batched_160_warp_adjoint_identity(c3):
    w, inp, plan, S, mots, trs = c3
    g = np.random.default_rng(1)
    x = (g.standard_normal(w.shape) + 1j * g.standard_normal(w.shape)).astype(np.complex64)
    v = (g.standard_normal(w.shape) + 1j * g.standard_normal(w.shape)).astype(np.complex64)
    Tx = plan.warp(to_dev(x), mots[3]).cpu().numpy().astype(np.complex128)
    THv = plan.warp_adjoint(to_dev(v), mots[3]).cpu().numpy().astype(np.complex128)
    lhs, rhs = np.vdot(v, Tx), np.vdot(THv, x)
    say(f"  <v, T x> vs <T^H v, x>: {abs(lhs - rhs) / abs(lhs):.2e}")
    assert abs(lhs - rhs) < 1e-5 * abs(lhs)


def test_batched_160_sense_adjoint_identity(c3):
    w, inp, plan, S, mots, trs = c3
    g = np.random.default_rng(2)
    x = (g.standard_normal(w.shape) + 1j * g.standard_normal(w.shape)).astype(np.complex64)
    M = sum(k.shape[0] for k in inp["k"])
    y = complex_noise((M, w.ncoils), g)
    Ax = plan.sense_forward(to_dev(x), mots, S, trs).cpu().numpy().astype(np.complex128)
    AHy = plan.sense_adjoint(to_dev(y), mots, S, trs).cpu().numpy().astype(np.complex128)
    lhs, rhs = np.vdot(y, Ax), np.vdot(AHy, x)
    say(f"  <y, A x> vs <A^H y, x>: {abs(lhs - rhs) / abs(lhs):.2e}")
    assert abs(lhs - rhs) < 1e-5 * abs(lhs)


def test_batched_160_normal_properties(c3):
    import torch
    w, inp, plan, S, mots, trs = c3
    lam = w.lam
    g = np.random.default_rng(3)
    x = (g.standard_normal(w.shape) + 1j * g.standard_normal(w.shape)).astype(np.complex64)
    z = (g.standard_normal(w.shape) + 1j * g.standard_normal(w.shape)).astype(np.complex64)
    xd, zd = to_dev(x), to_dev(z)
    Nx = plan.normal(xd, lam, mots, S, trs).cpu().numpy().astype(np.complex128)
    Nz = plan.normal(zd, lam, mots, S, trs).cpu().numpy().astype(np.complex128)
    a, b = np.vdot(z, Nx), np.conj(np.vdot(x, Nz))
    say(f"  Hermitian: {abs(a - b) / abs(a):.2e}")
    assert abs(a - b) < 1e-5 * abs(a)
    q = np.vdot(x, Nx)
    assert abs(q.imag) < 1e-5 * abs(q)
    assert q.real >= lam * np.vdot(x, x).real
    # N = A^H A + lambda I, composed through the forward and adjoint entry points
    y = plan.sense_forward(xd, mots, S, trs)
    comp = plan.sense_adjoint(y, mots, S, trs).cpu().numpy().astype(np.complex128) + lam * x
    e = rel(Nx, comp)
    say(f"  N vs A^H A + lambda I: {e:.2e}")
    assert e < TOL
    torch.cuda.synchronize()
