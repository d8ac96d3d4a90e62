"""Edge cases of the SENSE operators through the C ABI, against the FP64
oracle (or an exact expectation) on a small 3D problem with ragged tiles:

* a single sample;
* many samples at one k-space point (a cell whose spread sums every sample;
  with a small spread chunk the tile is split into partial tiles and reduced);
* samples exactly at k = -0.5 on every axis (the wrap of the oversampled
  grid) and at the origin;
* zero data (exact zeros out, also with half-precision grids, whose scales
  then fall back to 1);
* an empty trajectory is refused.

Tolerance: 1e-5 relative L2 for FP32 operators against FP64."""
import numpy as np
import pytest

import oracle
from synth import make_inputs, rng, small_workload

from gpu_util import pack, rel, say, to_dev, unpack

pytestmark = pytest.mark.gpu

TOL = 1e-5
SHAPE = (16, 20, 24)
C = 3


@pytest.fixture(scope="module")
def base():
    import torch
    assert torch.cuda.is_available()
    import paper_2501_16713_amd as isg
    w = small_workload(shape=SHAPE, ncoils=C, nphases=1, spokes=(30,), readout=max(SHAPE))
    inp = make_inputs(w)
    return isg, inp


def _check(isg, inp, k, chunk=None, storage="fp32", tol=TOL):
    """forward and adjoint of one state with trajectory k against the oracle"""
    plan = isg.Plan(SHAPE, ncoils=C, nphases=1, storage=storage)
    if chunk is not None:
        plan.set_option("spread_chunk", chunk)
    S = to_dev(inp["S"])
    mo, tr = plan.motion(to_dev(inp["d"][0])), plan.traj(to_dev(k))
    y = plan.sense_forward(to_dev(inp["x"]), [mo], S, [tr]).cpu().numpy()
    want = pack(oracle.sense.sense_forward(inp["x"], [inp["d"][0]], inp["S"], [k]))
    ef = rel(y, want)
    g = rng(100, 3, 7)
    yr = (g.standard_normal(y.shape) + 1j * g.standard_normal(y.shape)).astype(np.complex64)
    xa = plan.sense_adjoint(to_dev(yr), [mo], S, [tr]).cpu().numpy()
    want_a = oracle.sense.sense_adjoint(unpack(yr, [k]), [inp["d"][0]], inp["S"], [k], SHAPE)
    ea = rel(xa, want_a)
    say(f"  M={k.shape[0]} chunk={chunk} {storage}: A rel err {ef:.2e}, A^H rel err {ea:.2e}")
    assert ef < tol and ea < tol
    return plan


def test_single_sample(base):
    isg, inp = base
    k = np.array([[0.137, -0.291, 0.402]], dtype=np.float32)
    _check(isg, inp, k)


@pytest.mark.parametrize("chunk", [None, 32])
def test_samples_at_one_point(base, chunk):
    """600 samples at one point (plus a few elsewhere): the tile of that point
    is split into partial tiles when the chunk is smaller than its visits"""
    isg, inp = base
    g = rng(100, 4, 1)
    pile = np.tile(np.array([[0.031, -0.047, 0.012]], dtype=np.float32), (600, 1))
    other = (g.random((40, 3)) - 0.5).astype(np.float32)
    k = np.concatenate([pile[:300], other, pile[300:]]).astype(np.float32)
    _check(isg, inp, k, chunk=chunk)


def test_samples_on_the_wrap_and_origin(base):
    """k = -0.5 on every axis puts the taps across the periodic wrap of the
    oversampled grid; the origin is the densest point of radial sampling"""
    isg, inp = base
    k = np.array([[-0.5, -0.5, -0.5], [-0.5, 0.0, 0.25], [0.0, -0.5, -0.125], [0.0, 0.0, 0.0],
                  [0.4999, -0.5, 0.4999], [-0.25, 0.25, -0.5]], dtype=np.float32)
    _check(isg, inp, k)


@pytest.mark.parametrize("storage", ["fp32", "fp16", "bf16"])
def test_zero_data(base, storage):
    """zero image and zero data give exact zeros (half precision: the input
    and spread scales fall back to 1 for zero data)"""
    import torch
    isg, inp = base
    plan = isg.Plan(SHAPE, ncoils=C, nphases=1, storage=storage)
    S = to_dev(inp["S"])
    mo, tr = plan.motion(to_dev(inp["d"][0])), plan.traj(to_dev(inp["k"][0]))
    x0 = torch.zeros(SHAPE, dtype=torch.complex64, device="cuda")
    y = plan.sense_forward(x0, [mo], S, [tr])
    assert torch.count_nonzero(torch.view_as_real(y)).item() == 0
    y0 = torch.zeros_like(y)
    xa = plan.sense_adjoint(y0, [mo], S, [tr])
    assert torch.count_nonzero(torch.view_as_real(xa)).item() == 0
    n = plan.normal(x0, 1e-3, [mo], S, [tr])
    assert torch.count_nonzero(torch.view_as_real(n)).item() == 0


def test_empty_trajectory_is_refused(base):
    import torch
    isg, inp = base
    plan = isg.Plan(SHAPE, ncoils=C, nphases=1)
    with pytest.raises(isg.IsgError) as e:
        plan.traj(torch.zeros((0, 3), dtype=torch.float32, device="cuda"))
    assert "ISG_ERR_INVALID_ARG" in str(e.value)
