"""More states than one launch carries (18 > 16): the image-space spread of
sum_p T_p^H w_p then runs in two launches, the second accumulating into the
first's grid, and batched k-space launches carry 16 states and then 2.
Forward, adjoint and normal operator against the FP64 oracle on small 2D and
3D problems with ragged tiles, for one state per k-space launch and for the
largest batch.

Tolerance: 1e-5 relative L2 for FP32 operators against FP64."""
import numpy as np
import pytest

import oracle
from synth import make_inputs, small_workload

from gpu_util import pack, rel, say, to_dev, unpack

pytestmark = pytest.mark.gpu

TOL = 1e-5
C = 2
P = 18


@pytest.fixture(scope="module", params=[(16, 20, 24), (32, 40)], ids=["3d", "2d"])
def case(request):
    import torch
    assert torch.cuda.is_available()
    import paper_2501_16713_amd as isg
    shape = request.param
    w = small_workload(shape=shape, ncoils=C, nphases=P, spokes=tuple(4 + (p % 5) for p in range(P)),
                       readout=16, dmax=2.0)
    inp = make_inputs(w)
    assert len(inp["k"]) == P and len(inp["d"]) == P
    y_ref = oracle.sense.sense_forward(inp["x"], inp["d"], inp["S"], inp["k"])
    g = np.random.default_rng(18)
    yr = (g.standard_normal(pack(y_ref).shape) + 1j * g.standard_normal(pack(y_ref).shape)).astype(np.complex64)
    xa_ref = oracle.sense.sense_adjoint(unpack(yr, inp["k"]), inp["d"], inp["S"], inp["k"], shape)
    lam = 0.05
    n_ref = oracle.sense.normal(inp["x"], lam, inp["d"], inp["S"], inp["k"])
    return isg, shape, inp, y_ref, yr, xa_ref, lam, n_ref


@pytest.mark.parametrize("batch", [1, 16])
def test_eighteen_states(case, batch):
    isg, shape, inp, y_ref, yr, xa_ref, lam, n_ref = case
    say(f"18 states {shape}, phase batch {batch}")
    plan = isg.Plan(shape, ncoils=C, nphases=P)
    plan.set_option("phase_batch", batch)
    S = to_dev(inp["S"])
    mots = [plan.motion(to_dev(d)) for d in inp["d"]]
    trs = [plan.traj(to_dev(k)) for k in inp["k"]]
    y = plan.sense_forward(to_dev(inp["x"]), mots, S, trs).cpu().numpy()
    ef = rel(y, pack(y_ref))
    xa = plan.sense_adjoint(to_dev(yr), mots, S, trs).cpu().numpy()
    ea = rel(xa, xa_ref)
    n = plan.normal(to_dev(inp["x"]), lam, mots, S, trs).cpu().numpy()
    en = rel(n, n_ref)
    say(f"  A {ef:.2e}  A^H {ea:.2e}  N {en:.2e}")
    assert ef < TOL and ea < TOL and en < TOL
