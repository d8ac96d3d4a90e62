"""The allocation-free warp adjoint (isg_warp_adjoint_noalloc), through the
C ABI, against isg_warp_adjoint: the same kernels on a fixed device scratch
array instead of plan memory, so the results agree bit for bit.  Two calls
in a row, the second on a smaller problem (the shared scratch keeps the
first call's contents); then a shape too large for the scratch is refused
with a clear error.  Also checked against the FP64 oracle at 1e-5."""
import numpy as np
import pytest

import oracle
from synth import bump_displacement

from gpu_util import rel, say, to_dev

pytestmark = pytest.mark.gpu


def _case(shape, seed):
    g = np.random.default_rng(seed)
    d = bump_displacement(shape, 3, shape[0] / 4, 3.0, g)
    y = (g.standard_normal(shape) + 1j * g.standard_normal(shape)).astype(np.complex64)
    return d, y


def test_noalloc_matches_warp_adjoint_twice():
    import torch
    import paper_2501_16713_amd as isg
    for shape, seed in (((40, 32, 24), 1), ((48, 40), 2)):
        say(f"noalloc warp adjoint {shape}")
        d, y = _case(shape, seed)
        plan = isg.Plan(shape)
        mo = plan.motion(to_dev(d))
        yd = to_dev(y)
        want = plan.warp_adjoint(yd, mo)
        got = torch.full(shape, complex(float("nan"), float("nan")), dtype=torch.complex64, device="cuda")
        plan.warp_adjoint_noalloc(yd, mo, got)
        torch.cuda.synchronize()
        assert torch.equal(got, want)
        assert rel(got.cpu().numpy(), oracle.warp.warp_adjoint(y, d)) < 1e-5
        plan.close()


def test_noalloc_refuses_shapes_beyond_its_scratch():
    import torch
    import paper_2501_16713_amd as isg
    shape = (96, 96, 96)
    d = np.zeros((3,) + shape, dtype=np.float32)
    plan = isg.Plan(shape)
    mo = plan.motion(to_dev(d))
    y = torch.zeros(shape, dtype=torch.complex64, device="cuda")
    out = torch.zeros_like(y)
    with pytest.raises(isg.IsgError, match="64 MiB"):
        plan.warp_adjoint_noalloc(y, mo, out)
    plan.close()
