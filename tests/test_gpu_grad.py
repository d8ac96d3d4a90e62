"""Gradients through the torch.autograd wrappers (hand-written adjoint
kernels) against the FP64 oracle's analytic gradients, which the CPU tests
pin to central finite differences.

* small problem: L = sum_p 1/2 ||A_p x - y_p||^2, gradients in x and d_p;
* the warp alone: L = Re <v, T_d x>;
* the 128^3, 8-coil differentiation workload (first state): the gradient of
  the linear functional Re <v, A x> (grad_x = A^H v; grad_d from
  v_img = S^H G^H v), grad_d compared on sampled voxels.
Bar: 1e-5 relative L2 (FP32 against FP64)."""
import numpy as np
import pytest

import oracle
from synth import WORKLOADS, bump_displacement, complex_noise, ellipsoid_phantom, make_inputs, rng, small_workload

from gpu_util import pack, rel, say, to_dev, unpack

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def isg():
    import torch
    assert torch.cuda.is_available()
    import paper_2501_16713_amd as isg
    from paper_2501_16713_amd import autograd  # noqa: F401
    return isg


def test_sense_loss_gradients_small(isg):
    import torch
    from paper_2501_16713_amd.autograd import sense
    w = small_workload(shape=(16, 20, 24), ncoils=3, nphases=2, spokes=(30, 45), readout=24)
    inp = make_inputs(w)
    g = np.random.default_rng(7)
    M = sum(k.shape[0] for k in inp["k"])
    y = complex_noise((M, w.ncoils), g)
    plan = isg.Plan(w.shape, ncoils=w.ncoils, nphases=w.nphases)
    trs = [plan.traj(to_dev(k)) for k in inp["k"]]
    x = to_dev(inp["x"]).requires_grad_(True)
    ds = to_dev(np.stack(inp["d"])).requires_grad_(True)
    Ax = sense(plan, x, ds, to_dev(inp["S"]), trs)
    r = Ax - to_dev(y)
    loss = 0.5 * (r.abs() ** 2).sum()
    loss.backward()
    gx_o, gds_o = oracle.sense.loss_grads(inp["x"], inp["d"], inp["S"], inp["k"], unpack(y, inp["k"]))
    ex = rel(x.grad.cpu().numpy(), gx_o)
    ed = float(np.linalg.norm(ds.grad.cpu().numpy() - np.stack(gds_o)) / np.linalg.norm(np.stack(gds_o)))
    say(f"  grad_x rel err {ex:.2e}, grad_d rel err {ed:.2e}")
    assert ex < TOL and ed < TOL


def test_warp_autograd(isg):
    import torch
    from paper_2501_16713_amd.autograd import warp
    shape = (24, 20, 32)
    g = np.random.default_rng(8)
    x0 = ellipsoid_phantom(shape, 10, rng(13, 0)).astype(np.complex64)
    d0 = bump_displacement(shape, 3, 5.0, 3.0, g)
    v = (g.standard_normal(shape) + 1j * g.standard_normal(shape)).astype(np.complex64)
    plan = isg.Plan(shape)
    x = to_dev(x0).requires_grad_(True)
    d = to_dev(d0).requires_grad_(True)
    y = warp(plan, x, d)
    loss = (torch.conj(to_dev(v)) * y).real.sum()  # Re <v, T x>
    loss.backward()
    ex = rel(x.grad.cpu().numpy(), oracle.warp.warp_adjoint(v, d0))
    gd = oracle.warp.warp_grad_d(x0, d0, v)
    ed = float(np.linalg.norm(d.grad.cpu().numpy() - gd) / np.linalg.norm(gd))
    say(f"  warp grad_x rel err {ex:.2e}, grad_d rel err {ed:.2e}")
    assert ex < TOL and ed < TOL


def test_grad_128_first_state(isg):
    """the 128^3 differentiation workload, first state, sampled grad_d"""
    import torch
    from paper_2501_16713_amd.autograd import sense
    w = WORKLOADS["grad_128"]
    inp = make_inputs(w)
    k0, d0 = inp["k"][0], inp["d"][0]
    g = np.random.default_rng(128)
    v = complex_noise((k0.shape[0], w.ncoils), g)
    plan = isg.Plan(w.shape, ncoils=w.ncoils, nphases=1)
    trs = [plan.traj(to_dev(k0))]
    x = to_dev(inp["x"]).requires_grad_(True)
    ds = to_dev(d0[None]).requires_grad_(True)
    Ax = sense(plan, x, ds, to_dev(inp["S"]), trs)
    loss = (torch.conj(to_dev(v)) * Ax).real.sum()  # Re <v, A x>
    loss.backward()
    say("  oracle S^H G^H v and T^H for grad_128")
    vimg = oracle.sense.coil_adjoint(v.T.astype(np.complex128), inp["S"], k0, w.shape)
    ex = rel(x.grad.cpu().numpy(), oracle.warp.warp_adjoint(vimg, d0))
    vox = g.choice(int(np.prod(w.shape)), 4000, replace=False)
    u = oracle.warp.upsample(inp["x"])
    coords = oracle.warp.warp_coords(d0)[vox]
    gd_o = np.stack([2 * np.real(np.conj(vimg.reshape(-1)[vox]) * oracle.grid.gather_deriv(u, coords, i))
                     for i in range(3)])
    gd_g = ds.grad[0].reshape(3, -1)[:, vox].cpu().numpy()
    ed = float(np.linalg.norm(gd_g - gd_o) / np.linalg.norm(gd_o))
    say(f"  grad_128: grad_x rel err {ex:.2e}, sampled grad_d rel err {ed:.2e}")
    assert ex < TOL and ed < TOL
