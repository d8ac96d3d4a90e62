"""The 256^3, 16-coil, 8-state workload (mixed precision at scale): the GPU
operators of state 0 against stored FP64 oracle values
(tests/golden/mixed256_state0.json, written by
tests/golden/make_mixed256_reference.py from oracle/ and synth/ only), with
the coil-expanded 512^3 grids stored as FP32, FP16 and BF16; the error is
stated per result.

* forward A_0 x at 512 seeded samples, all 16 coils;
* adjoint A_0^H y at 4096 seeded voxels for seeded complex noise y.

Bars as in test_gpu_mixed.py: 1e-5 for FP32, 1e-3 for FP16 and BF16 grids
(one rounding per direction: the intermediates between the FFT passes stay
FP32).
"""
import json
import os
import sys

import numpy as np
import pytest

from synth import WORKLOADS, make_inputs

from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_mixed256_reference as ref_script  # noqa: E402  (seeded selections and data only)

BARS = {"fp32": 1e-5, "fp16": 1e-3, "bf16": 1e-3}


@pytest.fixture(scope="module")
def scale():
    path = os.path.join(HERE, "golden", "mixed256_state0.json")
    with open(path) as f:
        rec = json.load(f)
    w = WORKLOADS["mixed_256"]
    say("mixed_256 inputs")
    inp = make_inputs(w)
    M = inp["k"][0].shape[0]
    js, vs = ref_script.selections(M, int(np.prod(w.shape)))
    assert js.tolist() == rec["sample_indices"] and vs.tolist() == rec["voxels"]
    fwd = np.array(rec["forward"]) @ np.array([1.0, 1j])    # [512][C]
    adj = np.array(rec["adjoint"]) @ np.array([1.0, 1j])    # [4096]
    y = ref_script.adjoint_data(M, w.ncoils)
    return w, inp, js, vs, fwd, adj, y


@pytest.mark.parametrize("storage", ["fp32", "fp16", "bf16"])
def test_scale_state0(scale, storage):
    import torch
    import paper_2501_16713_amd as isg
    w, inp, js, vs, fwd, adj, y = scale
    say(f"mixed_256 state 0, {storage} grids")
    plan = isg.Plan(w.shape, ncoils=w.ncoils, nphases=1, storage=storage)
    S = to_dev(inp["S"])
    mo, tr = plan.motion(to_dev(inp["d"][0])), plan.traj(to_dev(inp["k"][0]))
    got = plan.sense_forward(to_dev(inp["x"]), [mo], S, [tr])
    got_f = got[torch.from_numpy(js).to(got.device)].cpu().numpy()
    ef = float(np.linalg.norm(got_f - fwd) / np.linalg.norm(fwd))
    xa = plan.sense_adjoint(to_dev(y), [mo], S, [tr]).reshape(-1)
    got_a = xa[torch.from_numpy(vs).to(xa.device)].cpu().numpy()
    ea = float(np.linalg.norm(got_a - adj) / np.linalg.norm(adj))
    say(f"  {storage}: A rel err {ef:.2e} (512 samples x 16 coils), A^H rel err {ea:.2e} (4096 voxels)")
    del plan, mo, tr, S, got, xa
    torch.cuda.empty_cache()
    assert np.isfinite(ef) and np.isfinite(ea)
    assert ef < BARS[storage] and ea < BARS[storage]
