"""The 30-iteration CG solve of the mixed-precision workload at 128^3 (16
coils, 8 respiratory states, 187k radial samples each; the 256^3 workload's
sampling density, at a size whose FP64 solve finishes in hours) against
stored FP64 oracle solves (tests/golden/mixed128_cg*.json, written by
tests/golden/make_mixed128_cg_reference.py from oracle/ and synth/ only), for
FP32, FP16 and BF16 grid storage with the options bench.py times:

* b = sum_p A_p^H y_p at 4096 seeded voxels (Fig. 3b): the operator bars,
  1e-5 for FP32 and 1e-3 for the half-precision grids;
* the CG iterate x_30 at the same voxels and the residual norms
  ||r_0|| .. ||r_30|| (l2 form of Eq. 11, x_0 = 0), at two lambdas:
  - lambda = 1e-3 (the workload's) on noise data is a stress case: the FP64
    solve itself has not converged after 30 iterations (||r_30|| / ||r_0|| =
    1.38, after a jump to 6.8 at the first step); measured x_30 errors
    0.10 (FP32), 0.15 (FP16), 0.19 (BF16).  The test states them and bounds
    them at about three times that, and the final residual ratio within a
    factor 2 of FP64's;
  - lambda = 0.5 is no better conditioned at this data scale: the FP64 solve
    ends at ||r_30|| / ||r_0|| = 0.93 (after 6.8 at the first step); measured
    x_30 errors 0.078 (FP32), 0.11 (FP16), 0.14 (BF16), bounded at about three
    times that.
  Both solves are followed step by step at first: the residual norms of the
  first five iterations agree with FP64's to 1e-5 for FP32 (measured 1.3e-7;
  FP16 4.5e-5 and BF16 2e-4, bounded at 5e-4 and 2e-3),
  so the later drift of the iterate comes from the solve itself, which does
  not converge and carries the operator's FP32 difference from FP64
  (5e-7 per application) into the slow components of x.  For FP32 the test
  also solves again with another k-space tile extent, which changes only
  the order of the spread's sums: the two FP32 iterates agree to 1e-3
  (measured 1e-5 and 4e-5).
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
GOLDEN = os.path.join(HERE, "golden", "mixed128_cg.json")
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_mixed128_cg_reference as ref_script  # noqa: E402  (seeded selections and data only)

TUNED = {"kblock": 2, "ktile_t1": 4, "spread_chunk": 1024, "phase_batch": 8, "graph": 1}
ADJ_BAR = {"fp32": 1e-5, "fp16": 1e-3, "bf16": 1e-3}
# CG iterate x_30 bars per lambda and storage (relative L2 over the sampled
# voxels); every case also keeps the final residual ratio within a factor 2
# of FP64's
X_BAR = {1e-3: {"fp32": 0.3, "fp16": 0.45, "bf16": 0.6},
         0.5: {"fp32": 0.25, "fp16": 0.35, "bf16": 0.45}}
# residual norms of the first five iterations against FP64's (relative)
EARLY_BAR = {"fp32": 1e-5, "fp16": 5e-4, "bf16": 2e-3}
GOLDENS = {1e-3: GOLDEN, 0.5: GOLDEN.replace(".json", "_lam0.5.json")}


def _load(lam):
    path = GOLDENS[lam]
    if not os.path.exists(path):
        pytest.skip(f"{os.path.basename(path)} has not been written")
    with open(path) as f:
        rec = json.load(f)
    assert abs(rec["lambda"] - lam) < 1e-12
    return rec


@pytest.fixture(scope="module")
def inputs():
    w = WORKLOADS["mixed_128"]
    say("mixed_128 inputs")
    inp = make_inputs(w)
    vs = ref_script.selections(int(np.prod(w.shape)))
    Mtot = sum(k.shape[0] for k in inp["k"])
    return w, inp, vs, ref_script.data(Mtot, w.ncoils)


def _golden(rec, vs):
    assert vs.tolist() == rec["voxels"]
    cplx = np.array([1.0, 1j])
    return np.array(rec["b"]) @ cplx, np.array(rec["x_final"]) @ cplx, np.array(rec["resnorm"])


def _err(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("lam", [1e-3, 0.5])
@pytest.mark.parametrize("storage", ["fp32", "fp16", "bf16"])
def test_mixed128_cg_against_fp64(inputs, storage, lam):
    import torch
    import paper_2501_16713_amd as isg
    rec = _load(lam)
    w, inp, vs, y = inputs
    b_ref, x_ref, hist_ref = _golden(rec, vs)
    say(f"mixed_128 CG, lambda {lam:g}, {storage} grids")
    plan = isg.Plan(w.shape, ncoils=w.ncoils, nphases=w.nphases, storage=storage)
    for k, v in TUNED.items():
        plan.set_option(k, v)
    S = to_dev(inp["S"])
    mots = [plan.motion(to_dev(d)) for d in inp["d"]]
    trs = [plan.traj(to_dev(k)) for k in inp["k"]]
    yd = to_dev(y)
    idx = torch.from_numpy(vs).to(yd.device)
    b = plan.sense_adjoint(yd, mots, S, trs).reshape(-1)[idx].cpu().numpy()
    x, hist = plan.cg_solve(yd, mots, S, trs, lam, w.cg_iters)
    xs = x.reshape(-1)[idx].cpu().numpy()
    torch.cuda.synchronize()
    hist = np.array(hist)
    eb, ex = _err(b, b_ref), _err(xs, x_ref)
    eh = float(np.max(np.abs(hist - hist_ref) / hist_ref))
    e5 = float(np.max(np.abs(hist[:6] - hist_ref[:6]) / hist_ref[:6]))
    say(f"  {storage}: A^H y {eb:.2e}, x_30 {ex:.2e}, residual history {eh:.2e}, first five {e5:.2e} "
        f"(||r_30||/||r_0|| {hist[-1] / hist[0]:.3e} vs FP64 {hist_ref[-1] / hist_ref[0]:.3e})")
    assert eb < ADJ_BAR[storage]
    assert e5 < EARLY_BAR[storage]
    assert np.all(np.isfinite(hist)) and np.isfinite(ex)
    assert ex < X_BAR[lam][storage]
    ratio = (hist[-1] / hist[0]) / (hist_ref[-1] / hist_ref[0])
    assert 0.5 < ratio < 2.0
    if storage == "fp32":
        # the same solve with the k-space spread's sums in another order
        # (8 x 8 x 8 tiles instead of 8 x 4 x 8; trajectories binned anew)
        plan.set_option("ktile_t1", 8)
        trs2 = [plan.traj(to_dev(k)) for k in inp["k"]]
        x2, _ = plan.cg_solve(yd, mots, S, trs2, lam, w.cg_iters)
        xs2 = x2.reshape(-1)[idx].cpu().numpy()
        d_order = _err(xs2, xs)
        say(f"  fp32 with another spread summation order: x_30 {d_order:.2e} from the first FP32 solve")
        assert d_order < 1e-3
