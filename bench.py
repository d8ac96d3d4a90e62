"""Benchmark of the nonrigid-SENSE normal operator on one MI355X.

A step is one application of the l2 normal operator of Eq. 11,
N x = sum_p A_p^H A_p x + lambda x, at 160^3, 12 coils, 6 respiratory states
with 80k..600k golden-angle radial samples each: every stage of the hot path
(upsampling FFTs, warp gather, coil-expanded FFTs, k-space gather and
spread, coil-reduced inverse FFTs, warp spread, adjoint upsampling FFTs and
the lambda term).  Inputs are seeded synthetic data already resident in HBM.
After the timed steps a 20-iteration CG solve (HIP graph per iteration) is
timed as well and reported under "cg".

Prints ONE JSON line (see the keys below).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic bytes of one launch of each operator stage (3D, C coils),
# element size es of the coil-expanded grids; B* are element counts
def stage_bytes(tag, n, G, C, es, M=0):
    n0, n1, n2 = n
    G0, G1, G2 = G
    N = n0 * n1 * n2
    NG = G0 * G1 * G2
    c8 = 8
    table = {
        "fft_coil_fwd_last": N * c8 * (1 + C) + n0 * n1 * G2 * C * es,
        "fft_coil_fwd_ax1": n0 * n1 * G2 * C * es + n0 * G1 * G2 * C * es,
        "fft_coil_fwd_ax0": n0 * G1 * G2 * C * es + NG * C * es,
        "fft_coil_adj_ax0": NG * C * es + n0 * G1 * G2 * C * es,
        "fft_coil_adj_ax1": n0 * G1 * G2 * C * es + n0 * n1 * G2 * C * es,
        "fft_coil_adj_last": n0 * n1 * G2 * C * es + N * c8 * (C + 1),
        "fft_up_ax2": 2 * N * c8,
        "fft_up_ax1": 2 * N * c8,
        "fft_up_ax0": N * c8 + G0 * n1 * n2 * c8,
        "fft_up_G1": G0 * n1 * n2 * c8 + G0 * G1 * n2 * c8,
        "fft_up_G2": G0 * G1 * n2 * c8 + NG * c8,
        "fft_uph_G2": NG * c8 + G0 * G1 * n2 * c8,
        "fft_uph_G1": G0 * G1 * n2 * c8 + G0 * n1 * n2 * c8,
        "fft_uph_ax0": G0 * n1 * n2 * c8 + N * c8,
        "fft_uph_ax1": 2 * N * c8,
        "fft_uph_ax2": 2 * N * c8,
    }
    return table.get(tag)


def kspace_bytes(stage, info, M, C, es):
    """algorithmic bytes of one state's k-space gather or spread: the
    touched cells of the coil grid, the 16-byte tap record per sample, and
    the visit-ordered coil values (8 C bytes per (sample, tile) visit)"""
    cells = info["touched_cells"] * C * es
    if stage == "kspread":  # touched cells written; tap records and visit values read
        return cells + info["visits"] * (16 + 8 * C)
    return M * 16 + cells + info["visits"] * 8 * C  # footprint read; visit values written


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batched_160")
    ap.add_argument("--storage", default="fp32", choices=["fp32", "bf16", "fp16"],
                    help="grid storage of the headline form")
    ap.add_argument("--forms", default="plain,tuned,bf16,fp16",
                    help="forms to time besides the headline: plain (one state per k-space launch, no graph), "
                         "tuned (autotuned batching / graph), bf16, fp16 (tuned, half-precision grids)")
    ap.add_argument("--no-tune", action="store_true", help="headline form without autotuning (options below)")
    ap.add_argument("--chunk", type=int, default=512, help="spread chunk with --no-tune")
    ap.add_argument("--batch", type=int, default=1, help="phase batch with --no-tune")
    ap.add_argument("--graph", type=int, default=0, help="graph replay (0/1) with --no-tune")
    ap.add_argument("--ktile", type=int, default=8, help="k-space spread tile extent along axis 1 with --no-tune")
    ap.add_argument("--kblock", type=int, default=3, help="k-space array row blocking (log2, 0 = plain) with --no-tune")
    ap.add_argument("--cg-iters", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-rows", action="store_true",
                    help="skip timing the reconstruction layer (wavelet, FISTA, registration, gridding recon, "
                         "the nonrigid-transform inversion)")
    ap.add_argument("--breakdown", action="store_true", help="print a per-stage timing table to stderr")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="also run one plain elementwise copy (negation) of this many MiB (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported "
              "(the path would shard over (state, coil) units of the states)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2501_16713_amd as isg
    from synth import WORKLOADS, make_inputs, rng, complex_noise, P_NOISE

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    w = WORKLOADS[args.workload]
    t0 = time.time()
    inp = make_inputs(w)
    log(f"inputs for {w.name} ready in {time.time() - t0:.1f}s")

    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(dev)
    lam = w.lam
    with torch.cuda.stream(stream):
        x = torch.from_numpy(inp["x"]).to(dev)
        S = torch.from_numpy(inp["S"]).to(dev)
        d_dev = [torch.from_numpy(d).to(dev) for d in inp["d"]]
        k_dev = [torch.from_numpy(k).to(dev) for k in inp["k"]]
    torch.cuda.synchronize()

    def make_plan(storage, options=None):
        with torch.cuda.stream(stream):
            t = time.time()
            plan = isg.Plan(w.shape, ncoils=w.ncoils, nphases=w.nphases, storage=storage)
            for name, v in (options or {}).items():
                plan.set_option(name, v)
            mots = [plan.motion(d) for d in d_dev]
            trs = [plan.traj(k) for k in k_dev]
            torch.cuda.synchronize()
        log(f"{storage} plan: preparation {time.time() - t:.1f}s")
        return plan, mots, trs

    def time_steps(plan, mots, trs, out, steps):
        """ms per normal-operator application over `steps` back-to-back calls"""
        with torch.cuda.stream(stream):
            torch.cuda.synchronize()
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            for _ in range(steps):
                plan.normal(x, lam, mots, S, trs, out=out)
            ev1.record(stream)
            torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / steps

    def run_form(storage, tune, options=None):
        plan, mots, trs = make_plan(storage, options)
        report = None
        with torch.cuda.stream(stream):
            out = torch.empty_like(x)
            if tune:
                t = time.time()
                report = plan.tune(x, lam, mots, S, trs, reps=3)
                log(f"{storage} tuned in {time.time() - t:.1f}s: {report['chosen']}")
            for _ in range(args.warmup):
                plan.normal(x, lam, mots, S, trs, out=out)
        ms = time_steps(plan, mots, trs, out, args.steps)
        opts = {k: plan.get_option(k) for k in ("kblock", "ktile_t1", "spread_chunk", "phase_batch", "graph")}
        log(f"{storage} {'tuned' if tune else 'plain'}: {ms:.3f} ms/apply, options {opts}")
        return plan, mots, trs, out, ms, opts, report

    # ---- headline form ------------------------------------------------------
    # the tile extent first: it decides how trajectories are binned
    fixed = None if not args.no_tune else {"kblock": args.kblock, "ktile_t1": args.ktile, "spread_chunk": args.chunk,
                                           "phase_batch": args.batch, "graph": args.graph}
    plan, mots, trs, out, ms_per_step, opts, tune_report = run_form(args.storage, not args.no_tune, fixed)
    value = 1000.0 / ms_per_step
    with torch.cuda.stream(stream):
        if args.calib_copy_mb > 0:
            # one plain streaming kernel of known size (reads and writes
            # calib_copy_mb MiB each) against which HBM counters are scaled
            src = torch.zeros(args.calib_copy_mb << 18, dtype=torch.float32, device=dev)
            dst = torch.empty_like(src)
            torch.cuda.synchronize()
            torch.neg(src, out=dst)
            torch.cuda.synchronize()
            del src, dst
        # per-stage pass (eager, every launch bracketed by events): the dominant stage
        plan.set_timing(True, "")
        plan.normal(x, lam, mots, S, trs, out=out)
        stages = plan.read_timing()
        plan.set_timing(False)
        dominant = max(stages, key=lambda t: stages[t][1])
        if args.breakdown:
            tot = sum(v[1] for v in stages.values())
            for t, (cnt, ms) in sorted(stages.items(), key=lambda kv: -kv[1][1]):
                log(f"  {t:22s} {cnt:4d} launches {ms:9.3f} ms  {100 * ms / tot:5.1f}%")
        # the dominant stage's launches over `steps` applications, bracketed
        # by events on the plan's stream (eager: a graph replay hides launches)
        plan.set_timing(True, dominant)
        for _ in range(args.steps):
            plan.normal(x, lam, mots, S, trs, out=out)
        dom = plan.read_timing().get(dominant, (0, 0.0))
        plan.set_timing(False)
        torch.cuda.synchronize()

        # CG (not part of the headline value)
        cg = None
        if args.cg_iters > 0:
            y = plan.sense_forward(x, mots, S, trs)
            rms = float(torch.sqrt(torch.mean(torch.abs(y) ** 2)).item())
            noise = torch.from_numpy(complex_noise(tuple(y.shape), rng(w.cfg, P_NOISE))).to(dev)
            y = y + 0.01 * rms * noise
            torch.cuda.synchronize()
            t0 = time.time()
            xs, hist = plan.cg_solve(y, mots, S, trs, lam, args.cg_iters)
            cg_s = time.time() - t0
            cg = {"iters": args.cg_iters, "seconds": round(cg_s, 4),
                  "ms_per_iter": round(1000 * cg_s / args.cg_iters, 3),
                  "resnorm_first_last": [hist[0], hist[-1]]}
            cg_y, cg_ref = y, xs
        ref_out = out.clone()
    torch.cuda.synchronize()

    es = 8 if args.storage == "fp32" else 4
    G = tuple(2 * n for n in w.shape)
    per_launch = stage_bytes(dominant, w.shape, G, w.ncoils, es)
    infos = [t.info() for t in trs]
    if dominant in ("fft_coil_fwd_ax0", "fft_coil_adj_ax0"):
        # these passes transform only the grid columns along axis 0 that hold
        # a run of cells some sample's taps reach, and of those move only the
        # touched runs on the k-space side and n0 cells on the image side, one
        # state per launch
        tot = sum((i["touched_cells"] + w.shape[0] * i["active_columns"]) * w.ncoils * es for i in infos)
        per_launch = tot // len(trs)
    if per_launch is None and dominant in ("kspread", "kgather"):
        # one state per launch unless batched: bytes of all states / launches
        per_launch = sum(kspace_bytes(dominant, i, k.shape[0], w.ncoils, es) for i, k in zip(infos, inp["k"]))
        per_launch = per_launch * args.steps // max(1, dom[0])
    roofline = None
    if per_launch and dom[0] > 0:
        avg_ms = dom[1] / dom[0]
        achieved = per_launch / (avg_ms * 1e-3) / 1e9
        copy_gbps = device_copy_gbps(stream)
        roofline = {"bound": "hbm", "kernel": dominant, "achieved": round(achieved, 1), "peak": 8000.0,
                    "unit": "GB/s", "frac": round(achieved / 8000.0, 4),
                    "traffic": measured_traffic(dominant, w.name, args.storage),
                    "bytes_per_launch": per_launch, "avg_launch_ms": round(avg_ms, 4),
                    "launches": dom[0],
                    # the same bandwidth against a plain device copy measured here
                    "copy_GBps": round(copy_gbps, 1), "frac_of_copy": round(achieved / copy_gbps, 4)}

    # ---- other forms, for the batched / mixed-precision speedups -------------
    if not args.no_tune:
        head = "tuned"
    else:
        head = "plain" if (args.kblock, args.ktile, args.chunk, args.batch, args.graph) == (0, 8, 512, 1, 0) \
            else "fixed"
    golden = golden_normal(w)
    forms = {f"{head}_{args.storage}": {"ms": round(ms_per_step, 4), "options": opts}}
    if golden is not None:
        forms[f"{head}_{args.storage}"]["rel_err_vs_fp64"] = golden_err(ref_out, golden)

    # ---- the reconstruction layer around the operator, at the same size ----
    rows = None
    if not args.no_rows:
        rows = recon_rows(plan, mots, trs, x, S, stream, log)
    del plan, mots, trs
    for f in [f.strip() for f in args.forms.split(",") if f.strip()]:
        storage = f if f in ("bf16", "fp16") else "fp32"
        tune = f != "plain"
        name = f"{'tuned' if tune else 'plain'}_{storage}"
        if name in forms:
            continue
        plain_opts = {"kblock": 0, "ktile_t1": 8, "spread_chunk": 512, "phase_batch": 1, "graph": 0}
        p2, m2, t2, o2, ms2, opts2, _ = run_form(storage, tune, None if tune else plain_opts)
        entry = {"ms": round(ms2, 4), "options": opts2}
        if golden is not None:
            entry["rel_err_vs_fp64"] = golden_err(o2, golden)
        if storage == args.storage:  # same storage, other options: only the summation order may differ
            diff = torch.linalg.vector_norm(o2 - ref_out) / torch.linalg.vector_norm(ref_out)
            entry["rel_diff_vs_headline"] = float(diff.item())
        if storage != args.storage:  # relative difference from the headline form's output
            diff = torch.linalg.vector_norm(o2 - ref_out) / torch.linalg.vector_norm(ref_out)
            entry["rel_diff_vs_" + args.storage] = float(diff.item())
            if cg is not None:  # the same CG solve with this form's grids
                with torch.cuda.stream(stream):
                    xs2, _ = p2.cg_solve(cg_y, m2, S, t2, lam, args.cg_iters)
                    cdiff = torch.linalg.vector_norm(xs2 - cg_ref) / torch.linalg.vector_norm(cg_ref)
                entry["cg_rel_diff_vs_" + args.storage] = float(cdiff.item())
        forms[name] = entry
        del p2, m2, t2, o2
        torch.cuda.synchronize()
    base = forms.get("plain_fp32", {}).get("ms")
    if base:
        for v in forms.values():
            v["speedup_vs_plain_fp32"] = round(base / v["ms"], 3)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(inp, w, log)

    total_samples = sum(k.shape[0] for k in inp["k"])
    line = {
        "metric": f"nonrigid-SENSE A^H A applies/s at {w.shape[0]}^3x{w.ncoils} coils",
        "value": round(value, 3),
        "unit": "applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64" if args.storage == "fp32" else f"c64+{args.storage}-grids",
        "data": "synthetic",
        "config": {"workload": w.name, "shape": list(w.shape), "coils": w.ncoils, "phases": w.nphases,
                   "samples_per_phase": [int(k.shape[0]) for k in inp["k"]], "lambda": lam,
                   "storage": args.storage, "options": opts},
        "per_state_applies_per_s": round(value * w.nphases, 3),
        "gridding_gpts_per_s": {
            # whole apply: both k-space directions / both warp directions per apply time
            "kspace_point_coil_interps": round(2 * total_samples * w.ncoils * value / 1e9, 4),
            "warp_voxels": round(2 * w.nphases * int(np.prod(w.shape)) * value / 1e9, 4),
            # per kernel, from its own time in one apply (eager pass with events)
            "per_kernel": per_kernel_gpts(stages, total_samples * w.ncoils, w.nphases * int(np.prod(w.shape))),
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "forms": forms,
        "tune": tune_report,
        "cg": cg,
        "rows": rows,
        "stages_ms": {k: round(v[1], 4) for k, v in sorted(stages.items(), key=lambda kv: -kv[1][1])},
    }
    print(json.dumps(line), flush=True)


def per_kernel_gpts(stages, point_coils, voxels):
    """Gpts/s of the gridding kernels from their stage times in one apply:
    k-space (sample, coil) interpolations for the gather (K5) and spread (K6,
    with its split-tile reduce), voxels over all states for the warp gather
    (K3) and spread (K4, with its halo sum)"""
    def ms(*tags):
        return sum(stages.get(t, (0, 0.0))[1] for t in tags)

    out = {}
    for name, pts, tags in (("K3_warp_gather", voxels, ("warp_gather",)),
                            ("K4_warp_spread", voxels, ("warp_spread", "warp_spread_sum")),
                            ("K5_kspace_gather", point_coils, ("kgather",)),
                            ("K6_kspace_spread", point_coils, ("kspread", "kspread_reduce"))):
        t = ms(*tags)
        if t > 0:
            out[name] = {"gpts_per_s": round(pts / (t * 1e-3) / 1e9, 3), "ms": round(t, 4)}
    return out


def golden_normal(w):
    """the stored FP64 oracle values of N x at seeded voxels for this
    workload (written by tests/golden/make_batched160_reference.py from the
    oracle alone), or None"""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", "batched160.json")
    if w.name != "batched_160" or not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("workload") != w.name or abs(rec.get("lambda", -1) - w.lam) > 0:
        return None
    return np.array(rec["voxels"]), np.array(rec["normal"]) @ np.array([1.0, 1j])


def golden_err(out, golden):
    import numpy as np
    vox, want = golden
    got = out.reshape(-1).cpu().numpy()[vox].astype(np.complex128)
    return float(f"{np.linalg.norm(got - want) / np.linalg.norm(want):.3e}")


def recon_rows(plan, mots, trs, x, S, stream, log):
    """Per-iteration times of the reconstruction layer at the benchmark's
    size (state 0's field, the largest state's samples), and the Appendix-1
    inversion on the 64 x 64 warp workload: the recovery error of the naive
    inverse (the negated field), of CG on the l2 form and of 400 iterations of
    wavelet-FISTA with lambda = 1e-6, against the ground-truth image."""
    import numpy as np
    import torch
    import paper_2501_16713_amd as isg
    from synth import WORKLOADS, make_inputs

    def timed(fn, reps, per):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return round(e0.elapsed_time(e1) / (reps * per), 4)

    out = {}
    with torch.cuda.stream(stream):
        mo, big = mots[0], trs[-1]
        q = plan.warp(x, mo)
        y = plan.sense_forward(x, mots, S, trs)
        yb = y[-big.M:].contiguous()
        buf = torch.empty_like(x)
        wv = plan.wavelet_forward(x, 3)
        lam_w, _ = plan.warp_power_iteration(mo, 4, x)
        out["warp_cg_iter_ms"] = timed(lambda: plan.warp_cg_solve(q, mo, 1e-3, 10), 2, 10)
        out["wavelet_fwd_ms"] = timed(lambda: plan.wavelet_forward(x, 3, out=buf), 5, 1)
        out["wavelet_inv_ms"] = timed(lambda: plan.wavelet_inverse(wv, 3, out=buf), 5, 1)
        out["warp_fista_iter_ms"] = timed(lambda: plan.warp_fista_solve(q, mo, 1e-6, 2.2 * lam_w, 3, 10), 2, 10)
        out["power_iter_ms"] = timed(lambda: plan.power_iteration(mots, S, trs, 3, x), 1, 3)
        # per FISTA iteration: 6 iterations less 3 (A^H y, formed once per solve, cancels)
        t6 = timed(lambda: plan.fista_solve(y, mots, S, trs, 1e-3, 2.0, 3, 6), 1, 1)
        t3 = timed(lambda: plan.fista_solve(y, mots, S, trs, 1e-3, 2.0, 3, 3), 1, 1)
        out["fista_iter_ms"] = round((t6 - t3) / 3, 4)
        mov = plan.warp(x, mots[1])
        out["register_step_ms"] = timed(lambda: plan.register(x, mov, 0.05, 0.02, 10), 2, 10)
        out["dcf_iter_ms"] = timed(lambda: plan.dcf(big, 10), 1, 10)
        wd = plan.dcf(big, 5)
        out["grid_recon_ms"] = timed(lambda: plan.grid_recon(big, yb, S, w=wd, out=buf), 5, 1)
        out["grid_recon_samples"] = big.M

        # Appendix 1 on the 64 x 64 warp workload
        w1 = WORKLOADS["warp2d_64"]
        inp = make_inputs(w1, with_traj=False)
        p_true = torch.from_numpy(inp["x"]).to(x.device)
        d = torch.from_numpy(inp["d"][0]).to(x.device)
        p2 = isg.Plan(w1.shape)
        m2, mneg = p2.motion(d), p2.motion(-d)
        q2 = p2.warp(p_true, m2)

        def err(a):
            return float(f"{(torch.linalg.vector_norm(a - p_true) / torch.linalg.vector_norm(p_true)).item():.4e}")

        l2, _ = p2.warp_power_iteration(m2, 30, q2)
        t0 = time.time()
        pc, _ = p2.warp_cg_solve(q2, m2, 1e-6, 100)
        t_cg = time.time() - t0
        t0 = time.time()
        pf, _ = p2.warp_fista_solve(q2, m2, 1e-6, 2.2 * l2, 3, 400)
        t_f = time.time() - t0
        out["inversion_warp2d_64"] = {
            "naive_rel_err": err(p2.warp(q2, mneg)),
            "cg_rel_err": err(pc), "cg_iters": 100, "cg_lambda": 1e-6, "cg_s": round(t_cg, 4),
            "fista_rel_err": err(pf), "fista_iters": 400, "fista_lambda": 1e-6, "fista_levels": 3,
            "fista_s": round(t_f, 4), "lipschitz": round(2.2 * l2, 4)}
        del p2, m2, mneg
    log(f"reconstruction layer: {out}")
    return out


def device_copy_gbps(stream, mib=1024, reps=5):
    """HBM bandwidth of a plain device-to-device tensor copy (reads and
    writes `mib` MiB each), GB/s, timed with events on `stream`"""
    import torch
    with torch.cuda.stream(stream):
        src = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for _ in range(reps):
            dst.copy_(src)
        t1.record(stream)
        t1.synchronize()
        ms = t0.elapsed_time(t1) / reps
    del src, dst
    return 2 * (mib << 20) / (ms * 1e-3) / 1e9


def measured_traffic(stage, workload, storage):
    """HBM bytes per launch of `stage` from the committed rocprofv3 counter
    summary of this workload, or None when there is none or the kernel
    sources have changed since the counters were taken."""
    from paper_2501_16713_amd.profile_summary import csrc_hash
    path = os.path.join(ROOT, "profiles", f"normal_op_{workload}_{storage}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("csrc_hash") != csrc_hash() or stage not in rec.get("stages", {}):
        return None
    return rec["stages"][stage]["traffic_bytes"]


def cpu_model():
    """the host CPU's model name (as lscpu prints it), from /proc/cpuinfo"""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(inp, w, log):
    """The FP64 oracle timed on this host on a bounded sample of the same
    workload, scaled to applies/s.  One apply is P x (T + T^H) plus
    P x C coil units (G_p then G_p^H).  The sample, all of state 0:
    * one coil unit, whole;
    * the upsampling FFTs of T, whole; the FFTs of T^H are the same
      transforms in reverse order and are taken to cost the same;
    * the warp gather on 1/32 of the voxels, scaled by 32;
    * the warp spread on the same 1/32 of the voxels, scaled by 32 after
      subtracting its fixed part (the per-tap sums over the whole grid),
      which is timed on its own with no points."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    import oracle

    # the oracle's FFTs (scipy.fft) run on the host's CPU share: the thread
    # count OMP_NUM_THREADS grants, else the CPUs this process may use;
    # everything else in the sampled steps runs on one thread
    cores = int(os.environ.get("OMP_NUM_THREADS") or 0) or len(os.sched_getaffinity(0)) or 1
    saved = oracle.warp.WORKERS, oracle.kspace.WORKERS
    oracle.warp.WORKERS = oracle.kspace.WORKERS = cores
    x = inp["x"].astype(np.complex128)
    d, k, S = inp["d"][0], inp["k"][0], inp["S"]
    shape = w.shape
    gshape = oracle.warp.oversampled_shape(shape)
    nvox = int(np.prod(shape))
    sub = np.arange(0, nvox, 32)
    with threadpool_limits(limits=1):
        t = time.time()
        u = oracle.warp.upsample(x)
        t_up = time.time() - t
        coords = oracle.warp.warp_coords(d)
        t = time.time()
        v = oracle.grid.gather(u, coords[sub])
        t_gather_sub = time.time() - t
        t = time.time()
        oracle.grid.spread(v[:0], coords[:0], gshape)
        t_spread_fixed = time.time() - t
        t = time.time()
        oracle.grid.spread(v, coords[sub], gshape)
        t_spread_sub = time.time() - t
        t = time.time()
        yk = oracle.kspace.nufft_forward(S[0].astype(np.complex128) * x, k)
        oracle.kspace.nufft_adjoint(yk, k, shape)
        t_coil = time.time() - t
        # the FFT-bearing steps again with scipy.fft on one thread
        oracle.warp.WORKERS = oracle.kspace.WORKERS = 1
        try:
            t = time.time()
            oracle.warp.upsample(x)
            t_up1 = time.time() - t
            t = time.time()
            yk = oracle.kspace.nufft_forward(S[0].astype(np.complex128) * x, k)
            oracle.kspace.nufft_adjoint(yk, k, shape)
            t_coil1 = time.time() - t
        finally:
            oracle.warp.WORKERS, oracle.kspace.WORKERS = saved
    t_spread = t_spread_fixed + 32 * max(0.0, t_spread_sub - t_spread_fixed)

    def per_apply_of(t_up_, t_coil_):
        return w.nphases * (2 * t_up_ + 32 * t_gather_sub + t_spread) + w.nphases * w.ncoils * t_coil_

    per_apply = per_apply_of(t_up, t_coil)
    per_apply1 = per_apply_of(t_up1, t_coil1)
    sampled = t_up + t_gather_sub + t_spread_fixed + t_spread_sub + t_coil
    log(f"oracle sample ({sampled:.1f}s): upsample {t_up:.1f}s, gather 1/32 {t_gather_sub:.1f}s, "
        f"spread fixed {t_spread_fixed:.1f}s, spread 1/32 {t_spread_sub:.1f}s, coil unit {t_coil:.1f}s "
        f"-> {per_apply:.0f}s per apply; one FFT thread: upsample {t_up1:.1f}s, coil unit {t_coil1:.1f}s "
        f"-> {per_apply1:.0f}s per apply")
    return {"value": float(f"{1.0 / per_apply:.4g}"), "unit": "applies/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "value_one_fft_thread": float(f"{1.0 / per_apply1:.4g}"),
            "sample": (f"FP64 oracle, state 0, {sampled:.0f}s timed: one coil's G then G^H ({t_coil:.1f}s), "
                       f"the upsampling FFTs ({t_up:.1f}s, also taken for the FFTs of T^H), the warp gather "
                       f"on 1/32 of the voxels ({t_gather_sub:.1f}s) and the warp spread on the same voxels "
                       f"({t_spread_sub:.1f}s, of which a fixed {t_spread_fixed:.1f}s measured with no points); "
                       f"scaled to {w.nphases} states x {w.ncoils} coils -> {per_apply:.0f}s per apply; "
                       f"FFTs on {cores} threads, the rest on one; value_one_fft_thread "
                       f"repeats the upsampling and coil-unit steps with one FFT thread")}

if __name__ == "__main__":
    main()
