"""Benchmark: batched BP+DC shots/s on one MI355X, against the plain GPU decoder
and the CPU oracle.

Workload: [[144,12,12]] bivariate bicycle code, code-capacity bit flips with
p = 0.05, 1e6 seeded synthetic shots per step (syndromes resident in HBM before
the timed region), scaled min-sum (alpha = 0.625), at most 100 iterations
before and 100 after degeneracy cutting, channel prior in the second pass.
A step decodes the whole batch in one persistent launch of the fused lane
kernel.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "shots/s BP+DC, BB[[144,12,12]] p=0.05: batched vs plain at equal LER"
PEAK_LANE_OPS = 256 * 64 * 2.4e9   # non-packed 32-bit VALU lane-ops/s (256 CUs, 4x16 lanes, 2.4 GHz)
OPS_PER_EDGE_ITER = 8               # algorithmic VALU ops per Tanner edge per iteration
OPS_PER_DC_ENTRY = 2                # per nonzero of D on shots that run DC


def wilson(k: int, n: int, z: float = 1.96):
    if n == 0:
        return (0.0, 0.0)
    ph = k / n
    den = 1 + z * z / n
    c = (ph + z * z / (2 * n)) / den
    h = z * math.sqrt(ph * (1 - ph) / n + z * z / (4 * n * n)) / den
    return (c - h, c + h)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--shots", type=int, default=1_000_000)
    ap.add_argument("--p", type=float, default=0.05)
    ap.add_argument("--plain-steps", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run one device-to-device copy of this many MiB (a known-size kernel that "
                         "calibrates hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only; --gpus {args.gpus} is not supported "
              "(shots are independent: run one process per GPU on disjoint shot ranges)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2510_08695_amd as P
    import synth

    torch.cuda.set_device(0)
    p, B = args.p, args.shots
    code = synth.bb_code("bb144", p=p)
    shots = synth.make_shots(code, B, 2000 + round(100 * p))
    prm = P.Params(max_iter=(100, 100), alpha=0.625, second_pass_prior=P.PRIOR_CHANNEL,
                   stop_on_converge=True, llr_sat=64.0, tie_eps=1e-3, tie_break=P.TIE_HASH, seed=1)
    c = P.Code.from_problem(code)
    plan = P.Plan([c], prm, kernel=P.KERNEL_LANE)
    syn = torch.from_numpy(synth.pack_bits(shots.syndromes).view(np.int64)).cuda()
    out = {"corr": torch.empty((B, 3), dtype=torch.int64, device="cuda"),
           "flags": torch.empty(B, dtype=torch.uint8, device="cuda")}
    stream = torch.cuda.current_stream()

    # untimed: counts for the roofline (deterministic, identical in every step)
    ref = plan.decode(syn, want_iters=True)
    torch.cuda.synchronize()
    iters = ref["iters"].cpu().numpy().astype(np.int64)
    flags = ref["flags"].cpu().numpy()
    ehat = synth.unpack_bits(ref["corr"].cpu().numpy().view(np.uint64), code.n)
    n_dc = int(((flags & 2) != 0).sum())
    ops_per_step = OPS_PER_EDGE_ITER * code.H.nnz * int(iters.sum()) + OPS_PER_DC_ENTRY * code.D.nnz * n_dc

    for _ in range(args.warmup):
        plan.decode(syn, out=out)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    for s in range(args.steps):
        ev[s][0].record(stream)
        plan.decode(syn, out=out)
        ev[s][1].record(stream)
    t1.record(stream)
    torch.cuda.synchronize()
    total_ms = t0.elapsed_time(t1)
    launch_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    ms_per_step = total_ms / args.steps
    value = B / (ms_per_step / 1e3)
    assert torch.equal(out["corr"], ref["corr"]) and torch.equal(out["flags"], ref["flags"])

    conv = (flags & 1) != 0
    fail = ~conv | synth.residual_is_logical(shots.errors ^ ehat, code.O)
    k_fail = int(fail.sum())
    lo, hi = wilson(k_fail, B)
    result = {
        "metric": METRIC, "value": value, "unit": "shots/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"BB[[144,12,12]] code capacity p={p}, {B} shots per step, min-sum "
                               "alpha=0.625, T=100+100, BP+DC, channel prior second pass",
                   "code": "bb144", "shots_per_step": B, "p": p, "kernel": "lane (fused persistent)"},
        "ler": k_fail / B, "ler_ci95": [lo, hi], "dc_rate": n_dc / B,
        "mean_iters": float(iters.sum()) / B,
    }
    achieved = ops_per_step / (launch_ms / 1e3)
    result["roofline"] = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                          "unit": "Tlane-op/s", "frac": achieved / PEAK_LANE_OPS, "traffic": None,
                          "launch_ms": launch_ms, "ops_per_launch": ops_per_step}

    if args.copy_probe_mib:
        src = torch.empty(args.copy_probe_mib << 18, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        result["copy_probe_bytes"] = {"read": src.numel() * 4, "write": dst.numel() * 4}
        del src, dst

    if not args.no_plain:
        pplan = P.Plan([c], prm, kernel=P.KERNEL_PLAIN)
        pout = {"corr": torch.empty((B, 3), dtype=torch.int64, device="cuda"),
                "flags": torch.empty(B, dtype=torch.uint8, device="cuda")}
        pplan.decode(syn, out=pout)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(args.plain_steps):
            pplan.decode(syn, out=pout)
        b.record(stream)
        torch.cuda.synchronize()
        plain_ms = a.elapsed_time(b) / args.plain_steps
        same = bool(torch.equal(pout["corr"], ref["corr"]) and torch.equal(pout["flags"], ref["flags"]))
        result["plain"] = {"shots_per_s": B / (plain_ms / 1e3), "ms_per_step": plain_ms,
                           "speedup_batched_vs_plain": value / (B / (plain_ms / 1e3)),
                           "identical_outputs": same}
        del pplan

    if not args.no_cpu:
        import oracle
        sys.path.insert(0, os.path.join(ROOT, "tests"))
        from gpu_helpers import oracle_params
        cores = len(os.sched_getaffinity(0))
        op = oracle_params(prm, "channel")
        done, el, fails = 0, 0.0, 0
        chunk = 20000
        while el < args.cpu_seconds and done < B:
            hi_ = min(B, done + chunk)
            t = time.perf_counter()
            o = oracle.decode(code, shots.syndromes[done:hi_], op, precision="f64", shot_offset=done,
                              want_post=False, threads=cores)
            el += time.perf_counter() - t
            f = ((o["flags"] & 1) == 0) | synth.residual_is_logical(shots.errors[done:hi_] ^ o["ehat"], code.O)
            fails += int(f.sum())
            done = hi_
        result["cpu_baseline"] = {"value": done / el, "unit": "shots/s", "cores": cores, "kind": "oracle",
                                  "sample": f"first {done} shots of the same batch, float64 oracle, "
                                            f"{cores} OpenMP threads",
                                  "ler_on_sample": fails / done,
                                  "gpu_ler_on_sample": float(fail[:done].mean())}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
