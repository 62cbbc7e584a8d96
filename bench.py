#!/usr/bin/env python
"""Benchmark of the all-pairs dislocation-segment force path on one MI355X.

A step is one pass of the path over the single-volume workload: segment
preparation, the all-pairs non-singular stress at every Gauss point, the
Peach-Koehler contraction, the quadrature to nodal forces (dd_nodal_forces),
then the glide-constrained mobility and forward-Euler update (dd_glide_step).
Workload: 16,384 straight segments (512 regular 32-gon glide loops on random
{111} planes, radii U[100, 500] b, centres in a 10,000 b cube, seed 1), 2 Gauss
points per segment, FP64, inputs resident in HBM.  value = segment pairs
(source i != target j, all Gauss points of j) per second over the timed steps.

Printed as one JSON line, with
* roofline: the all-pairs kernel's algorithmic FLOPs per launch (a fixed count
  per Gauss-point evaluation of the closed form, see FLOP_* below) over its
  average launch time from HIP events on the launch stream, against the FP64
  vector peak; traffic from the committed rocprofv3 counter summary when it
  was taken on the current kernel source;
* cpu_baseline: the FP64 C oracle, single-threaded, on a bounded sample of the
  same workload (the first --cpu-targets target segments against all sources);
* extras: the mixed FP32/FP64 path and 4 Gauss points on the same volume, and
  512 batched bursts (200 glide steps each) in one graph launch.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "segment-pair force evals/s (FP64 vs mixed) + surrogate speedup at fixed error"
UNIT = "segment-pair evals/s"

# Algorithmic FLOPs per (target Gauss point, source segment) evaluation,
# counted on the closed form as written in csrc/dd_pair.h (add, sub, mul = 1,
# fma = 2, sqrt / rsqrt / reciprocal = 1; selects and compares = 0).
FLOP_F64_EVAL = 169          # FP64 path
FLOP_MIX_PREP_F64 = 14       # mixed: FP64 offset, axial, perpendicular parts (every pair)
FLOP_MIX_BAND_F32 = 13       # mixed: |rho|^2 and distance-to-midpoint band test (every pair)
FLOP_MIX_QUAD_F32 = 145      # mixed: FP32 2-point source quadrature (well-separated pairs)
FLOP_MIX_CLASS_F32 = 3       # mixed: minimum-distance test (other pairs)
FLOP_MIX_FAR_F32 = 179       # mixed: FP32 cancellation-free closed form
FLOP_MIX_NEAR_F64 = 169      # mixed: FP64 closed form (near pairs)
PEAK_F64 = 78.6e12
PEAK_F32 = 157.3e12
HBM_PEAK = 8.0e12

TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_pair64_volume16384_q2_traffic.json")
KERNEL_SOURCES = ["paper_2005_02498_amd/csrc/dd_pair64.hip", "paper_2005_02498_amd/csrc/dd_pair64.h"]


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_bytes():
    """HBM bytes per launch of k_pair64 from the committed counter summary,
    or None when the kernel source changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except OSError:
        return None
    if t.get("kernel_source_sha") != kernel_source_sha():
        return None
    return t.get("bytes_per_launch")


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-targets", type=int, default=4096,
                    help="target segments in the CPU oracle sample (0: skip)")
    ap.add_argument("--no-extras", action="store_true", help="skip mixed / Q=4 / burst extras")
    ap.add_argument("--burst-instances", type=int, default=512)
    ap.add_argument("--burst-steps", type=int, default=200)
    ap.add_argument("--only", choices=["fp64", "mixed", "burst", "copy"], default=None,
                    help="profiling aid: run only one part (no JSON contract)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the force path shards by loops across GPUs by design, but no multi-GPU code "
              "path exists)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2005_02498_amd as dd
    from paper_2005_02498_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    mat = {"mu": W.MU, "nu": W.NU, "a": W.CORE_A, "B": W.DRAG_B}

    if args.only == "copy":
        # plain copy of a known size, for scaling HBM counters
        n = 1 << 28
        a = torch.ones(n, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n, "launches": 5}))
        return

    inst = W.config1()
    N = inst.n_segs
    pairs = N * (N - 1)
    x0 = torch.tensor(inst.x, device=dev)
    sn = torch.tensor(inst.seg_nodes, device=dev)
    bg = torch.tensor(inst.burgers, device=dev)
    nr = torch.tensor(inst.normal, device=dev)
    F = torch.empty((3, inst.n_nodes), dtype=torch.float64, device=dev)
    V = torch.empty_like(F)
    dd.dd_set_validation(False)

    def run(prec, Q, steps, warmup):
        x = x0.clone()

        def step():
            dd.dd_nodal_forces(x, sn, bg, nr, inst.sigma_app, mat, Q, prec, 20.0, force_out=F)
            dd.dd_glide_step(x, F, sn, nr, None, mat, W.DT, vel_out=V)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        dd.dd_timing_read(reset=True)
        dd.dd_timing_enable(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        dd.dd_timing_enable(False)
        kms, launches, near, quad = dd.dd_timing_read(reset=True)
        assert launches == steps, (launches, steps)
        return (t1 - t0) / steps, kms / 1e3 / launches, (near / launches, quad / launches)

    def roof(prec, Q, kernel_s, bands):
        if prec == dd.DD_FP64:
            f64 = FLOP_F64_EVAL * pairs * Q
            f32 = 0.0
        else:
            near, quad = bands
            allp = N * N * Q                 # including the (skipped) self pairs
            other = allp - quad              # pairs that take the minimum-distance test
            closed = pairs * Q - quad - near
            f64 = FLOP_MIX_PREP_F64 * allp + FLOP_MIX_NEAR_F64 * near
            f32 = (FLOP_MIX_BAND_F32 * allp + FLOP_MIX_QUAD_F32 * quad
                   + FLOP_MIX_CLASS_F32 * other + FLOP_MIX_FAR_F32 * closed)
        flops = f64 + f32
        t_roof = f64 / PEAK_F64 + f32 / PEAK_F32
        peak = flops / t_roof
        ach = flops / kernel_s
        return {"bound": "alu", "achieved": ach / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                "frac": ach / peak, "flop_per_launch": flops, "fp64_flop": f64, "fp32_flop": f32,
                "kernel_ms": kernel_s * 1e3}

    if args.only in ("fp64", "mixed"):
        prec = dd.DD_FP64 if args.only == "fp64" else dd.DD_MIXED
        s, k, _ = run(prec, 2, args.steps, args.warmup)
        print(json.dumps({"part": args.only, "ms_per_step": s * 1e3, "kernel_ms": k * 1e3}))
        return

    out = {}
    if args.only != "burst":
        step_s, ker_s, _ = run(dd.DD_FP64, 2, args.steps, args.warmup)
        r = roof(dd.DD_FP64, 2, ker_s, None)
        tb = traffic_bytes()
        rl = {"bound": "alu", "achieved": r["achieved"], "peak": r["peak"], "unit": "TFLOP/s",
              "frac": r["frac"], "traffic": tb, "kernel": "k_pair64",
              "kernel_ms": r["kernel_ms"], "flop_per_launch": r["flop_per_launch"],
              "flop_per_eval": FLOP_F64_EVAL}
        out = {
            "metric": METRIC, "value": pairs / step_s, "unit": UNIT, "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": step_s * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": "single volume: 16,384 segments (512 glide loops x 32) in a "
                                   "10,000 b cube, 2 Gauss points, FP64; nodal forces + glide step",
                       "segments": N, "gauss_points": 2, "precision": "fp64",
                       "pairs_per_step": pairs, "gauss_evals_per_step": 2 * pairs},
            "gauss_evals_per_s": 2 * pairs / step_s,
            "kernel_pairs_per_s": pairs / ker_s,
            "roofline": rl,
        }

    if not args.no_extras and args.only is None:
        extras = {}
        for name, prec, Q in (("mixed_q2", dd.DD_MIXED, 2), ("fp64_q4", dd.DD_FP64, 4),
                              ("mixed_q4", dd.DD_MIXED, 4)):
            s, k, bands = run(prec, Q, max(5, args.steps // 2), 2)
            r = roof(prec, Q, k, bands)
            extras[name] = {"pairs_per_s": pairs / s, "gauss_evals_per_s": Q * pairs / s,
                            "ms_per_step": s * 1e3, "kernel_ms": k * 1e3,
                            "near_fp64_evals_per_launch": bands[0],
                            "quad_fp32_evals_per_launch": bands[1],
                            "roofline": {kk: r[kk] for kk in ("bound", "achieved", "peak", "unit", "frac")}}
        out["extras"] = extras

    if (not args.no_extras and args.only is None) or args.only == "burst":
        insts = W.config2(args.burst_instances)
        bt = W.pack(insts)
        Ns = np.diff(bt.seg_off)
        bpairs = int(np.sum(Ns * (Ns - 1))) * args.burst_steps
        d = dict(x=torch.tensor(bt.x, device=dev), sn=torch.tensor(bt.seg_nodes, device=dev),
                 b=torch.tensor(bt.burgers, device=dev), n=torch.tensor(bt.normal, device=dev),
                 p=torch.tensor(bt.pinned, device=dev), s=torch.tensor(bt.sigma_app, device=dev),
                 v=torch.tensor(bt.volume, device=dev))
        # one short warm-up launch (graph capture path, kernels loaded)
        dd.dd_burst_batch(bt.node_off, bt.seg_off, d["x"].clone(), d["sn"], d["b"], d["n"], d["p"],
                          d["s"], d["v"], mat, 2, dd.DD_MIXED, 20.0, 1, W.DT)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rates, _ = dd.dd_burst_batch(bt.node_off, bt.seg_off, d["x"], d["sn"], d["b"], d["n"],
                                     d["p"], d["s"], d["v"], mat, 2, dd.DD_MIXED, 20.0,
                                     args.burst_steps, W.DT)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        bursts = {"workload": f"{bt.n_inst} independent bursts, 256-4096 segments each, "
                              f"{args.burst_steps} glide steps, 2 Gauss points, mixed, one graph launch",
                  "instances": bt.n_inst, "segments_total": int(bt.seg_off[-1]),
                  "steps": args.burst_steps, "seconds": t1 - t0, "pairs": bpairs,
                  "pairs_per_s": bpairs / (t1 - t0),
                  "finite": bool(torch.isfinite(rates).all().item())}
        if args.only == "burst":
            print(json.dumps(bursts))
            return
        out["bursts"] = bursts

    if args.cpu_targets > 0:
        import oracle as O
        nt = min(args.cpu_targets, N)
        t0 = time.perf_counter()
        O.nodal_forces_sampled(inst.x, inst.seg_nodes, inst.burgers, inst.sigma_app,
                               W.MU, W.NU, W.CORE_A, 2, 0, nt)
        t1 = time.perf_counter()
        out["cpu_baseline"] = {
            "value": nt * (N - 1) / (t1 - t0), "unit": UNIT, "cores": 1, "kind": "oracle",
            "sample": f"first {nt} of {N} target segments against all {N} sources, 2 Gauss "
                      f"points, FP64 C oracle single-threaded ({t1 - t0:.1f} s); host has "
                      f"{os.cpu_count()} logical CPUs",
            "seconds": t1 - t0}

    print(json.dumps(out))


if __name__ == "__main__":
    main()
