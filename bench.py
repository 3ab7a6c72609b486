#!/usr/bin/env python3
"""Throughput of sigma = H c on one MI355X.

Default workload: the selected determinant space with 64 spatial orbitals,
10 alpha + 10 beta electrons, 2,000,000 determinants (HF, all singles and
doubles, random triples/quadruples), real FP64 integrals, one random
normalised vector.  A step is one sigma = H c over that space (the group
contraction kernel plus the per-determinant gather); the plan (grouping,
integral repacking, diagonal) is built once beforehand, as it is amortised
over the Davidson iterations that call sigma.

Prints one JSON line:  value = nonzero H_IJ c_J terms per second
((connected ordered pairs + diagonal) x roots / step time), with the group
kernel's achieved algorithmic HBM bandwidth against MI355X's 8 TB/s and the
CPU oracle timed on a bounded sample of rows.

Usage: python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--roots 1]
                       [--workload sci-n64|fci-n8|spinor-40kp] [--cpu-rows 800]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


WORKLOADS = {
    "sci-n64": 1,       # 64 orbitals, 10a10b, 2e6 dets (headline)
    "fci-n8": 0,        # FCI 8 orbitals 4a4b, 4900 dets
    "spinor-40kp": 2,   # 40 Kramers pairs, 20 electrons, 1e6 dets, complex
    "fci-n10": 4,       # FCI 10 orbitals 3a3b
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--roots", type=int, default=1)
    ap.add_argument("--workload", default="sci-n64", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-rows", type=int, default=800, help="rows of the CPU oracle sample (0: skip)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2501_18185_amd import mw, synth

    if not torch.cuda.is_available():
        log("no GPU visible")
        sys.exit(1)
    torch.cuda.set_device(0)
    k = WORKLOADS[args.workload]
    t0 = time.perf_counter()
    prob = synth.workload(k)
    log(f"[bench] workload {args.workload}: ndet={prob.ndet} generated in {time.perf_counter() - t0:.1f}s")
    t0 = time.perf_counter()
    plan = mw.Plan(prob, max_roots=args.roots)
    log(f"[bench] plan: groups={plan.info('groups')} memberships={plan.info('memberships')} "
        f"pairs={plan.info('pairs')} workspace={plan.info('workspace_bytes') / 2**30:.2f} GiB "
        f"in {time.perf_counter() - t0:.1f}s")
    R = args.roots
    c_np = synth.ci_vectors(prob.ndet, R, synth.rng_for(k, 0, synth.SEED_C), complex_=prob.is_complex)
    c = torch.from_numpy(c_np).cuda()
    sig = torch.empty_like(c)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        plan.sigma(c, out=sig)
    torch.cuda.synchronize()
    log("[bench] warmup done")

    mw.profile(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        plan.sigma(c, out=sig)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    mw.profile(False)
    ms_step = ev0.elapsed_time(ev1) / args.steps
    n_grp, ms_grp = mw.profile_read("group_sigma")
    n_gat, ms_gat = mw.profile_read("gather")
    log(f"[bench] {args.steps} steps: {ms_step:.3f} ms/step (wall {wall / args.steps * 1e3:.3f} ms); "
        f"group_sigma {ms_grp / max(n_grp, 1):.3f} ms x{n_grp}, gather {ms_gat / max(n_gat, 1):.3f} ms x{n_gat}")

    pairs = plan.info("pairs")
    ndet = prob.ndet
    sb = 16 if prob.is_complex else 8
    terms = (pairs + ndet) * R
    value = terms / (ms_step * 1e-3)
    # algorithmic bytes: per connected pair the partner coefficients (R
    # scalars) and one integral word; per determinant its string, c_I and
    # sigma_I
    launches_per_step = max(n_grp // args.steps, 1)
    bytes_grp_launch = pairs * (sb * R + sb) / launches_per_step
    avg_grp_s = ms_grp / max(n_grp, 1) * 1e-3
    achieved = bytes_grp_launch / avg_grp_s / 1e9 if n_grp else 0.0
    step_bytes = pairs * (sb * R + sb) + ndet * (16 + 2 * sb * R)

    out = {
        "metric": "nonzero H_IJ*c_J terms/sec (sigma = H c, FP64)",
        "value": value,
        "unit": "terms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128" if prob.is_complex else "f64",
        "data": "synthetic",
        "config": {
            "workload": prob.name,
            "ndet": ndet,
            "norb": prob.norb,
            "electrons": prob.nelec,
            "nroots": R,
            "connected_pairs": pairs,
            "sigma_builds_per_s": 1e3 / ms_step,
            "effective_hbm_frac_step": step_bytes / (ms_step * 1e-3) / (HBM_PEAK_GBS * 1e9),
            "group_sigma_ms": ms_grp / max(n_grp, 1),
            "gather_ms": ms_gat / max(n_gat, 1),
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_group_sigma",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "bytes_per_launch": bytes_grp_launch,
        },
    }

    if args.cpu_rows > 0:
        from oracle import sc
        rng = np.random.default_rng(2026)
        rows = np.sort(rng.choice(ndet, size=min(args.cpu_rows, ndet), replace=False))
        t0 = time.perf_counter()
        sc.sigma(prob, c_np, rows=rows)
        dt = time.perf_counter() - t0
        deg = sc.degree_rows(prob, rows)
        sample_terms = float((deg + 1).sum() * R)
        out["cpu_baseline"] = {
            "value": sample_terms / dt,
            "unit": "terms/s",
            "cores": sc.num_threads(),
            "kind": "oracle",
            "sample": f"{len(rows)} random rows of the same space and vector "
                      f"({int(sample_terms)} terms, {dt:.1f} s)",
        }
        log(f"[bench] cpu oracle: {len(rows)} rows in {dt:.1f}s on {sc.num_threads()} threads")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
