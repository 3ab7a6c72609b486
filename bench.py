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

Further legs reported in the same line (skip with --legs none):
  batched   16 uneven spin-free problems (16-48 orbitals, 6-12 electrons per
            spin, 1e4-5e5 determinants) with 4 roots each: one graph-replayed
            persistent launch vs 16 plain 4-root calls vs 64 plain 1-root
            calls;
  batched_small
            32 small spin-free problems (16-20 orbitals, 5-6 electrons per
            spin, 8e3-2e4 determinants), 4 roots: the graph vs 32 plain
            4-root calls;
  spinor    complex sigma over 40 Kramers pairs, 20 electrons, 1e6
            determinants;
  rdm       forward sigma + energy and backward density matrices (gamma,
            Gamma) on the headline space;
  davidson  time per Davidson iteration on the headline space;
  ivi       time per step of the iterative vector interaction solver
            (lowest root) on the headline space;
  pt2       Epstein-Nesbet second-order energy of the lowest root of a
            20,000-determinant n=64 10a10b space over its external space
            (exact and screened), and the iCIPT2 selection of the next
            determinants from it;
  csf       sigma in the CSF basis (spin-adapted, S = 0) of the
            configuration-complete singles-and-doubles space of n=64
            10a10b and of an open-shell-rich space (n=32 8a8b, 10 and 12
            open shells), 1 and 4 roots, against the determinant sigma of
            the same space.

Usage: python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--roots 1]
                       [--workload sci-n64|fci-n8|spinor-40kp|fci-n10]
                       [--cpu-rows 30000] [--legs batched,batched_small,spinor,rdm,davidson,ivi,pt2,csf|none]
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def measured_traffic(workload, R):
    """HBM bytes per launch of each sigma kernel from the committed rocprofv3
    counters (profiles/traffic.json: FETCH_SIZE and WRITE_SIZE per dispatch,
    scaled by what the same counters read for a plain copy and fill of known
    size), or {} when the kernel sources changed since they were taken or
    the workload differs."""
    import hashlib
    try:
        with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
            t = json.load(f)
        h = hashlib.sha256()
        for src in t["sources"]:
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
        if h.hexdigest()[:16] != t["source_sha256_16"]:
            return {}
        e = t["workloads"].get(f"{workload}/R{R}", {})
        return {k: v["fetch_kib_per_dispatch"] * 1024 * t["fetch_factor"] +
                v["write_kib_per_dispatch"] * 1024 * t["write_factor"] for k, v in e.items()}
    except (OSError, KeyError, ValueError):
        return {}


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
    ap.add_argument("--cpu-rows", type=int, default=30000, help="rows of the CPU oracle sample (0: skip)")
    ap.add_argument("--legs", default="batched,batched_small,spinor,rdm,davidson,ivi,pt2,csf")
    ap.add_argument("--plan", default="device", choices=["device", "host"],
                    help="where the plan's grouping is built (the arrays are the same)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain 1 GiB device copy (reference kernel for HBM counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: libmw has no multi-GPU path "
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
    # the grouping is built on the device by default (the same arrays as the host build)
    plan = mw.Plan(prob, max_roots=args.roots, build=args.plan)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    log(f"[bench] plan: groups={plan.info('groups')} memberships={plan.info('memberships')} "
        f"pairs={plan.info('pairs')} workspace={plan.info('workspace_bytes') / 2**30:.2f} GiB "
        f"built on the {args.plan} in {plan_s:.2f}s")
    R = args.roots
    c_np = synth.ci_vectors(prob.ndet, R, synth.rng_for(k, 0, synth.SEED_C), complex_=prob.is_complex)
    c = torch.from_numpy(c_np).cuda()
    sig = torch.empty_like(c)
    stream = torch.cuda.current_stream()

    if args.copy_calib:
        src = torch.empty(2**27, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        plan.sigma(c, out=sig)
    torch.cuda.synchronize()
    log("[bench] warmup done")

    # Python's cyclic garbage collector is run before and held off during
    # the timed steps: a full collection (tens of ms) landing on the first
    # step would leave the GPU idle (the same is done in _time)
    gc.collect()
    gc.disable()
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
    gc.enable()
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
    kern = kernel_rooflines(plan, R, sb, args.steps, n_grp, ms_grp, n_gat, ms_gat,
                            traffic=measured_traffic(args.workload, R))
    step_bytes = pairs * (sb * R + sb) + ndet * (16 + 2 * sb * R)
    dbl = kern["k_group_double"]
    # the per-term model (every ordered pair reads its partner's R
    # coefficients and one integral word) unless the Hermitian half-work
    # beats it (a fraction above 1), then the evaluated-pair model
    ordered = dbl["frac"] <= 1.0
    roof_bytes = dbl["bytes_per_launch"] if ordered else dbl["bytes_per_launch_evaluated_pairs"]
    roof_ach = roof_bytes / (dbl["avg_ms"] * 1e-3) / 1e9 if dbl["avg_ms"] > 0 else 0.0

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
            "single_pairs": plan.info("single_pairs"),
            "double_pairs": plan.info("double_pairs"),
            "double_pairs_large_groups": plan.info("double_pairs_large_groups"),
            "sigma_builds_per_s": 1e3 / ms_step,
            "plan_build_s": plan_s,
            "plan_built_on": args.plan,
            "effective_hbm_frac_step": step_bytes / (ms_step * 1e-3) / (HBM_PEAK_GBS * 1e9),
            "group_sigma_ms": ms_grp / max(n_grp, 1),
            "gather_ms": ms_gat / max(n_gat, 1),
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_group_double",
            "achieved": roof_ach,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": roof_ach / HBM_PEAK_GBS,
            "traffic": dbl.get("traffic"),
            "bytes_per_launch": roof_bytes,
            "unit_count": ("double-excitation pairs (ordered) x (sb R + sb) B" if ordered else
                           "double-excitation pairs evaluated (large groups once per unordered pair) "
                           "x (sb R + sb) B") + f", sb = {sb}",
            "frac_ordered_pairs": dbl["frac"],
            "frac_evaluated_pairs": dbl["frac_evaluated_pairs"],
            "kernels": kern,
        },
    }

    legs = [x for x in args.legs.split(",") if x and x != "none"]
    if legs:
        out["legs"] = {}
    if "rdm" in legs:
        out["legs"]["rdm"] = leg_rdm(plan, c, prob)
    if "davidson" in legs:
        out["legs"]["davidson"] = leg_davidson(plan, prob)
    if "ivi" in legs:
        out["legs"]["ivi"] = leg_ivi(plan, prob)
    del plan, c, sig
    torch.cuda.empty_cache()
    if "batched" in legs:
        out["legs"]["batched"] = leg_batched()
    if "spinor" in legs:
        out["legs"]["spinor"] = leg_spinor(args.steps)
    if "pt2" in legs:
        out["legs"]["pt2"] = leg_pt2()
    if "csf" in legs:
        out["legs"]["csf"] = leg_csf(args.steps)
    if "batched_small" in legs:
        out["legs"]["batched_small"] = leg_batched_small()

    if args.cpu_rows > 0:
        from oracle import sc
        rng = np.random.default_rng(2026)
        rows = np.sort(rng.choice(ndet, size=min(args.cpu_rows, ndet), replace=False))
        t0 = time.perf_counter()
        sc.sigma(prob, c_np, rows=rows)  # noqa: the oracle, timed as the CPU baseline
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
        # the same oracle on one thread, on a tenth of the sample
        threads = sc.num_threads()
        sc.set_threads(1)
        rows1 = rows[:max(1, len(rows) // 10)]
        t0 = time.perf_counter()
        sc.sigma(prob, c_np, rows=rows1)  # noqa: the oracle, timed as the CPU baseline
        dt1 = time.perf_counter() - t0
        sc.set_threads(threads)
        terms1 = float((sc.degree_rows(prob, rows1) + 1).sum() * R)
        out["cpu_baseline"]["value_1_thread"] = terms1 / dt1
        out["cpu_baseline"]["sample_1_thread"] = f"{len(rows1)} of the same rows ({int(terms1)} terms, {dt1:.1f} s)"
        log(f"[bench] cpu oracle, 1 thread: {len(rows1)} rows in {dt1:.1f}s")
    print(json.dumps(out), flush=True)


def kernel_rooflines(plan, R, sb, steps, n_grp, ms_grp, n_gat, ms_gat, n_sgl=None, ms_sgl=None, traffic=None):
    """Algorithmic bandwidth of the three sigma kernels from the plan's
    counts and the event times recorded by the library (launch stream).

    k_group_double: per ordered double-excitation pair the partner's R
    coefficients and one integral word (sb R + sb bytes); the half-work
    figure counts the pairs the kernel evaluates (groups of 64 members or
    more: once per unordered pair).  k_group_single: the same per ordered
    single pair.  k_gather: per membership or column partial its 4-byte
    index and R partial sums; per determinant its row pointer, H_II, c_I
    and sigma_I."""
    from paper_2501_18185_amd import mw
    if n_sgl is None:
        n_sgl, ms_sgl = mw.profile_read("group_single")
    dp = plan.info("double_pairs")
    dpl = plan.info("double_pairs_large_groups")
    sp = plan.info("single_pairs")
    nslot = plan.info("memberships") + plan.info("column_partials")
    ndet = plan.ndet
    lp = max(n_grp // steps, 1)   # double-group launches per step (one per root chunk)
    res = {}

    def entry(bytes_launch, n, ms, extra=None):
        t = ms / max(n, 1) * 1e-3
        ach = bytes_launch / t / 1e9 if n else 0.0
        e = {"avg_ms": ms / max(n, 1), "launches": n, "bytes_per_launch": bytes_launch, "achieved_GBps": ach,
             "frac": ach / HBM_PEAK_GBS}
        if extra:
            e.update(extra)
        return e

    per = sb * R + sb
    b_ord = dp * per / lp
    b_eval = ((dp - dpl) + dpl / 2) * per / lp
    t_d = ms_grp / max(n_grp, 1) * 1e-3
    res["k_group_double"] = entry(b_ord, n_grp, ms_grp, {
        "bytes_per_launch_evaluated_pairs": b_eval,
        "frac_evaluated_pairs": (b_eval / t_d / 1e9 / HBM_PEAK_GBS) if n_grp else 0.0})
    res["k_group_single"] = entry(sp * per / max(n_sgl // steps, 1), n_sgl, ms_sgl)
    res["k_gather"] = entry(nslot * (4 + sb * R) + ndet * (4 + sb + 2 * sb * R), n_gat, ms_gat)
    for k, v in (traffic or {}).items():
        if k in res:
            res[k]["traffic"] = v
            res[k]["traffic_over_algorithmic"] = v / res[k]["bytes_per_launch"]
    return res


def _time(fn, steps, warmup=2):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    gc.collect()
    gc.disable()
    try:
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
    finally:
        gc.enable()
    return e0.elapsed_time(e1) / steps


def leg_rdm(plan, c, prob):
    """Forward E = c^T H c and backward (gamma, Gamma) on the same space."""
    import torch
    from paper_2501_18185_amd import mw
    c1 = c[:, 0].contiguous() if c.dim() == 2 else c
    t_fwd = _time(lambda: plan.sigma(c1), 5)
    mw.profile(True)
    t_bwd = _time(lambda: plan.rdm(c1, c1), 3, warmup=1)
    mw.profile(False)
    nd, md = mw.profile_read("rdm_double")
    ns, ms_ = mw.profile_read("rdm_single")
    nq, mq = mw.profile_read("rdm_diag")
    nf, mf = mw.profile_read("rdm_final")
    # the single pairs and the occupation correlations run on a second
    # stream beside the double pairs: their times overlap
    log(f"[bench] rdm: forward {t_fwd:.2f} ms, backward {t_bwd:.2f} ms (double pairs {md / max(nd, 1):.2f} ms; "
        f"beside them single pairs {ms_ / max(ns, 1):.2f} ms and occupation correlations {mq / max(nq, 1):.2f} ms; "
        f"final pass {mf / max(nf, 1):.2f} ms)")
    # the fixed-point mode (integer atomics, order-independent bits)
    plan.rdm_fixed_point = True
    try:
        t_fix = _time(lambda: plan.rdm(c1, c1), 3, warmup=1)
    finally:
        plan.rdm_fixed_point = False
    log(f"[bench] rdm: backward in fixed point {t_fix:.2f} ms")
    # the double-pair rows: with one vector each unordered connected double
    # pair is visited once, reading the member's position (2 B) and its
    # gathered coefficient (8 B); counters of these launches are kept in
    # profiles/rdm_sci-n64.md
    t_rows = md / max(nd, 1)
    rows_bytes = plan.info("double_pairs") // 2 * (2 + 8)
    rows_gbps = rows_bytes / max(t_rows * 1e-3, 1e-12) / 1e9
    roof = {"bound": "hbm", "kernel": "k_rdm_rows (four launches)", "achieved": rows_gbps, "peak": 8000.0,
            "unit": "GB/s", "frac": rows_gbps / 8000.0, "bytes_per_backward": rows_bytes,
            "unit_count": "unordered double pairs x (2 B position + 8 B gathered coefficient)", "traffic": None}
    return {"workload": prob.name, "forward_ms": t_fwd, "backward_ms": t_bwd, "roofline": roof,
            "rdm_double_ms": md / max(nd, 1), "rdm_single_ms": ms_ / max(ns, 1), "rdm_occ_ms": mq / max(nq, 1),
            "rdm_final_ms": mf / max(nf, 1), "backward_fixed_point_ms": t_fix,
            "gamma_shape": [prob.norb] * 2, "Gamma_shape": [prob.norb] * 4}


def leg_davidson(plan, prob, iters=10):
    """Wall time per Davidson iteration (fixed iteration count)."""
    import time as _t

    import torch
    from paper_2501_18185_amd import mw
    dg = plan.diag().cpu().numpy()
    i0 = int(np.argmin(dg))
    c0 = torch.zeros((prob.ndet, 1), dtype=plan.dtype, device="cuda")
    c0[i0, 0] = 1.0
    plan.davidson(c0, tol=1e-12, max_iter=1, check=False)  # untimed: first-call allocations
    torch.cuda.synchronize()
    t0 = _t.perf_counter()
    ev, X, it, conv = plan.davidson(c0, tol=1e-12, max_iter=iters, check=False)
    dt = _t.perf_counter() - t0
    log(f"[bench] davidson: {it} iterations in {dt:.2f}s, E = {ev[0]:.10f}")
    return {"workload": prob.name, "iterations": it, "ms_per_iteration": dt * 1e3 / max(it, 1),
            "energy_after": float(ev[0])}


def leg_ivi(plan, prob, steps=10):
    """Wall time per iVI step (fixed step count, lowest root)."""
    import time as _t

    import torch
    dg = plan.diag().cpu().numpy()
    c0 = torch.zeros((prob.ndet, 1), dtype=plan.dtype, device="cuda")
    c0[int(np.argmin(dg)), 0] = 1.0
    plan.ivi(c0, tol=1e-12, max_iter=1, check=False)  # untimed: first-call allocations
    torch.cuda.synchronize()
    t0 = _t.perf_counter()
    ev, X, it, conv = plan.ivi(c0, tol=1e-12, max_iter=steps, check=False)
    dt = _t.perf_counter() - t0
    log(f"[bench] ivi: {it} steps in {dt:.2f}s, E = {ev[0]:.10f}")
    return {"workload": prob.name, "steps": it, "ms_per_step": dt * 1e3 / max(it, 1), "energy_after": float(ev[0])}


def leg_batched():
    """16 uneven problems x 4 roots: batched graph vs plain launches."""
    from concurrent.futures import ThreadPoolExecutor

    import torch
    from paper_2501_18185_amd import mw, synth
    t0 = time.perf_counter()
    probs = [synth.workload(3, i) for i in range(16)]
    with ThreadPoolExecutor(4) as ex:
        plans = list(ex.map(lambda p: mw.Plan(p, max_roots=4, upload=False), probs))
    for pl in plans:
        pl.upload()
    log(f"[bench] batched: 16 problems, {sum(p.ndet for p in probs)} dets, plans in {time.perf_counter() - t0:.1f}s")
    R = 4
    cs = [torch.from_numpy(synth.ci_vectors(p.ndet, R, synth.rng_for(3, i, synth.SEED_C))).cuda()
          for i, p in enumerate(probs)]
    outs = [torch.empty_like(c) for c in cs]
    cs1 = [[c[:, k].contiguous() for k in range(R)] for c in cs]
    outs1 = [[torch.empty_like(x) for x in row] for row in cs1]
    bpc = mw.autotune_batched(plans, cs, outs)
    t_batched = _time(lambda: mw.sigma_batched(plans, cs, outs), 10)
    # per-problem baseline: the better of the default and the tuned launch
    # parameters of each plan
    t_plain4_default = _time(lambda: [pl.sigma(c, out=o) for pl, c, o in zip(plans, cs, outs)], 5)
    for pl, c, o in zip(plans, cs, outs):
        pl.autotune(c, o)
    t_plain4_tuned = _time(lambda: [pl.sigma(c, out=o) for pl, c, o in zip(plans, cs, outs)], 5)
    t_plain4 = min(t_plain4_default, t_plain4_tuned)
    t_plain1 = _time(lambda: [pl.sigma(x, out=o) for pl, row, orow in zip(plans, cs1, outs1)
                              for x, o in zip(row, orow)], 5)
    pairs = sum(pl.info("pairs") for pl in plans)
    terms = (pairs + sum(p.ndet for p in probs)) * R
    # byte models of the three batched kernels (per launch, all problems):
    # per ordered pair R coefficients and one integral word; the gather as
    # for plain sigma
    dp = sum(pl.info("double_pairs") for pl in plans)
    sp = sum(pl.info("single_pairs") for pl in plans)
    nslot = sum(pl.info("memberships") + pl.info("column_partials") for pl in plans)
    ndet = sum(p.ndet for p in probs)
    kernel_bytes = {"k_batched_flat (double groups)": dp * (8 * R + 8),
                    "k_batched_flat (single groups)": sp * (8 * R + 8),
                    "k_batched_gather": nslot * (4 + 8 * R) + ndet * (4 + 8 + 16 * R)}
    log(f"[bench] batched: graph {t_batched:.2f} ms, 16x4-root {t_plain4:.2f} ms, 64x1-root {t_plain1:.2f} ms")
    # energies and every gradient (c, h, g) of sum_i sum_k E_ik: batched
    # sigma + batched energies + one captured graph of the gradient kernels,
    # against the same calls made problem by problem
    ges = [torch.ones(R, dtype=torch.float64, device="cuda") for _ in cs]
    gouts = mw.energy_backward_batched(plans, cs, outs, ges)

    def batched_grad():
        mw.sigma_batched(plans, cs, outs)
        mw.energy_batched(plans, cs, outs)
        mw.energy_backward_batched(plans, cs, outs, ges, outs=gouts)

    def plain_grad():
        for pl, c, o, ge in zip(plans, cs, outs, ges):
            pl.sigma(c, out=o)
            pl.energy(c, o)
            pl.energy_backward(c, o, ge)

    t_grad_batched = _time(batched_grad, 5)
    t_grad_plain = _time(plain_grad, 5)
    log(f"[bench] batched energy+gradients: graph {t_grad_batched:.2f} ms, 16 plain {t_grad_plain:.2f} ms")
    return {"workload": "batch16-n16..48-6..12e-1e4..5e5-R4", "ndet_total": sum(p.ndet for p in probs),
            "pairs_total": pairs, "double_pairs_total": dp, "single_pairs_total": sp, "slots_total": nslot,
            "kernel_bytes_per_launch": kernel_bytes, "blocks_per_cu": bpc,
            "batched_graph_ms": t_batched, "plain_16x4_ms": t_plain4,
            "plain_16x4_default_ms": t_plain4_default, "plain_16x4_tuned_ms": t_plain4_tuned,
            "plain_64x1_ms": t_plain1,
            "batched_terms_per_s": terms / (t_batched * 1e-3),
            # algorithmic bytes of the whole batch: per connected pair one
            # integral word and the partner's R coefficients
            "batched_algorithmic_GBps": pairs * (8 * R + 8) / (t_batched * 1e-3) / 1e9,
            "batched_hbm_frac": pairs * (8 * R + 8) / (t_batched * 1e-3) / (HBM_PEAK_GBS * 1e9),
            "speedup_vs_16x4": t_plain4 / t_batched, "speedup_vs_64x1": t_plain1 / t_batched,
            "grad_batched_ms": t_grad_batched, "grad_plain_16_ms": t_grad_plain,
            "grad_speedup": t_grad_plain / t_grad_batched}


def leg_batched_small():
    """32 small problems x 4 roots (each far from filling the GPU alone):
    batched graph vs 32 plain launches, where batching pays off."""
    import torch
    from paper_2501_18185_amd import mw, synth
    t0 = time.perf_counter()
    probs = []
    for i in range(32):
        n, ne = 16 + i % 5, 5 + i % 2
        rng = synth.rng_for(8, i, synth.SEED_SPACE)
        d = synth.space_selected_spinfree(n, ne, ne, 8000 + 400 * i, rng)
        probs.append(synth.Problem("spinfree", n, ne, ne, d, synth.one_body_real(n, synth.rng_for(8, i, synth.SEED_H)),
                                   synth.two_body_real(n, synth.rng_for(8, i, synth.SEED_G))))
    plans = [mw.Plan(p, max_roots=4) for p in probs]
    R = 4
    cs = [torch.from_numpy(synth.ci_vectors(p.ndet, R, synth.rng_for(8, i, synth.SEED_C))).cuda()
          for i, p in enumerate(probs)]
    outs = [torch.empty_like(c) for c in cs]
    ndet = sum(p.ndet for p in probs)
    log(f"[bench] batched small: 32 problems, {ndet} dets, ready in {time.perf_counter() - t0:.1f}s")
    mw.autotune_batched(plans, cs, outs)
    t_batched = _time(lambda: mw.sigma_batched(plans, cs, outs), 20)
    t_plain = _time(lambda: [pl.sigma(c, out=o) for pl, c, o in zip(plans, cs, outs)], 20)
    log(f"[bench] batched small: graph {t_batched:.3f} ms, 32x4-root {t_plain:.3f} ms")
    return {"workload": "batch32-n16..20-5..6e-8e3..2e4-R4", "ndet_total": ndet,
            "pairs_total": sum(pl.info("pairs") for pl in plans),
            "batched_graph_ms": t_batched, "plain_32x4_ms": t_plain, "speedup": t_plain / t_batched}


def leg_pt2():
    """Second-order energy of the lowest root of a 20,000-determinant
    n=64 10a10b variational space over its external space (exact, and with
    the doubles screening at Q_min = 1e-7)."""
    import torch
    from paper_2501_18185_amd import mw, synth
    torch.cuda.empty_cache()
    t0 = time.perf_counter()
    p = synth.workload(5)
    pl = mw.Plan(p, max_roots=1)
    dg = pl.diag().cpu().numpy()
    c0 = np.zeros((p.ndet, 1))
    c0[int(np.argmin(dg)), 0] = 1.0
    ev, X, it, conv = pl.davidson(torch.from_numpy(c0).cuda(), tol=1e-6, max_iter=100, check=False)
    x = X[:, 0].contiguous()
    log(f"[bench] pt2: space {p.ndet} dets, E0 = {ev[0]:.10f} after {it} Davidson iterations "
        f"({time.perf_counter() - t0:.1f}s)")
    res = {"workload": "pt2-n64-10a10b-2e4", "ndet": p.ndet, "e0": float(ev[0])}
    for qmin in (0.0, 1e-7):
        torch.cuda.synchronize()
        mw.profile(True)
        t1 = time.perf_counter()
        e2, st = pl.pt2(x, ev[0], qmin=qmin)
        dt = time.perf_counter() - t1
        mw.profile(False)
        _, t_enum = mw.profile_read("pt2_enum")
        _, t_bucket = mw.profile_read("pt2_bucket")
        key = "exact" if qmin == 0.0 else "screened"
        res[key] = {"qmin": qmin, "e2": float(e2[0]), "seconds": dt, "excitations_enumerated": st["enumerated"],
                    "pairs_kept": st["kept_pairs"], "external_dets": st["external"], "passes": st["passes"],
                    "buckets": st["buckets"], "kept_pairs_per_s": st["kept_pairs"] / dt,
                    "emit_ms": t_enum, "bucket_ms": t_bucket}
        # Each kept pair is one record: 32 bytes (A, H_AA, hash key and J)
        # and 8 bytes of H_AJ c_J, claimed with one returning device atomic
        # and written by the emit passes, read once by the bucket kernels.
        # The emit is bound by the claims (memory-side atomics; no published
        # peak), so the record bytes are set against HBM for scale only.
        kept = st["kept_pairs"]
        rec_bytes = 2 * 40 * kept
        hbm = rec_bytes / max((t_enum + t_bucket) * 1e-3, 1e-12) / 1e9
        res[key]["roofline"] = {"bound": "memory-side atomics", "kernel": "k_pt2_enum emit passes",
                                "achieved": kept / max(t_enum * 1e-3, 1e-12), "unit": "claims/s",
                                "record_bytes": rec_bytes, "record_GBps": hbm, "record_frac_of_hbm": hbm / 8000.0}
        log(f"[bench] pt2 {key}: E2 = {e2[0]:.10f}, {st['kept_pairs']} pairs, {st['external']} external dets, "
            f"{st['passes']} passes, {dt:.2f}s (emit {t_enum:.0f} ms, buckets {t_bucket:.0f} ms)")
    # selection of the next determinants from the same state (one call,
    # output buffer large enough)
    cmin = 1e-5
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sel = pl.select(x, ev[0], cmin, max_out=50_000_000)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    res["select"] = {"cmin": cmin, "selected_dets": int(sel.shape[0]), "seconds": dt,
                     "excitations_per_s": st["enumerated"] / dt}
    log(f"[bench] select: C_min = {cmin}: {sel.shape[0]} determinants in {dt:.2f}s")
    return res


def leg_spinor(steps):
    """Complex spinor sigma, 40 Kramers pairs, 20 electrons, 1e6 dets."""
    import torch
    from paper_2501_18185_amd import mw, synth
    t0 = time.perf_counter()
    p = synth.workload(2)
    pl = mw.Plan(p)
    log(f"[bench] spinor: ndet={p.ndet} pairs={pl.info('pairs')} ready in {time.perf_counter() - t0:.1f}s")
    c = torch.from_numpy(synth.ci_vectors(p.ndet, 1, synth.rng_for(2, 0, synth.SEED_C), complex_=True)).cuda()
    o = torch.empty_like(c)
    mw.profile(True)
    n = max(steps // 2, 3)
    ms = _time(lambda: pl.sigma(c, out=o), n)
    mw.profile(False)
    ng, mg = mw.profile_read("group_sigma")
    na, ma = mw.profile_read("gather")
    ns, msg = mw.profile_read("group_single")
    # the warm-up calls of _time are recorded too: kernel averages are per launch
    kern = kernel_rooflines(pl, 1, 16, n + 2, ng, mg, na, ma, ns, msg, traffic=measured_traffic("spinor-40kp", 1))
    pairs = pl.info("pairs")
    d = kern["k_group_double"]
    log(f"[bench] spinor: {ms:.2f} ms per sigma")
    return {"workload": p.name, "ndet": p.ndet, "connected_pairs": pairs, "ms_per_sigma": ms,
            "terms_per_s": (pairs + p.ndet) / (ms * 1e-3), "group_sigma_ms": d["avg_ms"],
            # ordered pairs x 32 B exceed the peak: the Hermitian half-work
            # evaluates each unordered pair of a large group once, so the
            # evaluated-pair model is the one that bounds this kernel
            "group_sigma_GBps_ordered_pairs": d["achieved_GBps"],
            "frac_ordered_pairs": d["frac"],
            "group_sigma_GBps": d["bytes_per_launch_evaluated_pairs"] / (d["avg_ms"] * 1e-3) / 1e9,
            "hbm_frac": d["frac_evaluated_pairs"], "kernels": kern}


def leg_csf(steps):
    """CSF-basis sigma (T^T H T c) against the determinant sigma of the same
    configuration-complete space: the singles-and-doubles space of n=64
    10a10b, and an open-shell-rich space (n=32 8a8b, 10 and 12 open shells)
    where the determinants outnumber the CSFs most."""
    import torch
    from paper_2501_18185_amd import mw, synth
    out = {}
    for wk, tag in ((6, "sd"), (7, "open")):
        t0 = time.perf_counter()
        p = synth.workload(wk)
        res = {"workload": p.name, "ndet": p.ndet}
        for R in (1, 4):
            pl = mw.Plan(p, max_roots=R, build="device")
            cb = mw.Csf(pl, 0)
            if R == 1:
                log(f"[bench] csf {tag}: ndet={p.ndet} ncsf={cb.ncsf} configurations={cb.info('configurations')} "
                    f"max open shells={cb.info('max_open')} ready in {time.perf_counter() - t0:.1f}s")
                res.update({"ncsf": cb.ncsf, "configurations": cb.info("configurations"),
                            "max_open_shells": cb.info("max_open"),
                            "plan_workspace_bytes": pl.info("workspace_bytes"),
                            "csf_workspace_bytes": cb.info("workspace_bytes")})
            c = torch.from_numpy(synth.ci_vectors(cb.ncsf, R, synth.rng_for(wk, 0, synth.SEED_C))).cuda()
            o = torch.empty_like(c)
            x = cb.to_det(c)
            y = torch.empty_like(x)
            work = torch.empty(2 * p.ndet * R, dtype=torch.float64, device="cuda")
            n = max(steps // 2, 3)
            ms_csf = _time(lambda: cb.sigma(c, out=o, work=work), n)
            ms_det = _time(lambda: pl.sigma(x, out=y), n)
            ms_t = _time(lambda: cb.to_det(c, out=x), n)
            ms_tt = _time(lambda: cb.from_det(y, out=o), n)
            log(f"[bench] csf {tag}: {R} roots, {ms_csf:.2f} ms per CSF sigma, {ms_det:.2f} ms determinant sigma, "
                f"transforms {ms_t:.3f} + {ms_tt:.3f} ms")
            res[f"roots{R}"] = {"ms_per_csf_sigma": ms_csf, "ms_per_det_sigma": ms_det, "to_det_ms": ms_t,
                                "from_det_ms": ms_tt, "vector_bytes_det": p.ndet * R * 8,
                                "vector_bytes_csf": cb.ncsf * R * 8}
            del pl, cb, c, o, x, y, work
            torch.cuda.empty_cache()
        out[tag] = res
    return out


if __name__ == "__main__":
    main()
