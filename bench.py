#!/usr/bin/env python3
"""Throughput of the sFMM hot path on one MI355X.

One step = one full pass of the method over the workload: keys, sort, tree,
box geometry, Algorithm 1 walk, list sorting, target location (sfmm_plan) and
P2M, M2M, M2L, L2L, L2P, P2P (sfmm_execute).  Inputs are resident in HBM
before timing starts.  The metric is targets per second of psi + deflection
at relative error <= the tolerance.

Prints one JSON line (rank 0, N = 1 only).  Progress goes to stderr.
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

PEAK_FP64_TFLOPS = 78.6      # MI355X FP64 vector (and FP64 matrix) peak
PEAK_HBM_GBS = 8000.0
# FP64 flops of one particle-target pair as the pair loop executes them (FMA
# = 2): 3 for d, 5 for |d|^2, ~23 for log|d|^2 (range reduction, table entry,
# degree-7 series), 8 for 1/|d|^2 (hardware estimate + 2 Newton steps), 1 for
# q/|d|^2, 8 for the four accumulations; the VALU counters read 7.27e10 FP64
# flops for 1.52e9 pairs on clustered-1e7
FLOP_PER_P2P_PAIR = 48


# Source files of each timed kernel: the traffic measured by the counters is
# only used while these files are unchanged.
KERNEL_SOURCES = {
    "m2l": ["k_fmm.hip", "expand.hpp", "common.hpp", "k_tree.hip"],  # k_tree.hip: the box order
    "p2p": ["k_p2p.hip", "expand.hpp", "common.hpp"],
    "m2p": ["k_p2p.hip", "expand.hpp", "common.hpp"],
}
KERNEL_NAMES = {"m2l": "k_m2l_team", "p2p": "k_p2p", "m2p": "k_m2p"}
M2L_TEAM2_MIN_BOXES = 65536  # the library's switch to two-lane M2L teams (boxes)


def source_hash(stage: str) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[stage]:
        with open(os.path.join(ROOT, "paper_2210_07021_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, stage: str):
    """HBM bytes per launch (read + write) of a stage's kernel, from the
    committed counter summary profiles/traffic_<workload>.md (lines
    'traffic <stage> read=<bytes> write=<bytes> src=<hash>'), or None when
    there is none or the kernel's sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        for line in fh:
            parts = line.split()
            if len(parts) == 5 and parts[0] == "traffic" and parts[1] == stage:
                kv = dict(x.split("=", 1) for x in parts[2:])
                if kv["src"] != source_hash(stage):
                    return None
                return float(kv["read"]) + float(kv["write"])
    return None


def m2l_flops(p: int) -> int:
    """Algorithmic flops of one Lemma 3 translation at order p: two
    triangular Taylor-shift factors (p(p+1) complex*real FMAs, 4p^2 + 4p
    flops) plus the phase, diagonal and output terms (~28p)."""
    return 4 * p * p + 32 * p


def m2p_flops(p: int) -> int:
    """FP64 flops of one multipole evaluation at a target (close leaf taken
    by its Lemma 1 expansion): the two Horner recurrences for f and g
    (18 flops per order) plus projection, log and output (~180)."""
    return 18 * p + 180


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="clustered-1e7")
    ap.add_argument("--scale", type=float, default=1.0, help="shrink N (quick runs only)")
    ap.add_argument("--tolerance", type=float, default=1e-10)
    ap.add_argument("--order", type=int, default=0, help="fixed order instead of the tolerance")
    ap.add_argument("--leaf-size", type=int, default=56)  # the fastest of a leaf-size sweep on clustered-1e7
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--accuracy-targets", type=int, default=10000,
                    help="size of the seeded target subset the oracle checks (untimed)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true", help="only the FP64 leg (same as --legs fp64)")
    ap.add_argument("--legs", default="fp64,fp32_mixed,fp32_learned",
                    help="comma list of fp64 (the headline), fp32_mixed (fixed order), fp32_bound, "
                         "fp32_learned; the first one fills the top-level fields")
    ap.add_argument("--fp32-tolerance", type=float, default=1e-6)
    ap.add_argument("--shells", type=int, default=0,
                    help="measure the batched form instead: this many lensing shells (N_s log-uniform in "
                         "[1e5, 5e6], 786,432 grid targets each) in one recorded graph")
    ap.add_argument("--shells-leg", type=int, default=40,
                    help="after the main legs, the batched form on this many shells in FP64 (tolerance) and the "
                         "precision tier (fp32 tolerance), reported under 'shells' (0: skip)")
    ap.add_argument("--no-extra-legs", action="store_true",
                    help="skip the Hessian leg (psi, alpha and the Hessian of Sec. 2.2 on the same workload) and "
                         "the ray-tracing leg (8 lensing layers, Eq. DIS_PRO with the distortion matrix)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 1 GiB device to device (scale for the traffic counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "this build has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_probe:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters give
        # the scale from counter units to HBM bytes read / written
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": a.numel() * 8}), flush=True)
        return
    import paper_2210_07021_amd as sf
    from paper_2210_07021_amd import skies

    sf.load_library()
    if args.shells > 0:
        print(json.dumps(bench_shells(args, sf, skies, torch, args.shells, args.tolerance, 0)), flush=True)
        return
    torch.cuda.set_device(0)
    log(f"[bench] generating {args.workload} (scale {args.scale})")
    t = time.time()
    src_h, q_h, tgt_h = skies.workload(args.workload, scale=args.scale)
    N, M = src_h.shape[1], tgt_h.shape[1]
    log(f"[bench] N={N} M={M} generated in {time.time() - t:.1f}s")
    src = torch.from_numpy(src_h).cuda()
    q = torch.from_numpy(q_h).cuda()
    tgt = torch.from_numpy(tgt_h).cuda()
    psi = torch.empty(M, dtype=torch.float64, device="cuda")
    defl = torch.empty((3, M), dtype=torch.float64, device="cuda")
    opts = dict(leaf_size=args.leaf_size)
    if args.order > 0:
        opts["order"] = args.order
    else:
        opts["tolerance"] = args.tolerance
    torch.cuda.synchronize()

    def run(opts, out_psi, out_defl, label):
        """W untimed steps, then K timed ones; returns (seconds, stage ms, stats)."""
        def step():
            plan = sf.Plan(src, q, tgt, **opts)
            plan.execute(out_psi, out_defl)
            return plan

        for w in range(args.warmup):
            t = time.time()
            plan = step()
            torch.cuda.synchronize()
            stats = plan.stats()
            plan.close()
            log(f"[bench] {label} warmup {w}: {time.time() - t:.3f}s")
        if args.warmup == 0:
            plan = step()
            stats = plan.stats()
            plan.close()
        sf.profile_reset()
        sf.profile_enable(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            plan = step()
            plan.close()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sf.profile_enable(False)
        prof = sf.profile_read()
        log(f"[bench] {label}: {args.steps} steps in {t1 - t0:.3f}s")
        return t1 - t0, {k: v[0] / args.steps for k, v in prof.items()}, stats

    legs_req = ["fp64"] if args.no_fp32 else [x for x in args.legs.split(",") if x]
    bad = set(legs_req) - {"fp64", "fp32_mixed", "fp32_bound", "fp32_learned"}
    if bad or not legs_req:
        raise SystemExit(f"unknown legs {sorted(bad)}")
    legs, outs = {}, {}

    def run_leg(leg):
        if leg == "fp64":
            o, po, do = opts, psi, defl
        else:
            # the precision tier at its own tolerance, same workload; the
            # learned per-interaction order uses a network trained (untimed)
            # on labels of the clustered 1e6 sky, a different sky and seed
            o = dict(leaf_size=args.leaf_size, tolerance=args.fp32_tolerance, precision=sf.SFMM_FP32_MIXED)
            if leg == "fp32_bound":
                o["order_policy"] = sf.SFMM_ORDER_BOUND
            if leg == "fp32_learned":
                from paper_2210_07021_amd import learn
                t = time.time()
                f_tr, l_tr = learn.order_training_data([skies.workload("clustered-1e6")], args.fp32_tolerance,
                                                       leaf_size=args.leaf_size, samples_per_sky=60000, seed=1)
                w_net, _ = learn.train_order_network(f_tr, l_tr, epochs=30)
                log(f"[bench] order network trained in {time.time() - t:.1f}s (untimed)")
                o.update(order_policy=sf.SFMM_ORDER_LEARNED, mlp_weights=w_net)
            po, do = torch.empty_like(psi), torch.empty_like(defl)
        e, st, s_ = run(o, po, do, leg)
        outs[leg] = (po, do)
        rec = {"value": M * args.steps / e, "unit": "targets/s", "ms_per_step": 1e3 * e / args.steps,
               "tolerance": args.tolerance if leg == "fp64" else args.fp32_tolerance, "order": s_["order"],
               "dtype": "f64" if leg == "fp64" else "f32+f64",
               "m2l_work_vs_fixed": s_["m2l_order_sq"] / max(1, s_["n_m2l"] * s_["order"] ** 2),
               "stages_ms": {k: round(v, 4) for k, v in st.items()}, "_elapsed": e, "_stats": s_}
        if leg in ("fp32_bound", "fp32_learned"):
            rec["judge"] = {"targets": s_["judge_targets"], "psi_rel_l2": s_["judge_psi"],
                            "alpha_rel_l2": s_["judge_alpha"], "fell_back": bool(s_["fell_back"])}
        legs[leg] = rec

    for i, leg in enumerate(legs_req):
        if i == 0:
            run_leg(leg)  # the line's own leg: a failure ends the bench
            continue
        try:
            run_leg(leg)
        except Exception as e:  # noqa: BLE001  (another leg's failure is reported in its field)
            log(f"[bench] {leg} leg failed: {e!r}")
            legs[leg] = {"error": repr(e)}
            outs.pop(leg, None)
    main_leg = legs_req[0]
    elapsed, stats = legs[main_leg].pop("_elapsed"), legs[main_leg].pop("_stats")
    stages_ms = legs[main_leg]["stages_ms"]
    for leg in legs_req[1:]:
        legs[leg].pop("_elapsed", None)
        legs[leg].pop("_stats", None)
    psi, defl = outs[main_leg]

    p = stats["order"]
    roofline, kernels = None, None
    if main_leg == "fp64":
        work = {
            "m2l": ("alu", stats["n_m2l"] * m2l_flops(p), PEAK_FP64_TFLOPS, "TFLOP/s"),
            "p2p": ("alu", stats["n_p2p_pairs"] * FLOP_PER_P2P_PAIR, PEAK_FP64_TFLOPS, "TFLOP/s"),
            "m2p": ("alu", stats["n_m2p_evals"] * m2p_flops(p), PEAK_FP64_TFLOPS, "TFLOP/s"),
        }
        dom = max(work, key=lambda k: stages_ms[k])
        bound, flops, peak, unit = work[dom]
        achieved = flops / (stages_ms[dom] * 1e-3) / 1e12
        kname = KERNEL_NAMES[dom]
        if dom == "m2l" and stats["n_boxes"] >= M2L_TEAM2_MIN_BOXES:
            kname = "k_m2l_team2"  # two lanes per target box on large trees
        roofline = {"kernel": kname, "bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
                    "frac": achieved / peak, "traffic": measured_traffic(args.workload, dom),
                    "work_per_launch": flops, "avg_launch_ms": stages_ms[dom]}
        # every timed FMM kernel against its own roofline (stage time from the
        # library's HIP events; L2P by its algorithmic bytes: coordinates in,
        # psi and alpha out, each target leaf's local record once)
        kernels = {}
        for k, (bd, w, pk, u) in work.items():
            a_ = w / (stages_ms[k] * 1e-3) / 1e12
            kernels[k] = {"bound": bd, "achieved": round(a_, 3), "peak": pk, "unit": u, "frac": round(a_ / pk, 4),
                          "ms": stages_ms[k]}
        l2p_bytes = M * 56 + stats["n_target_leaves"] * (2 * p + 2) * 8
        a_ = l2p_bytes / (stages_ms["l2p"] * 1e-3) / 1e9
        kernels["l2p"] = {"bound": "hbm", "achieved": round(a_, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                          "frac": round(a_ / PEAK_HBM_GBS, 4), "ms": stages_ms["l2p"]}
        # the source keys and sort stage: per point 24 B of coordinates in,
        # 12 B of key and index out, 8 radix passes of 8 bits over the 62-bit
        # keys (12 B read and written each), and the gather of the 32-byte
        # sorted records (read and written)
        sort_bytes = N * (36 + 8 * 24 + 64)
        a_ = sort_bytes / (stages_ms["src_keys_sort"] * 1e-3) / 1e9
        kernels["sort"] = {"bound": "hbm", "achieved": round(a_, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                           "frac": round(a_ / PEAK_HBM_GBS, 4), "ms": stages_ms["src_keys_sort"]}

    result = {
        "metric": ("targets/s (psi+deflection) at 1e-10 rel err, N=1e7"
                   if (args.workload, legs_req[0], args.tolerance) == ("clustered-1e7", "fp64", 1e-10) else
                   f"targets/s (psi+deflection) at {legs[main_leg]['tolerance']:g} rel err, {args.workload}"),
        "value": M * args.steps / elapsed,
        "unit": "targets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": legs[main_leg]["dtype"],
        "data": "synthetic",
        "config": {"workload": args.workload, "N": N, "M": M,
                   "tolerance": None if (args.order > 0 and main_leg == "fp64") else legs[main_leg]["tolerance"],
                   "order": p, "leaf_size": args.leaf_size,
                   "precision": "fp64" if main_leg == "fp64" else "fp32_mixed", "c_s": 2.0, "c_t": 0.5,
                   "n_boxes": stats["n_boxes"], "n_m2l": stats["n_m2l"], "n_p2p_pairs": stats["n_p2p_pairs"],
                   "n_m2p_evals": stats["n_m2p_evals"]},
        "stages_ms": {k: round(v, 4) for k, v in stages_ms.items()},
        "roofline": roofline,
        "kernels": kernels,
    }
    if main_leg != "fp64":
        result["leg"] = main_leg
    result.update({k: v for k, v in legs.items() if k != main_leg})

    if not args.no_cpu_baseline:
        import oracle
        psi_h = psi.cpu().numpy()
        defl_h = defl.cpu().numpy()
        # the seeded 1e4-target subset of the accuracy claim (the same subset
        # as the full-size parity tests); its first k targets, timed alone,
        # are the CPU baseline (a bounded sample of about cpu_seconds)
        sub = np.random.default_rng(skies.BASE_SEED + 1001).choice(M, size=min(M, args.accuracy_targets),
                                                                  replace=False)
        # per-target cost from two probes (each call also pays a fixed set-up
        # of about a copy of the sources, which the difference removes)
        oracle.direct(src_h, q_h, tgt_h[:, sub[:8]])  # thread start-up
        t = time.perf_counter()
        oracle.direct(src_h, q_h, tgt_h[:, sub[:16]])
        t16 = time.perf_counter() - t
        t = time.perf_counter()
        oracle.direct(src_h, q_h, tgt_h[:, sub[:80]])
        t80 = time.perf_counter() - t
        per_target = max((t80 - t16) / 64, t80 / 80 * 0.05, 1e-9)
        k = int(min(len(sub), max(80, args.cpu_seconds / per_target)))
        log(f"[bench] cpu baseline: oracle on {k} of the {len(sub)} seeded targets")
        t = time.perf_counter()
        ref_p1, ref_a1 = oracle.direct(src_h, q_h, tgt_h[:, sub[:k]])
        t_cpu = time.perf_counter() - t
        cores = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
        result["cpu_baseline"] = {"value": k / t_cpu, "unit": "targets/s", "cores": cores, "kind": "oracle",
                                  "sample": f"{k} seeded targets of the same workload, all {N} sources, "
                                            f"{t_cpu:.1f}s"}
        if k < len(sub):
            log(f"[bench] accuracy: oracle on the other {len(sub) - k} targets (untimed)")
            ref_p2, ref_a2 = oracle.direct(src_h, q_h, tgt_h[:, sub[k:]])
            ref_p = np.concatenate([ref_p1, ref_p2])
            ref_a = np.concatenate([ref_a1, ref_a2], axis=1)
        else:
            ref_p, ref_a = ref_p1, ref_a1

        def accuracy(ph, dh):
            # relative L2 error, and the worst target over the rms of the reference
            dp = ph[sub] - ref_p
            da = np.linalg.norm(dh[:, sub] - ref_a, axis=0)
            rms_a = np.sqrt(np.mean(np.sum(ref_a * ref_a, axis=0)))
            return {"psi_rel_l2": float(np.linalg.norm(dp) / np.linalg.norm(ref_p)),
                    "alpha_rel_l2": float(np.linalg.norm(da) / np.linalg.norm(ref_a)),
                    "psi_worst_target": float(np.abs(dp).max() / np.sqrt(np.mean(ref_p * ref_p))),
                    "alpha_worst_target": float(da.max() / rms_a), "targets": int(len(sub))}

        result["accuracy"] = accuracy(psi_h, defl_h)
        for leg in legs_req[1:]:
            if leg in outs:
                p32, d32 = outs[leg]
                result[leg]["accuracy"] = accuracy(p32.cpu().numpy(), d32.cpu().numpy())
    # the extra legs report an error in their own field rather than losing
    # the line (the headline above is complete by now)
    def extra(name, fn):
        try:
            result[name] = fn()
        except Exception as e:  # noqa: BLE001
            log(f"[bench] {name} leg failed: {e!r}")
            result[name] = {"error": repr(e)}

    if not args.no_extra_legs and legs_req[0] == "fp64":
        extra("hessian", lambda: bench_hessian(args, sf, torch, src, q, tgt, src_h, q_h, tgt_h,
                                               None if args.no_cpu_baseline else sub[:500]))
        extra("raytrace", lambda: bench_raytrace(args, sf, skies, torch, check=not args.no_cpu_baseline))
    if args.shells_leg > 0 and legs_req[0] == "fp64":
        del src, q, tgt, psi, defl, outs
        torch.cuda.empty_cache()

        def shells():
            sh = {}
            for name, tol, prec in (("fp64", args.tolerance, sf.SFMM_FP64),
                                    ("fp32_mixed", args.fp32_tolerance, sf.SFMM_FP32_MIXED)):
                r = bench_shells(args, sf, skies, torch, args.shells_leg, tol, prec)
                sh[name] = {k: r[k] for k in ("value", "ms_per_step", "plan_ms", "execute_graph_ms",
                                             "execute_direct_ms", "execute_targets_per_s_graph")}
                sh[name]["tolerance"] = tol
                sh[name]["options"] = r["config"]["options"]
            sh["config"] = {"workload": f"shells-{args.shells_leg}", "N": r["config"]["N"], "M": r["config"]["M"]}
            return sh

        extra("shells", shells)
    print(json.dumps(result), flush=True)


def bench_hessian(args, sf, torch, src, q, tgt, src_h, q_h, tgt_h, sub):
    """Plan + execute_hessian on the main workload at the main tolerance
    (K timed steps after one warm-up); the Hessian against the oracle's on
    the first targets of the seeded subset (untimed)."""
    M = tgt.shape[1]

    def step():
        plan = sf.Plan(src, q, tgt, tolerance=args.tolerance, leaf_size=args.leaf_size)
        out = plan.execute_hessian()
        return plan, out

    plan, out = step()
    torch.cuda.synchronize()
    plan.close()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan, out = step()
        plan.close()
    torch.cuda.synchronize()
    e = (time.perf_counter() - t0) / args.steps
    log(f"[bench] hessian: {1e3 * e:.2f} ms per step")
    rec = {"value": M / e, "unit": "targets/s", "ms_per_step": 1e3 * e, "tolerance": args.tolerance,
           "dtype": "f64", "outputs": "psi, alpha, Hessian (H_11, H_12, H_22)"}
    if sub is not None:
        import oracle
        ref = oracle.hessian(src_h, q_h, tgt_h[:, sub])
        h = out[2].cpu().numpy()[:, sub]
        rec["accuracy"] = {"hessian_rel_l2": float(np.linalg.norm(h - ref) / np.linalg.norm(ref)),
                           "targets": int(len(sub))}
    return rec


def bench_raytrace(args, sf, skies, torch, check):
    """Multi-plane backtracking: 8 layers of the clustered recipe (N = 1e6
    each, own seeds), 786,432 rays on the N_side 256 grid, weights of a
    source plane behind the last layer, with the distortion matrix; K timed
    traces after one warm-up.  A seeded subset of 200 rays against the
    oracle's trace (untimed)."""
    n_layer = 8
    layers = []
    for i in range(n_layer):
        rng = skies.rng_for(500 + i)
        s_ = skies.clustered(1_000_000, rng)
        layers.append((torch.from_numpy(s_).cuda(), torch.from_numpy(skies.masses_lognormal(1_000_000, rng) * 1e-7).cuda()))
    rays = skies.grid(256)
    weights = [(n_layer - i) / (n_layer + 1) for i in range(n_layer)]
    rays_d = torch.from_numpy(rays).cuda()
    out = sf.raytrace(layers, weights, rays_d, tolerance=args.tolerance, leaf_size=args.leaf_size)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = sf.raytrace(layers, weights, rays_d, tolerance=args.tolerance, leaf_size=args.leaf_size)
    torch.cuda.synchronize()
    e = (time.perf_counter() - t0) / args.steps
    m = rays.shape[1]
    log(f"[bench] raytrace: {1e3 * e:.2f} ms per trace of {n_layer} layers")
    rec = {"value": m / e, "unit": "rays/s", "ms_per_trace": 1e3 * e, "layers": n_layer,
           "sources_per_layer": 1_000_000, "rays": m, "tolerance": args.tolerance, "distortion": True}
    if check:
        from oracle import raytrace as ort
        idx = np.random.default_rng(skies.BASE_SEED + 77).choice(m, size=200, replace=False)
        ref_n, ref_A = ort.trace([(a.cpu().numpy(), b.cpu().numpy()) for a, b in layers], weights, rays[:, idx])
        got_n, got_A = out[0].cpu().numpy()[:, idx], out[1].cpu().numpy()[:, idx]
        shift = np.linalg.norm(ref_n - rays[:, idx], axis=0)
        rec["accuracy"] = {
            "position_error_over_shift": float(np.linalg.norm(got_n - ref_n) / np.linalg.norm(shift)),
            "distortion_error_over_A_minus_I": float(
                np.linalg.norm(got_A - ref_A) / np.linalg.norm(ref_A - np.array([[1.0], [0.0], [0.0], [1.0]]))),
            "rays": 200}
    return rec


def bench_shells(args, sf, skies, torch, n_shell, tolerance, precision):
    """Batched shells: autotune on the median shell (untimed), plan the batch,
    record the graph (untimed warm-up), then time K graph replays and K
    direct per-shell executes; returns the record (plan + graph execute)."""
    from paper_2210_07021_amd import tune
    t = time.time()
    sh = skies.shells(n_shell, scale=args.scale)
    ntot = sum(x[0].shape[1] for x in sh)
    mtot = sum(x[2].shape[1] for x in sh)
    log(f"[bench] {n_shell} shells, N = {ntot}, M = {mtot}, generated in {time.time() - t:.1f}s")
    srcs = [torch.from_numpy(x[0]).cuda() for x in sh]
    qs = [torch.from_numpy(x[1]).cuda() for x in sh]
    tgts = [torch.from_numpy(x[2]).cuda() for x in sh]
    med = sorted(range(len(sh)), key=lambda i: sh[i][0].shape[1])[len(sh) // 2]
    best, t_best, _ = tune.autotune(srcs[med], qs[med], tgts[med], tolerance=tolerance, precision=precision,
                                    repeats=1)
    log(f"[bench] autotuned on shell {med}: {best}")
    opts = {k: v for k, v in best.items()}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = sf.Batch(srcs, qs, tgts, **opts)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    psi, defl = b.execute()  # direct pass + recording + first launch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.execute(psi, defl)
    torch.cuda.synchronize()
    t_graph = (time.perf_counter() - t0) / args.steps
    plans = [b.plan(i) for i in range(len(sh))]
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for i, p in enumerate(plans):
            p.execute(psi[i], defl[i])
    torch.cuda.synchronize()
    t_direct = (time.perf_counter() - t0) / args.steps
    log(f"[bench] shells: plan {1e3 * t_plan:.1f} ms, graph execute {1e3 * t_graph:.1f} ms, "
        f"direct {1e3 * t_direct:.1f} ms")
    b.close()
    return {
        "metric": "targets/s (psi+deflection), batched lensing shells, plan + execute",
        "value": mtot / (t_plan + t_graph), "unit": "targets/s", "n_gpus": 1, "steps": args.steps,
        "warmup": 1, "ms_per_step": 1e3 * (t_plan + t_graph), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if precision == 0 else "f32+f64", "data": "synthetic",
        "config": {"workload": f"shells-{n_shell}", "N": ntot, "M": mtot, "tolerance": tolerance,
                   "options": {k: v for k, v in opts.items() if k != "tolerance"}},
        "plan_ms": 1e3 * t_plan, "execute_graph_ms": 1e3 * t_graph, "execute_direct_ms": 1e3 * t_direct,
        "execute_targets_per_s_graph": mtot / t_graph,
    }


if __name__ == "__main__":
    main()
