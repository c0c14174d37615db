"""Benchmark of the MI355X Cartesian FMM (one JSON line on stdout).

Default workload: 100,000 point dipoles uniform in the unit cube, p = 8,
theta = 0.5, ncrit = 64, potential + field (the configuration the headline
metric is quoted on).  One step = upward pass + evaluation (P2M, M2M, M2L,
L2L, L2P, P2P) with the octree and interaction lists resident, as the metric
counts particle evaluations per second of N / (t_upward + t_evaluate); the
tree build (set-up, excluded by the paper's own timings) is reported
separately.  The headline precision is MIXED (FP32 M2L/P2P, FP64 elsewhere);
the plain FP64 GPU path is timed on the same tree and reported beside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 2] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks (dense, per GPU)
PEAK_FP32_VALU = 157.3e12
PEAK_FP64_VALU = 78.6e12
PEAK_HBM = 8.0e12


def _src_hash():
    h = hashlib.sha256()
    for f in ("paper_2005_12351_amd/csrc/gen_m2l.py", "paper_2005_12351_amd/csrc/m2l.hip",
              "paper_2005_12351_amd/csrc/tree_host.cpp"):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic(kernel_key: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources."""
    f = os.path.join(ROOT, "profiles", "counters.json")
    if not os.path.exists(f):
        return None
    try:
        d = json.load(open(f))
        e = d.get(kernel_key)
        if e and e.get("src_hash") == _src_hash():
            return e.get("bytes_per_launch")
    except Exception:
        return None
    return None


def serve_bench(fmm, W, torch, n_requests=512, slots=8, budget=2 << 30):
    """Serving workload: requests with N log-uniform in [1e3, 2e5], source
    order in {0,1,2}, p in {4,6,8}, uniform or Plummer positions, theta 0.5,
    ncrit 64, mixed precision.  A closed-loop pass (all submitted at once)
    measures the saturated request rate; the timed open-loop pass replays the
    Poisson arrivals at 0.7 times that rate.  Latency = done - arrival."""
    import threading
    reqs = W.serving_stream(n_requests, rate=1.0)
    dev = []
    for r in reqs:
        w = r.workload
        dev.append((w, torch.from_numpy(w.pos).cuda(), torch.from_numpy(w.moments).cuda(),
                    torch.empty(w.n, dtype=torch.float64, device="cuda"),
                    torch.empty((w.n, 3), dtype=torch.float64, device="cuda")))
    torch.cuda.synchronize()

    def submit(ctx, d):
        w = d[0]
        return ctx.submit(n=w.n, order=w.order, p=w.p, theta=w.theta, ncrit=w.ncrit, pos=d[1], moments=d[2],
                          phi=d[3], field=d[4], precision=fmm.FMM_PREC_MIXED)

    # closed loop: saturated rate
    ctx = fmm.Context(0, budget_bytes=budget)
    ctx.serve_start(slots)
    t0 = time.perf_counter()
    tk = [submit(ctx, d) for d in dev]
    for t in tk:
        ctx.wait(t)
    sat_rate = n_requests / (time.perf_counter() - t0)
    ctx.close()
    # open loop at 0.7 x saturated rate
    lam = 0.7 * sat_rate
    ctx = fmm.Context(0, budget_bytes=budget)
    ctx.serve_start(slots)
    tickets = [None] * n_requests
    start = time.perf_counter()

    def feeder():
        for k, (r, d) in enumerate(zip(reqs, dev)):
            delay = start + r.arrival / lam - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            tickets[k] = submit(ctx, d)

    th = threading.Thread(target=feeder)
    th.start()
    th.join()
    for t in tickets:
        ctx.wait(t)
    times = [ctx.request_times(t) for t in tickets]
    phases = [ctx.request_phases(t) for t in tickets]
    stats = ctx.serve_stats()
    ctx.close()
    lat = np.array([x["done"] - x["submit"] for x in times])
    span = max(x["done"] for x in times) - min(x["submit"] for x in times)
    nsum = sum(d[0].n for d in dev)
    return {"requests": n_requests, "slots": slots, "budget_bytes": budget, "lambda_req_per_s": lam,
            "saturated_req_per_s": sat_rate, "p50_latency_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_latency_ms": float(np.percentile(lat, 99) * 1e3), "mean_latency_ms": float(lat.mean() * 1e3),
            "throughput_evals_per_s": nsum / span, "peak_running": stats["peak_running"],
            "peak_admitted_bytes": stats["peak_in_use"], "total_particles": nsum,
            "mean_phase_ms": {"queued": float(np.mean([x["admit"] - x["submit"] for x in times]) * 1e3),
                              "tree_build": float(np.mean([p["built"] - x["admit"] for x, p in zip(times, phases)]) * 1e3),
                              "upward_evaluate": float(np.mean([p["computed"] - p["built"] for p in phases]) * 1e3),
                              "release": float(np.mean([x["done"] - p["computed"] for x, p in zip(times, phases)]) * 1e3)},
            "note": "latency = done - arrival; it includes the tree build of each request"}


def accuracy_run(fmm, torch, w, pos, mom, outputs, ctx, args, dev, sample, pd, Ed, theta=0.3, p=10):
    """The same particles at the smallest (theta, p) of a sweep (theta 0.5,
    0.4, 0.3; p 6, 8, 10) whose truncation error against the direct sum is
    below 1e-6 for both phi and E (theta 0.3, p 10; the literal parameters
    give 1.8e-4 / 1e-5 with the half-side cell radius).  Reported beside the
    headline, errors measured on the sampled targets."""
    import oracle
    tree = fmm.Tree(ctx, pos, w.ncrit, theta)
    phi = torch.empty(w.n, dtype=torch.float64, device=dev)
    fld = torch.empty((w.n, 3), dtype=torch.float64, device=dev)
    out = {"theta": theta, "p": p, "info": tree.info()}
    runs = (("mixed", fmm.FMM_PREC_MIXED, fmm.FMM_M2L_HARMONIC), ("fp64", fmm.FMM_PREC_FP64, fmm.FMM_M2L_HARMONIC),
            ("mixed_full_basis", fmm.FMM_PREC_MIXED, fmm.FMM_M2L_FULL))
    for name, prec, basis in runs:
        ctx.set_overlap(False)
        ctx.set_m2l_basis(basis)
        for _ in range(3):
            tree.run(w.order, mom, p, prec, outputs, phi, fld)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        k = max(3, args.steps // 2)
        for _ in range(k):
            tree.run(w.order, mom, p, prec, outputs, phi, fld)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / k
        ph, E = phi.cpu().numpy(), fld.cpu().numpy()
        out[name] = {"value": w.n / dt, "unit": "evals/s", "ms_per_step": dt * 1e3,
                     "phi_vs_direct": oracle.rel_l2(ph[sample], pd), "E_vs_direct": oracle.rel_l2(E[sample], Ed)}
    ctx.set_m2l_basis(fmm.FMM_M2L_HARMONIC)
    tree.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--method", choices=["fmm", "bh"], default="fmm",
                    help="FMM with dual-tree lists (default) or multipolar Barnes-Hut")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline and error checks")
    ap.add_argument("--n", type=int, default=0, help="shrink the workload (testing only)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving-stream measurement")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run one plain device-to-device copy of MIB MiB (reference for HBM counters)")
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the run at the smallest (theta, p) that reaches 1e-6 against the direct sum")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only (no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2005_12351_amd import fmm, workloads as W

    bh = args.method == "bh"
    w = W.config(args.config, n_override=args.n or None)
    dev = torch.device("cuda", 0)
    pos = torch.from_numpy(w.pos).to(dev)
    mom = torch.from_numpy(w.moments).to(dev)
    outputs = fmm.FMM_FIELD if w.outputs == "field" else (fmm.FMM_POT | fmm.FMM_FIELD)
    ctx = fmm.Context(0)
    if args.calibrate_copy:
        a_ = torch.ones(args.calibrate_copy << 18, dtype=torch.float32, device=dev)
        b_ = torch.empty_like(a_)
        torch.cuda.synchronize()
        b_.copy_(a_)
        torch.cuda.synchronize()
        del a_, b_

    t0 = time.perf_counter()
    tree = fmm.Tree(ctx, pos, w.ncrit, w.theta, fmm.FMM_METHOD_BH if bh else fmm.FMM_METHOD_FMM)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    info = tree.info()

    def run(prec, steps, warmup):
        """the timed region: each step is fmm_run (upward + evaluate as one
        captured graph, replayed, on one stream), no per-kernel events"""
        phi = torch.empty(w.n, dtype=torch.float64, device=dev) if outputs & fmm.FMM_POT else None
        fld = torch.empty((w.n, 3), dtype=torch.float64, device=dev)
        ctx.profile(False)
        ctx.set_overlap(False)
        for _ in range(warmup):
            tree.run(w.order, mom, w.p, prec, outputs, phi, fld)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            tree.run(w.order, mom, w.p, prec, outputs, phi, fld)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return dt / steps, (phi, fld)

    def kernel_pass(prec, steps):
        """per-kernel durations: the same steps with every launch bracketed by
        HIP events on its own stream, kernels serialised so that each is timed
        alone"""
        phi = torch.empty(w.n, dtype=torch.float64, device=dev) if outputs & fmm.FMM_POT else None
        fld = torch.empty((w.n, 3), dtype=torch.float64, device=dev)
        ctx.set_overlap(False)
        ctx.profile_reset()
        ctx.profile(True)
        for _ in range(steps):
            tree.upward(w.order, mom, w.p, prec)
            tree.evaluate(outputs, phi, fld)
        torch.cuda.synchronize()
        ctx.profile(False)
        return ctx.profile_read(), tree.work_counts()

    res = {}
    for name, prec in (("mixed", fmm.FMM_PREC_MIXED), ("fp64", fmm.FMM_PREC_FP64)):
        step_s, out = run(prec, args.steps, args.warmup)
        prof, work = kernel_pass(prec, args.steps)
        res[name] = dict(step_s=step_s, prof=prof, out=(None if out[0] is None else out[0].cpu().numpy(),
                                                         out[1].cpu().numpy()), work=work)
    grad_line = None
    if bh or w.p - w.order >= 2:
        # the field gradient after the timed steps' upward state (MIXED)
        grd = torch.empty((w.n, 6), dtype=torch.float64, device=dev)
        tree.run(w.order, mom, w.p, fmm.FMM_PREC_MIXED, outputs)
        for _ in range(args.warmup):
            tree.evaluate_grad(fmm.FMM_GRAD, None, None, grd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            tree.evaluate_grad(fmm.FMM_GRAD, None, None, grd)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        what = ("fmm_evaluate_grad(FMM_GRAD) after the MIXED upward pass: the traversal kernel's gradient "
                "variant (M2P second derivatives, pair gradients)" if bh else
                "fmm_evaluate_grad(FMM_GRAD) after the MIXED upward pass: far field again plus a "
                "near-field gradient pass")
        grad_line = {"ms_per_call": dt * 1e3, "unit": "evals/s", "value": w.n / dt, "what": what,
                     "out": grd.cpu().numpy()}
    bh_half = None
    if bh:
        # the same particles at theta_BH = 0.3, half the literal opening angle:
        # the setting whose error matches the FMM's at theta 0.6
        t2 = fmm.Tree(ctx, pos, w.ncrit, 0.3, fmm.FMM_METHOD_BH)
        hphi = torch.empty(w.n, dtype=torch.float64, device=dev) if outputs & fmm.FMM_POT else None
        hfld = torch.empty((w.n, 3), dtype=torch.float64, device=dev)
        for _ in range(args.warmup):
            t2.run(w.order, mom, w.p, fmm.FMM_PREC_MIXED, outputs, hphi, hfld)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            t2.run(w.order, mom, w.p, fmm.FMM_PREC_MIXED, outputs, hphi, hfld)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        bh_half = {"theta": 0.3, "value": w.n / dt, "unit": "evals/s", "ms_per_step": dt * 1e3,
                   "out": hfld.cpu().numpy()}
        t2.close()
    mixed_line = None
    if not bh and args.config == 2:
        # the same particles carrying a charge, a dipole and a quadrupole each
        # (order code MIXED | 7: expansions from order 0, three near-field sums)
        mrng = np.random.default_rng(20052)
        mmom_np = W.mixed_moments(mrng, 7, w.n)
        mmom = torch.from_numpy(mmom_np).to(dev)
        code = fmm.FMM_MIXED + 7
        mphi = torch.empty(w.n, dtype=torch.float64, device=dev)
        mfld = torch.empty((w.n, 3), dtype=torch.float64, device=dev)
        for _ in range(args.warmup):
            tree.run(code, mmom, w.p, fmm.FMM_PREC_MIXED, outputs, mphi, mfld)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            tree.run(code, mmom, w.p, fmm.FMM_PREC_MIXED, outputs, mphi, mfld)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        mixed_line = {"what": "charge + dipole + quadrupole on every particle (order code MIXED | 7), same tree, "
                              "p %d, MIXED precision" % w.p,
                      "value": w.n / dt, "unit": "evals/s", "ms_per_step": dt * 1e3,
                      "moments": mmom_np, "out": (mphi.cpu().numpy(), mfld.cpu().numpy())}
    full_basis = None
    if not bh:
        # the same MIXED steps with the M2L contracting every Cartesian component
        ctx.set_m2l_basis(fmm.FMM_M2L_FULL)
        step_s, _ = run(fmm.FMM_PREC_MIXED, args.steps, args.warmup)
        prof, work = kernel_pass(fmm.FMM_PREC_MIXED, args.steps)
        ctx.set_m2l_basis(fmm.FMM_M2L_HARMONIC)
        k_ms = prof["m2l"][0] / max(1, prof["m2l"][1])
        full_basis = {"value": w.n / step_s, "unit": "evals/s", "ms_per_step": step_s * 1e3,
                      "m2l_avg_launch_ms": k_ms, "m2l_flops_per_launch": work["m2l_flops"],
                      "m2l_achieved_tflops": work["m2l_flops"] / (k_ms * 1e-3) / 1e12 if k_ms > 0 else None}

    def kavg(prof, k):
        v = prof.get(k)
        return v[0] / max(1, v[1]) if v else float("nan")

    m, f64 = res["mixed"], res["fp64"]
    kern_ms = {k: v[0] / max(1, v[1]) for k, v in m["prof"].items()}
    if bh:
        # dominant (and only) evaluation kernel: the traversal with M2P and direct sums
        k_ms = kavg(m["prof"], "bh")
        flops = m["work"]["m2p_flops"] + m["work"]["p2p_flops"]
        achieved = flops / (k_ms * 1e-3) if k_ms > 0 else None
        roofline = {"bound": "alu", "kernel": "bh traversal + M2P + P2P (FP32)",
                    "achieved": achieved / 1e12 if achieved else None, "peak": PEAK_FP32_VALU / 1e12,
                    "unit": "TFLOP/s", "frac": (achieved / PEAK_FP32_VALU) if achieved else None,
                    "traffic": _traffic("bh_c%d_mixed" % args.config), "flops_per_launch": flops,
                    "avg_launch_ms": k_ms, "m2p_pairs": m["work"]["m2p_pairs"], "p2p_pairs": m["work"]["p2p_pairs"]}
        f64_ms = kavg(f64["prof"], "bh")
        f64_flops = f64["work"]["m2p_flops"] + f64["work"]["p2p_flops"]
        f64_k = {"bh_avg_launch_ms": f64_ms,
                 "bh_achieved_tflops": f64_flops / (f64_ms * 1e-3) / 1e12 if f64_ms > 0 else None}
    else:
        # dominant kernel: M2L (FP32 VALU contraction)
        m2l_ms, p2p_ms = kavg(m["prof"], "m2l"), kavg(m["prof"], "p2p")
        m2l_flops = m["work"]["m2l_flops"]
        achieved = m2l_flops / (m2l_ms * 1e-3) if m2l_ms > 0 else None
        roofline = {"bound": "alu", "kernel": "m2l (FP32, harmonic basis)",
                    "achieved": achieved / 1e12 if achieved else None,
                    "peak": PEAK_FP32_VALU / 1e12, "unit": "TFLOP/s",
                    "frac": (achieved / PEAK_FP32_VALU) if achieved else None,
                    "traffic": _traffic("m2l_c%d_mixed" % args.config),
                    "flops_per_launch": m2l_flops, "avg_launch_ms": m2l_ms,
                    "p2p": {"achieved": m["work"]["p2p_flops"] / (p2p_ms * 1e-3) / 1e12 if p2p_ms > 0 else None,
                            "avg_launch_ms": p2p_ms, "flops_per_launch": m["work"]["p2p_flops"]}}
        f64_ms = kavg(f64["prof"], "m2l")
        f64_k = {"m2l_avg_launch_ms": f64_ms,
                 "m2l_achieved_tflops": f64["work"]["m2l_flops"] / (f64_ms * 1e-3) / 1e12 if f64_ms > 0 else None,
                 "m2l_frac_fp64_peak": (f64["work"]["m2l_flops"] / (f64_ms * 1e-3) / PEAK_FP64_VALU) if f64_ms > 0 else None}
    value = w.n / m["step_s"]
    evals = "field" if w.outputs == "field" else "pot+field"
    line = {
        "metric": "FMM particle evals/sec (%s), FP32-bulk (MIXED); FP64 GPU path reported beside it" % evals
                  if not bh else "Barnes-Hut particle evals/sec (%s), FP32-bulk (MIXED); FP64 beside it" % evals,
        "value": value, "unit": "evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": m["step_s"] * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (M2L, P2P) + f64 (P2M, M2M, L2L, L2P)" if not bh else "f32 (M2P, P2P) + f64 (P2M, M2M)",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "source_order": w.order, "p": w.p, "theta": w.theta,
                   "ncrit": w.ncrit, "outputs": w.outputs,
                   "method": "FMM (dual-tree lists)" if not bh else "Barnes-Hut (per-particle traversal, M2P)",
                   "basis": "harmonic (M2L / M2P on the folded rows)"},
        "fp64": {"value": w.n / f64["step_s"], "unit": "evals/s", "ms_per_step": f64["step_s"] * 1e3, **f64_k},
        **({} if bh else {"m2l_full_basis": full_basis}),
        **({} if grad_line is None else {"field_gradient": {k: v for k, v in grad_line.items() if k != "out"}}),
        **({} if bh_half is None else {"bh_theta_0.3": {k: v for k, v in bh_half.items() if k != "out"}}),
        **({} if mixed_line is None else
           {"mixed_sources": {k: v for k, v in mixed_line.items() if k not in ("out", "moments")}}),
        "kernel_timing": "separate pass of the same steps, kernels serialised, HIP events on the launch stream",
        "kernel_avg_ms_mixed": kern_ms,
        "kernel_avg_ms_fp64": {k: v[0] / max(1, v[1]) for k, v in f64["prof"].items()},
        "tree": {"build_ms": t_build * 1e3, **info},
        "roofline": roofline,
    }

    if not args.no_cpu:
        import oracle
        oracle.lib()
        cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
        t0 = time.perf_counter()
        ot = oracle.Tree(w.pos, w.ncrit, None if bh else w.theta)
        tb = time.perf_counter() - t0
        sample = w.sample if w.sample is not None else np.arange(w.n)
        full = w.n <= 200_000
        # the same evaluation repeated until at least 10 s of CPU work has run
        full = full and not bh
        reps = 0
        t0 = time.perf_counter()
        while True:
            if bh:
                po_s, Eo_s = ot.bh(w.order, w.moments, w.p, w.theta, targets=sample)
            elif full:
                po, Eo = ot.fmm(w.order, w.moments, w.p)
                po_s, Eo_s = (po[sample] if po is not None else None), Eo[sample]
            else:
                po_s, Eo_s = ot.fmm(w.order, w.moments, w.p, targets=sample)
            reps += 1
            tc = time.perf_counter() - t0
            if tc >= 10.0:
                break
        nev = (w.n if full else len(sample)) * reps
        kind = "Barnes-Hut" if bh else "FMM"
        line["cpu_baseline"] = {"value": nev / tc, "unit": "evals/s", "cores": cores, "kind": "oracle",
                                "sample": ("full workload, upward+evaluate of the plain FP64 C oracle, repeated "
                                           "%d times (tree build %.2f s excluded)" % (reps, tb)) if full else
                                          ("%d sampled targets of the workload, plain FP64 C oracle %s (full upward "
                                           "pass), repeated %d times (tree build %.2f s excluded)"
                                           % (len(sample), kind, reps, tb)),
                                "seconds": tc}
        pd, Ed = oracle.direct(w.pos, w.order, w.moments, targets=sample)

        def per_particle(a, b):
            """median / p99 / max over targets of |a - b| / |b| (vector norm
            for E), the distribution behind the pooled L2 figure"""
            num = np.linalg.norm(np.reshape(a - b, (len(b), -1)), axis=1)
            den = np.linalg.norm(np.reshape(b, (len(b), -1)), axis=1)
            r = num / np.where(den > 0, den, 1.0)
            return {"median": float(np.median(r)), "p99": float(np.percentile(r, 99)), "max": float(r.max())}

        errs = {}
        for name in ("mixed", "fp64"):
            ph, E = res[name]["out"]
            e = {"E_vs_direct": oracle.rel_l2(E[sample], Ed), "E_vs_oracle": oracle.rel_l2(E[sample], Eo_s),
                 "E_per_particle_vs_direct": per_particle(E[sample], Ed),
                 "E_per_particle_vs_oracle": per_particle(E[sample], Eo_s)}
            if ph is not None:
                e["phi_vs_direct"] = oracle.rel_l2(ph[sample], pd)
                e["phi_vs_oracle"] = oracle.rel_l2(ph[sample], po_s)
            errs[name] = e
        errs["targets"] = ("%d sampled targets, direct O(N) sum per target in FP64; oracle = CPU %s; per-particle "
                           "figures: median, 99th percentile and maximum of the relative error of one target"
                           % (len(sample), kind))
        line["rel_l2_error"] = errs
        if bh_half is not None:
            hEo = oracle.Tree(w.pos, w.ncrit).bh(w.order, w.moments, w.p, 0.3, targets=sample)[1]
            line["bh_theta_0.3"]["E_vs_direct"] = oracle.rel_l2(bh_half["out"][sample], Ed)
            line["bh_theta_0.3"]["E_vs_oracle"] = oracle.rel_l2(bh_half["out"][sample], hEo)
        if mixed_line is not None:
            code = oracle.MIXED + 7
            mpo, mEo = ot.fmm(code, mixed_line["moments"], w.p, targets=sample)
            mph, mE = mixed_line["out"]
            line["mixed_sources"]["phi_vs_oracle"] = oracle.rel_l2(mph[sample], mpo)
            line["mixed_sources"]["E_vs_oracle"] = oracle.rel_l2(mE[sample], mEo)
        if grad_line is not None:
            Go = (ot.bh(w.order, w.moments, w.p, w.theta, targets=sample, want_grad=True) if bh else
                  ot.fmm(w.order, w.moments, w.p, targets=sample, want_grad=True))[2]
            Gd = oracle.direct_grad(w.pos, w.order, w.moments, targets=sample)
            line["field_gradient"]["G_vs_oracle"] = oracle.rel_l2(grad_line["out"][sample], Go)
            line["field_gradient"]["G_vs_direct"] = oracle.rel_l2(grad_line["out"][sample], Gd)
        if not args.no_accuracy and not bh and args.config == 2:
            line["at_1e-6"] = accuracy_run(fmm, torch, w, pos, mom, outputs, ctx, args, dev, sample, pd, Ed)
    if not args.no_serve:
        line["serving"] = serve_bench(fmm, W, torch, n_requests=args.serve_requests)
    print(json.dumps(line), flush=True)
    tree.close()
    ctx.close()


if __name__ == "__main__":
    main()
