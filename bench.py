"""Benchmark of the MI355X Cartesian FMM (one JSON line on stdout).

Default workload: 100,000 point dipoles uniform in the unit cube, ncrit 64,
potential + field, at the accuracy the metric is quoted at: a relative error
of at most 1e-6 against the direct sum.  With the half-side cell radius the
literal parameters of this workload (theta 0.5, p 8) give 1.8e-4 (phi) and
1e-5 (E); the smallest point of the sweep theta in {0.5, 0.4, 0.3}, p in
{6, 8, 10} below 1e-6 for both is theta 0.3, p 10, which is timed as the
headline (--literal times theta 0.5, p 8 instead; the literal row is always
reported beside it).  One step = upward pass + evaluation (P2M, M2M, M2L,
L2L, L2P, P2P) with the octree and interaction lists resident, as the metric
counts particle evaluations per second of N / (t_upward + t_evaluate); the
tree build (set-up, excluded by the paper's own timings) is reported
separately.  The headline precision is MIXED (FP32 M2L/P2P, FP64 elsewhere);
the plain FP64 GPU path is timed on the same tree and reported beside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 2] [--literal] [--no-cpu]
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


KERNEL_SOURCES = {
    "m2l": ("paper_2005_12351_amd/csrc/gen_m2l.py", "paper_2005_12351_amd/csrc/m2l.hip",
            "paper_2005_12351_amd/csrc/tree_host.cpp", "paper_2005_12351_amd/csrc/tree_gpu.hip"),
    "p2p": ("paper_2005_12351_amd/csrc/p2p_kernel.h", "paper_2005_12351_amd/csrc/pair_kernels.h",
            "paper_2005_12351_amd/csrc/fmm_capi.cpp"),
}


def _src_hash(kernel="m2l"):
    """hash of the sources that decide a kernel's memory traffic"""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(kernel, KERNEL_SOURCES["m2l"]):
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
        if e and e.get("src_hash") == _src_hash(kernel_key.split("_")[0]):
            return e.get("bytes_per_launch")
    except Exception:
        return None
    return None


def _progress(msg):
    """a progress line on stderr (the JSON line alone goes to stdout)"""
    print(f"bench.py: {msg}", file=sys.stderr, flush=True)


def serve_bench(fmm, W, torch, n_requests=512, slots=4, budget=2 << 30):
    """Serving workload: requests with N log-uniform in [1e3, 2e5], source
    order in {0,1,2}, p in {4,6,8}, uniform or Plummer positions, theta 0.5,
    ncrit 64, mixed precision.  A closed-loop pass (all submitted at once)
    measures the saturated request rate; the timed open-loop pass replays the
    Poisson arrivals at 0.7 times that rate, a second one at a fixed 130
    requests/s.  Latency = done - arrival.  Four slots: one per hardware
    queue of the process."""
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

    def open_loop(lam):
        """the Poisson arrivals of the stream replayed at rate lam"""
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
        return times, phases, stats

    # open loop at 0.7 x saturated rate
    lam = 0.7 * sat_rate
    times, phases, stats = open_loop(lam)
    lat = np.array([x["done"] - x["submit"] for x in times])
    span = max(x["done"] for x in times) - min(x["submit"] for x in times)
    nsum = sum(d[0].n for d in dev)
    # and at a fixed rate, the same for every build of the library
    fixed = 130.0
    ft, _, _ = open_loop(fixed)
    flat = np.array([x["done"] - x["submit"] for x in ft])
    return {"requests": n_requests, "slots": slots, "budget_bytes": budget, "lambda_req_per_s": lam,
            "saturated_req_per_s": sat_rate, "p50_latency_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_latency_ms": float(np.percentile(lat, 99) * 1e3), "mean_latency_ms": float(lat.mean() * 1e3),
            "throughput_evals_per_s": nsum / span, "peak_running": stats["peak_running"],
            "peak_admitted_bytes": stats["peak_in_use"], "total_particles": nsum,
            "mean_phase_ms": {"queued": float(np.mean([x["admit"] - x["submit"] for x in times]) * 1e3),
                              "tree_build": float(np.mean([p["built"] - x["admit"] for x, p in zip(times, phases)]) * 1e3),
                              "upward_evaluate": float(np.mean([p["computed"] - p["built"] for p in phases]) * 1e3),
                              "release": float(np.mean([x["done"] - p["computed"] for x, p in zip(times, phases)]) * 1e3)},
            "fixed_rate": {"lambda_req_per_s": fixed, "p50_latency_ms": float(np.percentile(flat, 50) * 1e3),
                           "p99_latency_ms": float(np.percentile(flat, 99) * 1e3),
                           "mean_latency_ms": float(flat.mean() * 1e3)},
            "note": "latency = done - arrival; it includes the tree build of each request"}


# (theta, p) of the sweep point the headline is timed at, per workload: the
# smallest of theta in {0.5, 0.4, 0.3}, p in {6, 8, 10} whose error against
# the direct sum is below 1e-6 for phi and E (measured: 3.9e-7 / 1.8e-7)
HEADLINE = {2: (0.3, 10)}


def overlap_mode(fmm, args):
    """the near-field overlap of the timed fmm_run steps"""
    return {"off": fmm.FMM_OVERLAP_OFF, "whole": fmm.FMM_OVERLAP_WHOLE, "split": fmm.FMM_OVERLAP_SPLIT,
            "tail": fmm.FMM_OVERLAP_TAIL}[args.overlap]


def literal_run(fmm, torch, w, pos, mom, outputs, ctx, args, dev, theta, p):
    """The same particles at the workload's literal (theta, p), MIXED and
    FP64 (harmonic basis), reported beside the headline with their errors
    (filled in by the CPU leg)."""
    tree = fmm.Tree(ctx, pos, w.ncrit, theta)
    phi = torch.empty(w.n, dtype=torch.float64, device=dev)
    fld = torch.empty((w.n, 3), dtype=torch.float64, device=dev)
    out = {"theta": theta, "p": p, "info": tree.info()}
    for name, prec in (("mixed", fmm.FMM_PREC_MIXED), ("fp64", fmm.FMM_PREC_FP64)):
        ctx.set_overlap(overlap_mode(fmm, args))
        for _ in range(max(3, args.warmup)):
            tree.run(w.order, mom, p, prec, outputs, phi, fld)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            tree.run(w.order, mom, p, prec, outputs, phi, fld)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        out[name] = {"value": w.n / dt, "unit": "evals/s", "ms_per_step": dt * 1e3,
                     "_out": (phi.cpu().numpy(), fld.cpu().numpy())}
    tree.close()
    return out


def cpu_baseline(args, w, theta, p, method):
    """The oracle on the host cores, all of them and one, with pinned OpenMP
    threads (close placement on cores, active waiting, as the paper's timing
    protocol), each the median of repeated runs on a bounded sample."""
    import subprocess
    cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    res = {}
    for label, nt, frac, runs in (("all", cores, 16, 10), ("one", 1, 128, 10)):
        env = dict(os.environ, OMP_NUM_THREADS=str(nt), OMP_PROC_BIND="close", OMP_PLACES="cores",
                   OMP_WAIT_POLICY="active")
        cmd = [sys.executable, "-m", "oracle.timing", "--config", str(args.config), "--theta", repr(theta),
               "--p", str(p), "--leaf-fraction", str(frac), "--runs", str(runs), "--method", method]
        r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True)
        if r.returncode != 0:
            res[label] = {"error": r.stderr[-500:]}
            continue
        res[label] = json.loads(r.stdout.strip().splitlines()[-1])
    return res


def tree_builds(fmm, torch, w, pos, k, method):
    """K builds of the workload's tree on one context (the first grows its
    arena and loads the sort kernels), with the context's host phases"""
    ctx = fmm.Context(0)
    ts = []
    for i in range(k + 1):
        ctx.profile(True)
        ctx.profile_reset()
        t0 = time.perf_counter()
        tree = fmm.Tree(ctx, pos, w.ncrit, w.theta, method)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
        phases = {n: v[0] for n, v in ctx.profile_read().items() if n.startswith("host:")}
        info = tree.info()
        tree.close()
    ctx.close()
    print(json.dumps({"tree_build_ms": float(np.median(ts[1:])) * 1e3, "first_build_ms": ts[0] * 1e3, "builds": k,
                      "n": w.n, "theta": w.theta, "ncrit": w.ncrit, "last_build_phases_ms": phases, "tree": info}),
          flush=True)


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
    ap.add_argument("--literal", action="store_true",
                    help="time the workload's literal (theta, p) as the headline instead of the 1e-6 point")
    ap.add_argument("--theta", type=float, default=None, help="override the opening angle")
    ap.add_argument("--p", type=int, default=None, help="override the expansion order")
    ap.add_argument("--no-literal-row", action="store_true", help="skip the literal-parameter row")
    ap.add_argument("--serve-slots", type=int, default=None, help="worker slots of the serving pass")
    ap.add_argument("--overlap", choices=["off", "whole", "split", "tail"], default="tail",
                    help="near field beside the far field in the timed steps (default tail: after the M2L, beside the combine and L2L)")
    ap.add_argument("--m2l-engine", choices=["auto", "mfma", "valu"], default="auto",
                    help="units of the FP32 harmonic-basis M2L (auto: matrix cores for p >= 8)")
    ap.add_argument("--tree-builds", type=int, default=0, metavar="K",
                    help="only time K tree builds of the workload's particles (one JSON line; no FMM steps)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only (no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2005_12351_amd import fmm, workloads as W

    bh = args.method == "bh"
    w = W.config(args.config, n_override=args.n or None)
    literal = (w.theta, w.p)
    if args.theta is not None or args.p is not None:
        w.theta = w.theta if args.theta is None else args.theta
        w.p = w.p if args.p is None else args.p
    elif not args.literal and not bh and args.config in HEADLINE:
        w.theta, w.p = HEADLINE[args.config]
    at_literal = (w.theta, w.p) == literal
    dev = torch.device("cuda", 0)
    pos = torch.from_numpy(w.pos).to(dev)
    mom = torch.from_numpy(w.moments).to(dev)
    outputs = fmm.FMM_FIELD if w.outputs == "field" else (fmm.FMM_POT | fmm.FMM_FIELD)
    if args.tree_builds:
        tree_builds(fmm, torch, w, pos, args.tree_builds, fmm.FMM_METHOD_BH if bh else fmm.FMM_METHOD_FMM)
        return
    ctx = fmm.Context(0)
    # device work of this script runs on the context's stream, so the
    # binding has no cross-stream ordering to add around each call
    torch.cuda.set_stream(ctx.stream)
    ctx.set_m2l_engine({"auto": fmm.FMM_M2L_ENGINE_AUTO, "mfma": fmm.FMM_M2L_ENGINE_MFMA,
                        "valu": fmm.FMM_M2L_ENGINE_VALU}[args.m2l_engine])
    if args.calibrate_copy:
        a_ = torch.ones(args.calibrate_copy << 18, dtype=torch.float32, device=dev)
        b_ = torch.empty_like(a_)
        torch.cuda.synchronize()
        b_.copy_(a_)
        torch.cuda.synchronize()
        del a_, b_

    # the first build also loads the sort kernels and grows the context's
    # arena; the figure is the median of the next five
    method = fmm.FMM_METHOD_BH if bh else fmm.FMM_METHOD_FMM
    t0 = time.perf_counter()
    tree = fmm.Tree(ctx, pos, w.ncrit, w.theta, method)
    torch.cuda.synchronize()
    t_first = time.perf_counter() - t0
    tb = []
    for _ in range(5):
        tree.close()
        t0 = time.perf_counter()
        tree = fmm.Tree(ctx, pos, w.ncrit, w.theta, method)
        torch.cuda.synchronize()
        tb.append(time.perf_counter() - t0)
    t_build = float(np.median(tb))
    info = tree.info()

    def run(prec, steps, warmup):
        """the timed region: each step is fmm_run (upward + evaluate as one
        captured graph, replayed, on one stream), no per-kernel events"""
        phi = torch.empty(w.n, dtype=torch.float64, device=dev) if outputs & fmm.FMM_POT else None
        fld = torch.empty((w.n, 3), dtype=torch.float64, device=dev)
        ctx.profile(False)
        ctx.set_overlap(overlap_mode(fmm, args))
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

    _progress("timed steps done")
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
        # dominant kernel: the longer of M2L and P2P per step (kernels timed
        # alone, HIP events on their launch stream); both are reported
        def kern(name, flops_key, what):
            ms = kavg(m["prof"], name)
            per_step = m["prof"][name][0] / max(1, args.steps) if name in m["prof"] else 0.0
            fl = m["work"][flops_key]
            ach = fl / (ms * 1e-3) if ms > 0 else None
            return {"bound": "alu", "kernel": what, "achieved": ach / 1e12 if ach else None,
                    "peak": PEAK_FP32_VALU / 1e12, "unit": "TFLOP/s",
                    "frac": (ach / PEAK_FP32_VALU) if ach else None,
                    "traffic": _traffic("%s_c%d_mixed_p%d_t%g" % (name, args.config, w.p, w.theta)),
                    "flops_per_launch": fl, "avg_launch_ms": ms, "ms_per_step": per_step,
                    "frac_of_nonpacked_issue": (ach / (PEAK_FP32_VALU / 2)) if ach else None}
        k_m2l = kern("m2l", "m2l_flops", "m2l (FP32, harmonic basis): 2 flops per multiply-add of the reduced "
                                         "contraction per list entry")
        k_p2p = kern("p2p", "p2p_flops", "p2p (FP32 + Kahan): per (i, j) pair, phi+E closed form")
        dom, other = (k_m2l, k_p2p) if k_m2l["ms_per_step"] >= k_p2p["ms_per_step"] else (k_p2p, k_m2l)
        roofline = dict(dom)
        roofline["other"] = other
        roofline["note"] = ("peak = MI355X FP32 vector 157.3 TFLOP/s (packed); the kernels are built without "
                            "packed FP32, whose issue ceiling is 78.6 TFLOP/s (frac_of_nonpacked_issue)")
        f64_ms = kavg(f64["prof"], "m2l")
        f64_k = {"m2l_avg_launch_ms": f64_ms,
                 "m2l_achieved_tflops": f64["work"]["m2l_flops"] / (f64_ms * 1e-3) / 1e12 if f64_ms > 0 else None,
                 "m2l_frac_fp64_peak": (f64["work"]["m2l_flops"] / (f64_ms * 1e-3) / PEAK_FP64_VALU) if f64_ms > 0 else None}
    value = w.n / m["step_s"]
    evals = "field" if w.outputs == "field" else "pot+field"
    line = {
        "metric": ("FMM particle evals/sec (%s) at rel err 1e-6, FP32 (MIXED) vs FP64; p50/p99 latency" % evals
                   if not at_literal else
                   "FMM particle evals/sec (%s), FP32-bulk (MIXED); FP64 GPU path reported beside it" % evals)
                  if not bh else "Barnes-Hut particle evals/sec (%s), FP32-bulk (MIXED); FP64 beside it" % evals,
        "value": value, "unit": "evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": m["step_s"] * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (M2L, P2P) + f64 (P2M, M2M, L2L, L2P)" if not bh else "f32 (M2P, P2P) + f64 (P2M, M2M)",
        "data": "synthetic",
        "config": {"workload": w.name if at_literal else
                   "%s at theta %g, p %d (smallest sweep point below 1e-6 against the direct sum; literal "
                   "theta %g, p %d reported as literal_parameters)" % (w.name.split(":")[0] + ": %d dipoles "
                   "uniform in the unit cube" % w.n, w.theta, w.p, literal[0], literal[1]),
                   "n": w.n, "source_order": w.order, "p": w.p, "theta": w.theta,
                   "ncrit": w.ncrit, "outputs": w.outputs,
                   "method": "FMM (dual-tree lists)" if not bh else "Barnes-Hut (per-particle traversal, M2P)",
                   "basis": "harmonic (M2L / M2P on the folded rows)",
                   "near_field_overlap": args.overlap,
                   "m2l_engine": ("matrix cores (v_mfma_f32_4x4x1)" if args.m2l_engine == "mfma" or
                                  (args.m2l_engine == "auto" and w.p >= 8) else "vector units")},
        "fp64": {"value": w.n / f64["step_s"], "unit": "evals/s", "ms_per_step": f64["step_s"] * 1e3, **f64_k},
        **({} if bh else {"m2l_full_basis": full_basis}),
        **({} if grad_line is None else {"field_gradient": {k: v for k, v in grad_line.items() if k != "out"}}),
        **({} if bh_half is None else {"bh_theta_0.3": {k: v for k, v in bh_half.items() if k != "out"}}),
        **({} if mixed_line is None else
           {"mixed_sources": {k: v for k, v in mixed_line.items() if k not in ("out", "moments")}}),
        "kernel_timing": "separate pass of the same steps, kernels serialised, HIP events on the launch stream",
        "kernel_avg_ms_mixed": kern_ms,
        "kernel_avg_ms_fp64": {k: v[0] / max(1, v[1]) for k, v in f64["prof"].items()},
        "tree": {"build_ms": t_build * 1e3, "first_build_ms": t_first * 1e3, **info},
        "roofline": roofline,
    }

    lit = None
    if not bh and not at_literal and not args.no_literal_row:
        lit = literal_run(fmm, torch, w, pos, mom, outputs, ctx, args, dev, literal[0], literal[1])
        _progress("literal-parameter row done")
    if not args.no_cpu:
        import oracle
        oracle.lib()
        ot = oracle.Tree(w.pos, w.ncrit, None if bh else w.theta)
        sample = w.sample if w.sample is not None else np.arange(w.n)
        kind = "Barnes-Hut" if bh else "FMM"
        if bh:
            po_s, Eo_s = ot.bh(w.order, w.moments, w.p, w.theta, targets=sample)
        else:
            po_s, Eo_s = ot.fmm(w.order, w.moments, w.p, targets=sample)
        _progress("CPU baseline (oracle on a bounded sample)")
        cb = cpu_baseline(args, w, w.theta, w.p, "bh" if bh else "fmm")
        _progress("CPU baseline done; error checks against the oracle")
        allc, one = cb.get("all", {}), cb.get("one", {})
        if "median_s" in allc:
            line["cpu_baseline"] = {
                "value": allc["targets"] / allc["median_s"], "unit": "evals/s", "cores": allc["threads"],
                "kind": "oracle",
                "sample": ("plain FP64 C oracle %s at theta %g, p %d: every particle of %d of the %d leaves "
                           "(%d targets), each run a full upward pass plus the far and near field of those "
                           "targets; median of %d runs, OpenMP threads pinned close on cores, active wait"
                           % (kind, w.theta, w.p, allc["leaves"], allc["leaves_total"], allc["targets"],
                              len(allc["seconds"]))),
                "median_s": allc["median_s"],
                "one_core": ({"value": one["targets"] / one["median_s"], "unit": "evals/s", "cores": 1,
                              "targets": one["targets"], "median_s": one["median_s"], "runs": len(one["seconds"])}
                             if "median_s" in one else one)}
        else:
            line["cpu_baseline"] = {"value": None, "unit": "evals/s", "cores": None, "kind": "oracle",
                                    "sample": "timing failed", "error": allc.get("error")}
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
        if lit is not None:
            lo = oracle.Tree(w.pos, w.ncrit, lit["theta"]).fmm(w.order, w.moments, lit["p"], targets=sample)
            for name in ("mixed", "fp64"):
                ph, E = lit[name].pop("_out")
                lit[name].update({"phi_vs_direct": oracle.rel_l2(ph[sample], pd),
                                  "E_vs_direct": oracle.rel_l2(E[sample], Ed),
                                  "phi_vs_oracle": oracle.rel_l2(ph[sample], lo[0]),
                                  "E_vs_oracle": oracle.rel_l2(E[sample], lo[1])})
    if lit is not None:
        for name in ("mixed", "fp64"):
            lit[name].pop("_out", None)
        line["literal_parameters"] = lit
    if not args.no_serve:
        kw = {} if args.serve_slots is None else {"slots": args.serve_slots}
        _progress("serving stream")
        line["serving"] = serve_bench(fmm, W, torch, n_requests=args.serve_requests, **kw)
        _progress("serving done")
    print(json.dumps(line), flush=True)
    tree.close()
    ctx.close()


if __name__ == "__main__":
    main()
