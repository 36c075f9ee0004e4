"""Benchmark of the Domain Transform Solver hot path on one MI355X.

Workload: the 10240 x 10240, 16-band multispectral solve (1-channel target, confidence 1,
sigma_s = 32, sigma_r = 0.15, 3 filter iterations, 10 solver iterations) on seeded
synthetic inputs already resident in HBM.  One step = one full dts_solve (distances,
weights, 2 x 3 x 10 recursive passes and the 10 fused updates).

Prints ONE JSON line: Mpixel/s of the solve, the roofline of the dominant kernel from
HIP events recorded around every launch, and the FP64 CPU oracle timed on a bounded band
of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DTS solve Mpixel/s & % of HBM peak; batched and fwd+bwd vs plain fwd"
HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "solve_10240x10240_hbm_traffic.md")
FWD_BWD_TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "fwd_bwd_8x1024_hbm_traffic.md")


def sources_digest(names=None):
    """SHA-256 over library sources (`names`: file names under csrc/ plus dts.h; None: all
    of them): hardware-counter traffic recorded for one digest is reported only while the
    sources its kernels are built from are unchanged."""
    import hashlib

    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1805_04590_amd", "csrc")
    files = sorted(os.path.join(csrc, f) for f in os.listdir(csrc) if f.endswith((".hip", ".hpp")))
    files += [os.path.join(ROOT, "include", "dts.h")]
    if names is not None:
        files = [f for f in files if os.path.basename(f) in set(names)]
    for path in files:
        h.update(os.path.basename(path).encode())
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(kernel, profile=TRAFFIC_PROFILE):
    """HBM bytes per launch of `kernel` measured with rocprofv3 FETCH_SIZE / WRITE_SIZE
    (scaled by a plain copy of known size), or None when no record matches these sources."""
    import re

    try:
        text = open(profile).read()
    except OSError:
        return None
    m = re.search(r"<!-- traffic: (\{.*?\}) -->", text, flags=re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec.get("sources_sha256") != sources_digest(rec.get("sources")):
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k.get("traffic_bytes")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-rows", type=int, default=512,
                    help="rows of the workload the CPU oracle baseline solves (0 = skip)")
    ap.add_argument("--no-profile", action="store_true", help="skip the per-kernel timing run")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched (64 uneven solves) and forward+backward legs")
    ap.add_argument("--no-graph", action="store_true",
                    help="time the batched leg with direct launches instead of graph replays")
    ap.add_argument("--no-solve", action="store_true",
                    help="skip the single-image solve (for profiling the other legs alone)")
    ap.add_argument("--batched-only", type=int, default=None, metavar="VARIANT",
                    help="profiling mode: only the 64 uneven solves, batched kernel variant VARIANT, "
                         "direct launches, no one-by-one comparison")
    ap.add_argument("--fwd-bwd-only", action="store_true",
                    help="profiling mode: only the 8 x 1024^2 forward + backward leg")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first fill and copy a MIB-sized float32 buffer with torch: kernels of "
                         "known traffic that calibrate the hardware byte counters")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# GPU outputs of the other workloads kept on the host for the CPU leg, which compares them
# with the oracle: {name: (inputs, gpu output)}
SAMPLES = {}
BATCHED_SAMPLE_INSTANCES = (42, 57, 26)  # Cg, Ct = (8, 1), (16, 3), (1, 3): small instances


def host_info():
    """Logical CPUs and the CPU model of this host."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return os.cpu_count(), model


def cpu_baseline(rows):
    """Time the FP64 oracle on a full-width band of the workload (same generator)."""
    import dts_inputs
    import oracle

    case = dts_inputs.multispectral_10240(rows=(0, rows))
    px = case["target"].shape[1] * case["target"].shape[2]
    t0 = time.perf_counter()
    ref = oracle.solve(case["guide"], case["target"], case["conf"], case["sigma_s"], case["sigma_r"],
                       case["filter_iters"], case["solver_iters"], case["lam"], case["step"])
    dt = time.perf_counter() - t0
    err = None
    try:
        import torch

        import paper_1805_04590_amd as dts

        if torch.cuda.is_available():
            g, t, c = (torch.from_numpy(case[k]).cuda() for k in ("guide", "target", "conf"))
            z = dts.solve(g, t, c, case["sigma_s"], case["sigma_r"], case["filter_iters"], case["solver_iters"],
                          case["lam"], case["step"]).cpu().numpy()
            err = float(np.abs(z - ref).max())
            del g, t, c
    except Exception as e:  # the baseline itself stands without the comparison
        log(f"  GPU comparison on the sample skipped: {e}")
    try:
        import threadpoolctl
        threads = max(p.get("num_threads", 1) for p in threadpoolctl.threadpool_info()) or 1
    except Exception:
        threads = 1
    # the other workloads' GPU outputs against the oracle (max abs error over the
    # sample, divided by the signal's value range where it is not 1)
    errs = {}
    for name, (inp, got) in SAMPLES.items():
        ref = oracle.solve(inp["guide"], inp["target"], inp["conf"], inp["sigma_s"], inp["sigma_r"],
                           inp["filter_iters"], inp["solver_iters"])
        errs[name] = float(np.abs(got - ref).max()) / inp.get("value_range", 1.0)
        log(f"  oracle vs GPU, {name}: {errs[name]:.3e}")
    ncpu, model = host_info()
    return dict(value=px / dt / 1e6, unit="Mpixel/s", cores=1, kind="oracle",
                sample=(f"rows 0-{rows} x all {case['target'].shape[2]} columns of the same "
                        f"workload, full solve (T={case['solver_iters']}), FP64 NumPy; "
                        f"{dt:.1f} s; elementwise NumPy runs on one core "
                        f"(BLAS pool {threads} threads unused)"),
                host_logical_cpus=ncpu, host_cpu_model=model,
                gpu_max_abs_err=err, gpu_max_abs_err_by_workload=errs, seconds=dt)


def timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def batched_leg(steps, warmup, graph=True, variant=None, sequential=True):
    """64 uneven solves: one graph-captured persistent launch (graph=False: the launch
    made directly) against the same solves run one by one through dts_solve (workspaces
    preallocated)."""
    import ctypes

    import torch

    import dts_inputs
    import paper_1805_04590_amd as dts

    cases = dts_inputs.uneven_batch_64()
    dev = torch.device("cuda:0")
    probs = [dict(guide=torch.from_numpy(c["guide"]).to(dev), target=torch.from_numpy(c["target"]).to(dev),
                  conf=torch.from_numpy(c["conf"]).to(dev), sigma_s=c["sigma_s"], sigma_r=c["sigma_r"],
                  filter_iters=3, solver_iters=10) for c in cases]
    px = sum(c["target"].shape[1] * c["target"].shape[2] for c in cases)
    bs = dts.BatchedSolver(probs, variant=variant)  # None: autotuned
    ms_b = timed(bs.capture().replay if graph else bs.run, steps, warmup)
    bs.status()
    if not sequential:
        return dict(workload="64 uneven solves 320-1920 x 240-1080, Cg in {1,3,8,16}, Ct 1-3, T=10",
                    pixels=px, variant=bs.variant, launch="hip graph replay" if graph else "direct",
                    batched_ms=round(ms_b, 3), batched_mpix_s=round(px / ms_b / 1e3, 1))
    outs = [torch.empty_like(q["target"]) for q in probs]
    wss = []
    for q in probs:
        Ct, H, W = q["target"].shape
        p = dts.Params(q["sigma_s"], q["sigma_r"], 3, 10).c()
        wss.append(torch.empty(dts.library().dts_solve_workspace_bytes(1, H, W, Ct, ctypes.byref(p)),
                               dtype=torch.uint8, device=dev))

    def seq():
        for q, o, w in zip(probs, outs, wss):
            dts.solve(q["guide"], q["target"], q["conf"], q["sigma_s"], q["sigma_r"], 3, 10,
                      out=o[None], workspace=w)

    ms_s = timed(seq, steps, warmup)
    err = max((o - b).abs().max().item() for o, b in zip(outs, bs.outputs))
    for i in BATCHED_SAMPLE_INSTANCES:
        c = cases[i]
        SAMPLES[f"uneven_batch_64 instance {i} (batched kernel)"] = (
            dict(c, filter_iters=3, solver_iters=10), bs.outputs[i].cpu().numpy())
    return dict(workload="64 uneven solves 320-1920 x 240-1080, Cg in {1,3,8,16}, Ct 1-3, T=10",
                pixels=px, variant=bs.variant, launch="hip graph replay" if graph else "direct", batched_ms=round(ms_b, 3),
                batched_mpix_s=round(px / ms_b / 1e3, 1), sequential_ms=round(ms_s, 3),
                sequential_mpix_s=round(px / ms_s / 1e3, 1), speedup=round(ms_s / ms_b, 3),
                max_abs_diff=err)


def fwd_bwd_leg(steps, warmup):
    """Batch of 8 1024x1024 RGB -> 3-channel solves, T=15: forward with checkpoints alone,
    and forward + hand-written adjoint for the loss sum((z - r)^2)."""
    import ctypes

    import torch

    import dts_inputs
    import paper_1805_04590_amd as dts

    c = dts_inputs.rgb_batch_8x1024()
    dev = torch.device("cuda:0")
    g = torch.from_numpy(c["guide"]).to(dev)
    t = torch.from_numpy(c["target"]).to(dev)
    cf = torch.from_numpy(c["conf"]).to(dev)
    r = torch.from_numpy(c["ref"]).to(dev)
    B, Ct, H, W = t.shape
    T = c["solver_iters"]
    p = dts.Params(c["sigma_s"], c["sigma_r"], 3, T).c()
    ws = torch.empty(dts.library().dts_solve_workspace_bytes(B, H, W, Ct, ctypes.byref(p)),
                     dtype=torch.uint8, device=dev)
    wsb = torch.empty(dts.library().dts_solve_backward_workspace_bytes(B, H, W, g.shape[1], Ct,
                                                                       ctypes.byref(p)),
                      dtype=torch.uint8, device=dev)
    out = torch.empty_like(t)
    state = {}

    def fwd():
        state["z"], state["ck"] = dts.solve(g, t, cf, c["sigma_s"], c["sigma_r"], 3, T,
                                            checkpoints=True, out=out, workspace=ws)

    def fwd_bwd_recompute():
        fwd()
        go = 2.0 * (state["z"] - r)
        dts.solve_backward(g, t, cf, state["ck"], go, c["sigma_s"], c["sigma_r"], 3, T,
                           workspace=wsb)

    # the forward keeps every filter pass's output (2N - 1 signals per iteration) and the
    # backward reads them instead of recomputing them (the tape comes from torch's caching
    # allocator, reused call after call)
    def fwd_bwd():
        res = dts.solve(g, t, cf, c["sigma_s"], c["sigma_r"], 3, T, tape=True, out=out, workspace=ws)
        z, ck, tp = res
        state["z"] = z
        go = 2.0 * (z - r)
        dts.solve_backward(g, t, cf, ck, go, c["sigma_s"], c["sigma_r"], 3, T, workspace=wsb, tape=tp)

    ms_f = timed(fwd, steps, warmup)
    ms_fbr = timed(fwd_bwd_recompute, steps, warmup)
    ms_fb = timed(fwd_bwd, steps, warmup)
    dts.workspace_status(ws)
    dts.workspace_status(wsb)
    SAMPLES["rgb_batch_8x1024 image 0 forward"] = (
        dict(guide=c["guide"][0], target=c["target"][0], conf=c["conf"][0], sigma_s=c["sigma_s"],
             sigma_r=c["sigma_r"], filter_iters=3, solver_iters=T), state["z"][0].cpu().numpy())
    px = B * H * W
    # algorithmic bytes of every launch of one forward + backward, from the library's own
    # per-launch records (forward passes with checkpoints, recomputed passes, adjoint passes)
    kernels, stats = kernel_table(fwd_bwd, 2)
    fb_bytes = sum(s["bytes_per_launch"] * s["launches"] for s in stats.values()) / 2
    kern = {k: dict(launches_per_step=round(v["launches_per_step"], 2), avg_us=round(v["avg_us"], 2),
                    share=round(v["share"], 4), algorithmic_GBps=round(v["algorithmic_GBps"], 1),
                    hbm_frac=round(v["algorithmic_GBps"] / HBM_PEAK_GBPS, 4),
                    traffic=recorded_traffic(k, FWD_BWD_TRAFFIC_PROFILE))
            for k, v in kernels.items()}
    return dict(workload="8 x 1024x1024 RGB -> 3 channels, T=15, loss sum((z-r)^2)", pixels=px,
                fwd_ms=round(ms_f, 3), fwd_mpix_s=round(px / ms_f / 1e3, 1),
                fwd_bwd_ms=round(ms_fb, 3), fwd_bwd_mpix_s=round(px / ms_fb / 1e3, 1),
                fwd_bwd_over_fwd=round(ms_fb / ms_f, 3),
                fwd_bwd_mode=f"pass tape: the forward keeps 2N-1 = 5 pass outputs per iteration "
                             f"({T * 5 * B * Ct * H * W * 4 / 1e9:.2f} GB) for the backward",
                fwd_bwd_recompute_ms=round(ms_fbr, 3),
                fwd_bwd_algorithmic_bytes=fb_bytes,
                algorithmic_GBps=round(fb_bytes / (ms_fb / 1e3) / 1e9, 1),
                hbm_frac=round(fb_bytes / (ms_fb / 1e3) / 1e9 / HBM_PEAK_GBPS, 4),
                kernels=kern)


def kernel_table(step, steps):
    """Per-kernel launches, average duration and algorithmic GB/s over `steps` calls of
    `step`, from the HIP events the library records around each of its launches."""
    import torch

    import paper_1805_04590_amd as dts

    dts.profile_enable(True)
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    stats = dts.profile_read()
    dts.profile_enable(False)
    total = sum(v["total_ms"] for v in stats.values())
    kernels = {}
    for name, s in stats.items():
        kernels[name] = dict(launches_per_step=s["launches"] / steps, avg_us=s["avg_ms"] * 1e3,
                             share=s["total_ms"] / total,
                             algorithmic_GBps=s["bytes_per_launch"] / (s["avg_ms"] / 1e3) / 1e9)
    return kernels, stats


def solve_leg(args, dev):
    """The headline workload: Mpixel/s of dts_solve and, unless --no-profile, the per-kernel
    timing (HIP events around every launch) and the dominant kernel's roofline."""
    import ctypes

    import torch

    import dts_inputs
    import paper_1805_04590_amd as dts

    H, W, Cg = dts_inputs.multispectral_shape()
    t0 = time.time()
    log(f"generating the {W}x{H}x{Cg} workload ...")
    case = dts_inputs.multispectral_10240()
    log(f"  generated in {time.time() - t0:.1f} s; uploading")
    guide = torch.from_numpy(case["guide"]).to(dev)
    target = torch.from_numpy(case["target"]).to(dev)
    conf = torch.from_numpy(case["conf"]).to(dev)
    del case["guide"]
    Ct = target.shape[0]
    T, N = case["solver_iters"], case["filter_iters"]
    ss, sr = case["sigma_s"], case["sigma_r"]
    lib = dts.library()
    p = dts.Params(ss, sr, N, T).c()
    ws = torch.empty(lib.dts_solve_workspace_bytes(1, H, W, Ct, ctypes.byref(p)),
                     dtype=torch.uint8, device=dev)
    out = torch.empty_like(target)
    torch.cuda.synchronize()

    def step():
        dts.solve(guide, target, conf, ss, sr, N, T, out=out[None], workspace=ws)

    log(f"warmup x{args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    dts.workspace_status(ws)
    log(f"timing x{args.steps}")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = e0.elapsed_time(e1) / args.steps
    dts.workspace_status(ws)
    px = H * W
    mpix = px / (ms / 1e3) / 1e6
    solve_bytes = px * (T * (60 * Ct + 24) + 4 * Cg + 4)
    log(f"  {ms:.3f} ms/solve  {mpix:.1f} Mpixel/s  (wall {wall:.2f} s)")

    kernels = {}
    roofline = None
    if not args.no_profile:
        log("per-kernel timing run (HIP events around each launch)")
        kernels, stats = kernel_table(step, args.steps)
        dom = max(stats, key=lambda k: stats[k]["total_ms"])
        s = stats[dom]
        achieved = s["bytes_per_launch"] / (s["avg_ms"] / 1e3) / 1e9
        roofline = dict(bound="hbm", kernel=dom, achieved=round(achieved, 1), peak=HBM_PEAK_GBPS,
                        unit="GB/s", frac=round(achieved / HBM_PEAK_GBPS, 4),
                        traffic=recorded_traffic(dom),
                        bytes_per_launch=s["bytes_per_launch"], avg_us=round(s["avg_ms"] * 1e3, 2))
        # every filter-pass kernel of the solve, and their time-weighted aggregate: the
        # dominant kernel alone does not show the slower ones
        tot_b = sum(v["bytes_per_launch"] * v["launches"] for v in stats.values())
        tot_s = sum(v["total_ms"] for v in stats.values()) / 1e3
        roofline["filter_passes"] = dict(
            achieved=round(tot_b / tot_s / 1e9, 1), frac=round(tot_b / tot_s / 1e9 / HBM_PEAK_GBPS, 4),
            per_kernel={k: dict(avg_us=round(v["avg_ms"] * 1e3, 2),
                                achieved=round(v["bytes_per_launch"] / (v["avg_ms"] / 1e3) / 1e9, 1),
                                frac=round(v["bytes_per_launch"] / (v["avg_ms"] / 1e3) / 1e9 / HBM_PEAK_GBPS, 4),
                                traffic=recorded_traffic(k))
                        for k, v in stats.items()})
        log("  " + json.dumps(kernels))

    # Eq. (7): confidence from the edge-aware variance of the target, same guide
    sc = 0.05
    wsv = torch.empty(lib.dts_variance_confidence_workspace_bytes(1, H, W, Ct), dtype=torch.uint8,
                      device=dev)
    confv = torch.empty_like(target)

    def vstep():
        dts.variance_confidence(guide, target, ss, sr, sc, N, out=confv, workspace=wsv)

    ms_v = timed(vstep, args.steps, args.warmup)
    dts.workspace_status(wsv)
    # first row pass: z in, (z, z^2) out, guide in, dx and dy out; 2N - 2 further passes over
    # the pairs; the last column pass reads the pairs and writes the confidences
    v_bytes = px * (4 * (3 * Ct + Cg + 2) + (2 * N - 2) * 4 * (4 * Ct + 1) + 4 * (3 * Ct + 1))
    variance = dict(workload=f"variance confidence (Eq. 7) of the {W}x{H} target, {Cg}-band guide, "
                             f"sigma_c={sc}, N={N}",
                    ms=round(ms_v, 3), mpix_s=round(px / ms_v / 1e3, 1),
                    algorithmic_GBps=round(v_bytes / (ms_v / 1e3) / 1e9, 1),
                    hbm_frac=round(v_bytes / (ms_v / 1e3) / 1e9 / HBM_PEAK_GBPS, 4))
    log("  variance confidence: " + json.dumps(variance))
    del wsv, confv

    # support of the edge-aware kernel and the support-weighted confidence, same guide
    wss = torch.empty(lib.dts_support_workspace_bytes(1, H, W), dtype=torch.uint8, device=dev)
    sup = torch.empty((1, H, W), dtype=torch.float32, device=dev)
    confs = torch.empty_like(conf)
    Cc = conf.shape[0]

    def sstep():
        dts.support(guide, ss, sr, N, conf=conf, out=sup, conf_out=confs, workspace=wss)

    ms_s = timed(sstep, args.steps, args.warmup)
    dts.workspace_status(wss)
    # distances (guide in, dx and dy out); pass 1: rows of ones (dx in, plane out), columns
    # (plane and dy in, plane out); N - 1 more row and column passes over the support
    # plane; the last column pass also reads and writes the Cc confidence planes
    s_bytes = px * (4 * (Cg + 2) + 8 + 12 + 24 * (N - 1) + 8 * Cc)
    support = dict(workload=f"support and support-weighted confidence of the {W}x{H} "
                            f"{Cg}-band guide, N={N}",
                   ms=round(ms_s, 3), mpix_s=round(px / ms_s / 1e3, 1),
                   algorithmic_GBps=round(s_bytes / (ms_s / 1e3) / 1e9, 1),
                   hbm_frac=round(s_bytes / (ms_s / 1e3) / 1e9 / HBM_PEAK_GBPS, 4))
    if not args.no_profile:
        support["kernels"] = {k: {kk: round(vv, 3) for kk, vv in v.items()}
                              for k, v in kernel_table(sstep, 2)[0].items()}
    log("  support: " + json.dumps(support))
    del wss, sup, confs

    # the box form of the edge-aware mean (Eq. (10) as written) in the same solve
    wsb = torch.empty(lib.dts_box_workspace_bytes(1, H, W, Ct, N), dtype=torch.uint8, device=dev)
    outb = torch.empty_like(target)

    def bstep():
        dts.solve_box(guide, target, conf, ss, sr, N, T, out=outb[None], workspace=wsb)

    ms_b = timed(bstep, args.steps, args.warmup)
    # codes (guide in, two code planes out); row and column bounds (codes in, N bound planes
    # out each); per iteration N row passes (signal and bounds in, signal out), N - 1 column
    # passes (the same) and one column pass with the update (z^k, t and c in as well)
    b_bytes = px * (4 * (Cg + 2) + 2 * (4 + 2 * N)
                    + T * (N * (8 * Ct + 2) + (N - 1) * 10 * Ct + 18 * Ct + 4 * Cc))
    box = dict(workload=f"solve with the box kernel (Eq. 10 as written) on the same {W}x{H} workload, "
                        f"N={N}, T={T}",
               ms=round(ms_b, 3), mpix_s=round(px / ms_b / 1e3, 1),
               algorithmic_GBps=round(b_bytes / (ms_b / 1e3) / 1e9, 1),
               hbm_frac=round(b_bytes / (ms_b / 1e3) / 1e9 / HBM_PEAK_GBPS, 4),
               over_recursive=round(ms_b / ms, 3))
    if not args.no_profile:
        box["kernels"] = {k: {kk: round(vv, 3) for kk, vv in v.items()}
                          for k, v in kernel_table(bstep, 2)[0].items()}
    log("  box: " + json.dumps(box))
    del guide, target, conf, out, ws, wsb, outb
    torch.cuda.empty_cache()
    return dict(ms=ms, mpix=mpix, solve_bytes=solve_bytes, kernels=kernels, roofline=roofline,
                H=H, W=W, Cg=Cg, Ct=Ct, T=T, N=N, ss=ss, sr=sr, variance=variance, support=support, box=box)


def stereo_leg(steps, warmup):
    """Eq. (11) disparity refinement on the 1920x1080 stereo pair (T = 20) against the
    plain solve of the same target and confidence with the left image as guide."""
    import torch

    import dts_inputs
    import paper_1805_04590_amd as dts

    c = dts_inputs.stereo_pair_1920x1080()
    dev = torch.device("cuda:0")
    L = torch.from_numpy(c["left"]).to(dev)
    R = torch.from_numpy(c["right"]).to(dev)
    t = torch.from_numpy(c["target"]).to(dev)
    cf = torch.from_numpy(c["conf"]).to(dev)
    _, H, W = t.shape
    T, ss, sr = c["solver_iters"], c["sigma_s"], c["sigma_r"]
    lib = dts.library()
    wss = torch.empty(lib.dts_solve_stereo_workspace_bytes(1, H, W), dtype=torch.uint8, device=dev)
    import ctypes
    p = dts.Params(ss, sr, 3, T).c()
    wsp = torch.empty(lib.dts_solve_workspace_bytes(1, H, W, 1, ctypes.byref(p)), dtype=torch.uint8, device=dev)
    out = torch.empty_like(t)

    def stereo():
        dts.solve_stereo(L, R, t, cf, ss, sr, 3, T, gamma=c["gamma"], eps=c["eps"], out=out, workspace=wss)

    def plain():
        dts.solve(L, t, cf, ss, sr, 3, T, out=out[None], workspace=wsp)

    ms_s = timed(stereo, steps, warmup)
    dts.workspace_status(wss)
    ms_p = timed(plain, steps, warmup)
    px = H * W
    Cg = L.shape[0]
    # per iteration: data-term gradient (z, t, c, D and both images) + 6 passes + the
    # update's reads of z and D; the distances once
    s_bytes = px * (T * (4 * (4 + 2 * Cg) + 6 * 12 + 8) + 4 * Cg + 8)
    return dict(workload=f"stereo refinement (Eq. 11) {W}x{H} RGB pair, T={T}, gamma={c['gamma']}, "
                         f"eps={c['eps']}", stereo_ms=round(ms_s, 3), stereo_mpix_s=round(px / ms_s / 1e3, 1),
                plain_ms=round(ms_p, 3), stereo_over_plain=round(ms_s / ms_p, 3),
                algorithmic_GBps=round(s_bytes / (ms_s / 1e3) / 1e9, 1))


def sweep_leg(steps, warmup):
    """Scaling checks on the polygon-scene recipe (N = 3, one-channel target): Mpixel/s over
    image sizes 256^2 .. 8192^2 (T = 10), the solve time over sigma_s x sigma_r at 2048^2
    (the recursive filter's cost does not depend on either), and the time against the
    number of solver iterations T at 2048^2 (linear)."""
    import ctypes

    import torch

    import dts_inputs
    import paper_1805_04590_amd as dts

    dev = torch.device("cuda:0")
    lib = dts.library()

    def prepare(n, seed):
        c = dts_inputs.random_case(seed, n, n, 3, 1, sigma_s=8.0, sigma_r=0.2, T=10, n_poly=12)
        g, t, cf = (torch.from_numpy(c[k]).to(dev) for k in ("guide", "target", "conf"))
        p = dts.Params(8.0, 0.2, 3, 10).c()
        ws = torch.empty(lib.dts_solve_workspace_bytes(1, n, n, 1, ctypes.byref(p)), dtype=torch.uint8,
                         device=dev)
        return g, t, cf, torch.empty_like(t), ws

    sizes = []
    for n in (256, 512, 1024, 2048, 4096, 8192):
        g, t, cf, out, ws = prepare(n, 700 + n)
        ms = timed(lambda: dts.solve(g, t, cf, 8.0, 0.2, 3, 10, out=out[None], workspace=ws), steps, warmup)
        sizes.append(dict(size=n, ms=round(ms, 4), mpix_s=round(n * n / ms / 1e3, 1)))
        log(f"  size {n}: {ms:.3f} ms, {n * n / ms / 1e3:.1f} Mpixel/s")
        del g, t, cf, out, ws
    n = 2048
    g, t, cf, out, ws = prepare(n, 900)
    sig = []
    for ss in (16.0, 32.0, 128.0, 256.0):
        for sr in (0.1, 0.3, 0.5, 0.7, 0.9):
            ms = timed(lambda: dts.solve(g, t, cf, ss, sr, 3, 10, out=out[None], workspace=ws), steps, warmup)
            sig.append(dict(sigma_s=ss, sigma_r=sr, ms=round(ms, 4)))
    times = [r["ms"] for r in sig]
    log(f"  sigma sweep at {n}^2: {min(times):.3f} .. {max(times):.3f} ms")
    # time against the number of solver iterations: a least-squares line and the largest
    # relative deviation from it
    its = []
    for T in (1, 2, 5, 10, 20, 40):
        ms = timed(lambda: dts.solve(g, t, cf, 8.0, 0.2, 3, T, out=out[None], workspace=ws), steps, warmup)
        its.append(dict(T=T, ms=round(ms, 4)))
    Ts = np.array([r["T"] for r in its], dtype=np.float64)
    ms_T = np.array([r["ms"] for r in its], dtype=np.float64)
    slope, icpt = np.polyfit(Ts, ms_T, 1)
    dev_T = float(np.max(np.abs(ms_T - (slope * Ts + icpt)) / ms_T))
    log(f"  iteration sweep at {n}^2: {slope:.4f} ms per iteration + {icpt:.4f} ms, max deviation {dev_T:.3f}")
    del g, t, cf, out, ws
    torch.cuda.empty_cache()
    return dict(workload="polygon-scene recipe, Cg=3, Ct=1, N=3, T=10", sizes=sizes,
                sigma=dict(size=n, runs=sig, min_ms=min(times), max_ms=max(times),
                           max_over_min=round(max(times) / min(times), 3)),
                iterations=dict(size=n, runs=its, ms_per_iteration=round(float(slope), 4),
                                intercept_ms=round(float(icpt), 4), max_rel_deviation=round(dev_T, 4)))


def graph_leg(steps, warmup):
    """Small solves, launch-bound: the 256^2 polygon scene (T=10) and the 1920x1080 disparity scene (T=20),
    each as eager dts_solve calls and as replays of one captured HIP graph (SolveGraph)."""
    import torch

    import dts_inputs
    import paper_1805_04590_amd as dts

    dev = torch.device("cuda:0")
    res = {}
    for name, c in (("polygon_256x256_T10", dts_inputs.polygon_256()), ("disparity_1920x1080_T20", dts_inputs.disparity_1920x1080())):
        g, t, cf = (torch.from_numpy(c[k]).to(dev) for k in ("guide", "target", "conf"))
        args = (c["sigma_s"], c["sigma_r"], c["filter_iters"], c["solver_iters"])
        sg = dts.SolveGraph(g, t, cf, *args)
        ms_e = timed(lambda: dts.solve(sg.guide, sg.target, sg.conf, *args, out=sg.out, workspace=sg.workspace),
                     steps * 4, warmup)
        ms_g = timed(sg.replay, steps * 4, warmup)
        SAMPLES[name.replace("_T", " T=") + " (graph replay)"] = (c, sg.out[0].cpu().numpy())
        px = t.shape[-1] * t.shape[-2]
        res[name] = dict(eager_ms=round(ms_e, 4), graph_ms=round(ms_g, 4), eager_mpix_s=round(px / ms_e / 1e3, 1),
                         graph_mpix_s=round(px / ms_g / 1e3, 1), speedup=round(ms_e / ms_g, 3))
        log(f"  {name}: eager {ms_e:.3f} ms, graph {ms_g:.3f} ms")
        del sg, g, t, cf
    torch.cuda.empty_cache()
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): libdts runs each "
              "solve on a single GPU and has no multi-GPU sharding.", file=sys.stderr)
        sys.exit(2)

    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.calibrate_copy > 0:
        n = args.calibrate_copy * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)  # writes 4n bytes
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)  # reads 4n, writes 4n bytes
        torch.cuda.synchronize()
        log(f"calibration: fill and 3 copies of {4 * n} bytes")
        del a, b
        torch.cuda.empty_cache()
    if args.fwd_bwd_only:
        log("forward+backward leg only (profiling mode) ...")
        log("  " + json.dumps(fwd_bwd_leg(args.steps, args.warmup)))
        return
    if args.batched_only is not None:
        log("batched solves only (profiling mode) ...")
        b = batched_leg(args.steps, args.warmup, graph=False, variant=args.batched_only, sequential=False)
        log("  " + json.dumps(b))
        return
    sol = None if args.no_solve else solve_leg(args, dev)

    extras = {}
    if not args.no_extras:
        log("batched leg (64 uneven solves) ...")
        extras["batched"] = batched_leg(max(3, args.steps // 2), 2, graph=not args.no_graph)
        log("  " + json.dumps(extras["batched"]))
        torch.cuda.empty_cache()
        log("forward+backward leg (8 x 1024^2, T=15) ...")
        extras["fwd_bwd"] = fwd_bwd_leg(max(3, args.steps // 2), 2)
        log("  " + json.dumps(extras["fwd_bwd"]))
        torch.cuda.empty_cache()
        log("stereo leg (1920x1080 pair, T=20) ...")
        extras["stereo"] = stereo_leg(max(3, args.steps // 2), 2)
        log("  " + json.dumps(extras["stereo"]))
        torch.cuda.empty_cache()
        log("size and sigma sweeps (polygon-scene recipe) ...")
        extras["sweeps"] = sweep_leg(max(3, args.steps // 2), 2)
        log("small solves: eager against one captured HIP graph ...")
        extras["graph"] = graph_leg(max(3, args.steps // 2), 2)

    cpu = None
    if args.cpu_rows > 0:
        log(f"CPU oracle baseline on {args.cpu_rows} rows ...")
        cpu = cpu_baseline(args.cpu_rows)
        log(f"  {cpu['value']:.3f} Mpixel/s in {cpu['seconds']:.1f} s")
        cpu.pop("seconds")

    if sol is None:
        sol = dict(ms=None, mpix=None, solve_bytes=None, kernels={}, roofline=None, H=None, W=None,
                   Cg=None, Ct=None, T=None, N=None, ss=None, sr=None, variance=None, support=None, box=None)
    ms, mpix = sol["ms"], sol["mpix"]
    gbps = None if ms is None else sol["solve_bytes"] / (ms / 1e3) / 1e9
    res = {
        "metric": METRIC,
        "value": None if mpix is None else round(mpix, 2),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": None if ms is None else round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"multispectral solve {sol['W']}x{sol['H']}, {sol['Cg']}-band guide, "
                        f"{sol['Ct']}-channel target, sigma_s={sol['ss']}, sigma_r={sol['sr']}, "
                        f"N={sol['N']} filter iterations, T={sol['T']}",
            "H": sol["H"], "W": sol["W"], "Cg": sol["Cg"], "Ct": sol["Ct"], "T": sol["T"], "N": sol["N"],
        },
        "solve_algorithmic_GBps": None if gbps is None else round(gbps, 1),
        "solve_hbm_frac": None if gbps is None else round(gbps / HBM_PEAK_GBPS, 4),
        "roofline": sol["roofline"],
        "cpu_baseline": cpu,
        "kernels": sol["kernels"],
        "variance": sol["variance"],
        "support": sol["support"],
        "box": sol["box"],
    }
    res.update(extras)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
