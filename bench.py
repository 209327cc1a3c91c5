"""Benchmark: CGLS reconstruction on the 512^3 x 720-view cone-beam problem.

    python bench.py [--steps K] [--warmup W] [--dtype f32|bf16|f16] [--config c3]

One step is one full CGLS solve (Algorithm 1, 30 iterations, x0 = 0, ERR = 0)
of the 512^3 volume (0.25 mm voxels) from 720 views of a 616 x 480 detector
(0.6 mm pixels), SID 500 mm, SDD 1000 mm, on seeded synthetic data: a
20-ellipsoid phantom projected by the library and corrupted with Poisson
noise at 1e4 photons per ray (log-transformed).  Inputs are resident in HBM
before the timed region.  The value is CGLS iterations per second.

Besides the JSON fields of the benchmark contract the line carries
  roofline      effective bandwidth of the dominant projector kernel:
                (nonzeros * s + outputs * s) bytes per launch / launch time,
                timed with HIP events, against the 8 TB/s HBM peak;
  cpu_baseline  the FP64 oracle (plain C, OpenMP) timed on a sample of views
                of the same problem, extrapolated to CGLS iterations per second.
Progress goes to stderr; stdout carries exactly one JSON line.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Files each projector kernel is compiled from; the measured-traffic record in
# profiles/ is valid only for the sources it was taken with.
KERNEL_SOURCES = {
    "forward": ("csrc/projector.hip", "csrc/kct_ray.h", "csrc/kct_weights.h", "csrc/kct_internal.h",
                "csrc/kct_epilogue.h", "csrc/kct_batch.h", "csrc/geometry.cpp", "build.py"),
    "backward": ("csrc/backproject.hip", "csrc/kct_gather.h", "csrc/kct_weights.h", "csrc/kct_internal.h",
                 "csrc/kct_epilogue.h", "csrc/kct_batch.h", "csrc/geometry.cpp", "build.py"),
}
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "projector_c3_hbm_counters.json")


def kernel_source_hash(kind):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kind]:
        with open(os.path.join(ROOT, "paper_2110_13526_amd", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic_bytes(kind, workload, dtype):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated against a copy
    of known size) from the committed counter record, or None when there is no
    record for this kernel, workload and storage type, or the kernel's sources
    changed since it was taken."""
    try:
        with open(TRAFFIC_RECORD) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    ent = rec.get("kernels", {}).get(f"{kind}_{dtype}")
    if not ent or rec.get("workload") != workload or ent.get("source_sha256") != kernel_source_hash(kind):
        return None
    cal = rec["calibration"]
    return (ent["fetch_kib"] * cal["fetch_factor"] + ent["write_kib"] * cal["write_factor"]) * 1024.0


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c3")
    ap.add_argument("--iters", type=int, default=30)
    ap.add_argument("--dtype", default="f32", choices=["f32", "bf16", "f16"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--cpu-views", type=int, default=64, help="views in the CPU-oracle sample (all threads)")
    ap.add_argument("--cpu-views-1t", type=int, default=6, help="views in the one-thread CPU-oracle sample")
    ap.add_argument("--nnz-views", type=int, default=90, help="views sampled to count nonzeros")
    ap.add_argument("--no-precision", action="store_true", help="skip the BF16 / FP16 comparison solves")
    ap.add_argument("--no-tt", action="store_true", help="skip the timing of the TT footprint projector pair")
    ap.add_argument("--kernels-only", action="store_true",
                    help="profiling pass: one forward, one backward, one CGLS iteration (the solver's "
                         "instantiations) and one 1 GiB device copy (the calibration of the HBM byte "
                         "counters), nothing timed")
    ap.add_argument("--tt-pair", action="store_true",
                    help="with --kernels-only: also one forward and one backward of the TT footprint pair")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU design shards views, see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch

    import kct_inputs as ki
    import paper_2110_13526_amd as kct

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    tdt = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}[args.dtype]
    s_bytes = torch.tensor([], dtype=tdt).element_size()

    g = ki.config(args.config)
    log(f"[bench] {args.config}: volume {g.vol_shape}, projections {g.proj_shape}, dtype {args.dtype}")
    G = kct.Geometry.from_desc(g, device=dev)
    x_true = ki.phantom(g, ki.N_ELLIPSOIDS[args.config], ki.SEEDS[args.config])
    xt = torch.from_numpy(x_true).to(dev)
    b32 = kct.project(G, xt)
    bn = ki.poisson_log_noise(b32.cpu().numpy(), 1e4, ki.SEEDS[args.config] + 1_000_000)
    b = torch.from_numpy(bn).to(dev).to(tdt)
    del b32, bn
    if args.kernels_only:
        xin = xt.to(tdt)
        pbuf = torch.empty(g.proj_shape, dtype=tdt, device=dev)
        vbuf = torch.empty(g.vol_shape, dtype=tdt, device=dev)
        pws = torch.empty(G.project_workspace_bytes(tdt), dtype=torch.uint8, device=dev)
        kct.project(G, xin, out=pbuf, workspace=pws)
        kct.backproject(G, b, out=vbuf)
        del pbuf, vbuf, pws
        # one CGLS iteration: the solver's own instantiations (r = A^T e with its
        # norm epilogue, p = A d with its norm epilogue), one launch each
        wsk = torch.empty(G.solver_workspace_bytes(tdt, "cgls"), dtype=torch.uint8, device=dev)
        xk = torch.empty(g.vol_shape, dtype=torch.float32, device=dev)
        kct.cgls(G, b, 1, workspace=wsk, out=xk)
        del wsk, xk
        if args.tt_pair:
            G.set_projector("tt")
            pbuf = torch.empty(g.proj_shape, dtype=tdt, device=dev)
            vbuf = torch.empty(g.vol_shape, dtype=tdt, device=dev)
            pws = torch.empty(G.project_workspace_bytes(tdt), dtype=torch.uint8, device=dev)
            kct.project(G, xin, out=pbuf, workspace=pws)
            kct.backproject(G, b, out=vbuf)
            G.set_projector("siddon")
            del pbuf, vbuf, pws
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)  # 1 GiB read, 1 GiB written
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("[bench] kernels-only pass done: forward, backward, one CGLS iteration, "
            + ("the TT pair, " if args.tt_pair else "") + "1 GiB copy")
        return
    ws = torch.empty(G.solver_workspace_bytes(tdt, "cgls"), dtype=torch.uint8, device=dev)
    out = torch.empty(g.vol_shape, dtype=torch.float32, device=dev)  # the iterate is always FP32
    torch.cuda.synchronize()
    log("[bench] inputs ready")

    for i in range(args.warmup):
        kct.cgls(G, b, args.iters, workspace=ws, out=out)
        log(f"[bench] warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    # every projector launch of the timed solves is bracketed by HIP events on
    # the solve's stream (the library's launch timing): the roofline is priced
    # on the solver's own launches inside the timed region
    kct.timing_enable(True)
    t0 = time.perf_counter()
    infos = []
    step_s = []  # each solve returns after its final synchronisation
    for i in range(args.steps):
        ts = time.perf_counter()
        _, info = kct.cgls(G, b, args.iters, workspace=ws, out=out)
        step_s.append(time.perf_counter() - ts)
        infos.append(info)
        log(f"[bench] step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n_fwd_s, t_fwd_s, t_fwd_s_min, t_fwd_s_max = kct.timing_get("forward")
    n_bwd_s, t_bwd_s, t_bwd_s_min, t_bwd_s_max = kct.timing_get("backward")
    kct.timing_enable(False)
    log(f"[bench] in the timed solves: forward {t_fwd_s:.2f} ms over {n_fwd_s} launches, "
        f"backward {t_bwd_s:.2f} ms over {n_bwd_s} launches")
    iters_total = sum(i.iterations for i in infos)
    value = iters_total / dt
    ms_per_step = 1e3 * dt / args.steps
    e_final = infos[-1].nb / infos[-1].nb0
    rec_err = (torch.linalg.vector_norm((out - xt).double()) / torch.linalg.vector_norm(xt.double())).item()

    # --- the projector pair launched alone, plain epilogue (HIP events on the launch stream)
    def timed(fn, reps):
        st = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fn()
        e0.record(st)
        for _ in range(reps):
            fn()
        e1.record(st)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps / 1e3

    xin = xt.to(tdt)
    pbuf = torch.empty(g.proj_shape, dtype=tdt, device=dev)
    vbuf = torch.empty(g.vol_shape, dtype=tdt, device=dev)
    pws = torch.empty(G.project_workspace_bytes(tdt), dtype=torch.uint8, device=dev)
    t_fwd = timed(lambda: kct.project(G, xin, out=pbuf, workspace=pws), 3)
    t_bwd = timed(lambda: kct.backproject(G, b, out=vbuf), 3)
    log(f"[bench] forward {t_fwd * 1e3:.2f} ms, backward {t_bwd * 1e3:.2f} ms per launch")

    # measured STREAM triad a = b + s c on 2^28-element FP32 arrays (3 GiB moved per launch)
    ta = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    tb_ = torch.ones_like(ta)
    tc_ = torch.ones_like(ta)
    t_triad = timed(lambda: torch.add(tb_, tc_, alpha=0.5, out=ta), 5)
    triad_gbs = 3.0 * ta.numel() * 4 / t_triad / 1e9
    del ta, tb_, tc_
    log(f"[bench] STREAM triad {triad_gbs:.0f} GB/s")

    # nonzeros of A (exact count of the oracle on evenly spaced views, scaled)
    import oracle
    step = max(1, g.n_views // args.nnz_views)
    sub = g.replace(n_views=len(range(0, g.n_views, step)), explicit_angles=g.angles()[::step])
    nnz = oracle.count_nnz(sub) * (g.n_views / sub.n_views)
    log(f"[bench] nonzeros per application ~ {nnz:.4g}")
    fwd_bytes = nnz * s_bytes + g.n_rays * s_bytes
    bwd_bytes = nnz * s_bytes + g.n_vox * s_bytes
    # the solver's launches in the timed region (seconds per launch)
    t_fwd_r, t_bwd_r = t_fwd_s / 1e3, t_bwd_s / 1e3
    dominant = "backward" if t_bwd_r >= t_fwd_r else "forward"
    ach = (bwd_bytes / t_bwd_r if dominant == "backward" else fwd_bytes / t_fwd_r) / 1e9
    t_dom = t_bwd_r if dominant == "backward" else t_fwd_r
    tb = measured_traffic_bytes(dominant, args.config, args.dtype)
    roofline = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4),
                "stream_triad_GBs": round(triad_gbs, 1), "frac_of_stream": round(ach / triad_gbs, 4),
                "traffic": None if tb is None else round(tb / t_dom / 1e9, 1),
                "traffic_bytes_per_launch": None if tb is None else float(f"{tb:.4g}"),
                "kernel": dominant, "timed_in": "the solver's launches in the timed steps",
                "forward_ms": round(t_fwd_s, 3), "backward_ms": round(t_bwd_s, 3),
                "forward_launches": n_fwd_s, "backward_launches": n_bwd_s,
                "forward_ms_min_max": [round(t_fwd_s_min, 3), round(t_fwd_s_max, 3)],
                "backward_ms_min_max": [round(t_bwd_s_min, 3), round(t_bwd_s_max, 3)],
                "forward_GBs": round(fwd_bytes / t_fwd_r / 1e9, 1), "backward_GBs": round(bwd_bytes / t_bwd_r / 1e9, 1),
                "forward_ms_plain": round(t_fwd * 1e3, 3), "backward_ms_plain": round(t_bwd * 1e3, 3),
                "nnz_per_application": float(f"{nnz:.4g}")}

    # --- the separable trapezoid-footprint pair on the same workload (secondary)
    tt = None
    if not args.no_tt:
        G.set_projector("tt")
        t_fwd_tt = timed(lambda: kct.project(G, xin, out=pbuf, workspace=pws), 2)
        t_bwd_tt = timed(lambda: kct.backproject(G, b, out=vbuf), 2)
        G.set_projector("siddon")
        # each operand read once and the result written once: the least HBM
        # traffic of a launch; the TT pair is bound by its arithmetic (VALU
        # issue), far from this
        io_bytes = (g.n_vox + g.n_rays) * s_bytes
        tt = {"forward_ms": round(t_fwd_tt * 1e3, 3), "backward_ms": round(t_bwd_tt * 1e3, 3),
              "pair_per_s": round(1.0 / (t_fwd_tt + t_bwd_tt), 4), "bound": "alu",
              "io_bytes_per_launch": io_bytes,
              "io_frac_of_hbm": [round(io_bytes / t_fwd_tt / 1e9 / HBM_PEAK_GBS, 5),
                                 round(io_bytes / t_bwd_tt / 1e9 / HBM_PEAK_GBS, 5)]}
        log(f"[bench] TT pair: forward {t_fwd_tt * 1e3:.2f} ms, backward {t_bwd_tt * 1e3:.2f} ms per launch")

    cpu = None
    if not args.no_cpu:
        import oracle
        xs = x_true.astype(np.float64)

        def oracle_pair(n_views):
            """One A and one A^T of the oracle over n_views evenly spaced views of
            the workload (full volume): seconds for each."""
            cstep = max(1, g.n_views // n_views)
            idx = np.arange(0, g.n_views, cstep)[:n_views]
            subc = g.replace(n_views=len(idx), explicit_angles=g.angles()[idx])
            t = time.perf_counter()
            bs = oracle.project(subc, xs)
            t_a = time.perf_counter() - t
            t = time.perf_counter()
            oracle.backproject(subc, bs)
            t_at = time.perf_counter() - t
            return subc.n_views, t_a, t_at

        threads = oracle.num_threads()
        nv_all, t_a, t_at = oracle_pair(args.cpu_views)
        scale = g.n_views / nv_all
        log(f"[bench] cpu oracle, {threads} threads: A {t_a:.2f} s, A^T {t_at:.2f} s on {nv_all} views")
        oracle.set_num_threads(1)
        try:
            nv_1, t_a1, t_at1 = oracle_pair(args.cpu_views_1t)
        finally:
            oracle.set_num_threads(threads)
        scale1 = g.n_views / nv_1
        log(f"[bench] cpu oracle, 1 thread: A {t_a1:.2f} s, A^T {t_at1:.2f} s on {nv_1} views")
        try:
            affinity = len(os.sched_getaffinity(0))
        except (AttributeError, OSError):
            affinity = None
        cpu = {"value": round(1.0 / ((t_a + t_at) * scale), 6), "unit": "CGLS iters/s", "cores": threads,
               "kind": "oracle",
               "sample": f"one A and one A^T of the FP64 oracle over {nv_all} of {g.n_views} views (full "
                         f"volume) with {threads} threads, {t_a + t_at:.1f} s, scaled by {scale:g} to the "
                         f"workload; vector updates excluded (full solves incl. updates: "
                         f"profiles/oracle_solver_timings.md)",
               "cpu_model": _cpu_model(), "nproc": os.cpu_count(), "affinity_cpus": affinity,
               "ms_per_A": round(1e3 * t_a * scale, 1), "ms_per_AT": round(1e3 * t_at * scale, 1),
               "one_thread": {"value": round(1.0 / ((t_a1 + t_at1) * scale1), 7),
                              "ms_per_A": round(1e3 * t_a1 * scale1, 1),
                              "ms_per_AT": round(1e3 * t_at1 * scale1, 1),
                              "sample": f"{nv_1} of {g.n_views} views, {t_a1 + t_at1:.1f} s, scaled by {scale1:g}"}}

    # --- the same solve with the other storage types (BF16 / FP16 work vectors and b, FP32
    # iterate), with the same warm-up and number of timed steps as the main solve; their steps
    # are interleaved so that drift of the clock affects both alike
    precision = None
    if not args.no_precision:
        def rate_stats(times):
            r = np.array([args.iters / t for t in times])
            return {"iters_per_s": round(float(r.mean()), 4), "iters_per_s_std": round(float(r.std()), 4),
                    "iters_per_s_min": round(float(r.min()), 4), "iters_per_s_max": round(float(r.max()), 4),
                    "steps": len(times)}

        def rec_error():
            return (torch.linalg.vector_norm((out - xt).double()) / torch.linalg.vector_norm(xt.double())).item()

        precision = {args.dtype: {**rate_stats(step_s), "rel_error_vs_x_true": round(rec_err, 6),
                                  "relative_discrepancy": round(e_final, 6)}}
        others = [(n, d) for n, d in (("f32", torch.float32), ("bf16", torch.bfloat16), ("f16", torch.float16))
                  if n != args.dtype]
        inputs = {n: (b.float().to(d), torch.empty(G.solver_workspace_bytes(d, "cgls"), dtype=torch.uint8,
                                                     device=dev)) for n, d in others}
        times = {n: [] for n, _ in others}
        last = {}
        for i in range(args.warmup + args.steps):
            for n, _ in others:
                bo, wso = inputs[n]
                ts = time.perf_counter()
                _, info = kct.cgls(G, bo, args.iters, workspace=wso, out=out)
                if i >= args.warmup:
                    times[n].append(time.perf_counter() - ts)
                last[n] = (info, rec_error())
            log(f"[bench] storage comparison round {i + 1}/{args.warmup + args.steps} done")
        for n, _ in others:
            info, err_o = last[n]
            precision[n] = {**rate_stats(times[n]), "rel_error_vs_x_true": round(err_o, 6),
                            "relative_discrepancy": round(info.nb / info.nb0, 6)}
            log(f"[bench] {n}: {precision[n]}")
        del inputs
        ref = precision["f32"]
        for name, r in precision.items():
            r["speedup_vs_f32"] = round(r["iters_per_s"] / ref["iters_per_s"], 4)
            r["error_ratio_vs_f32"] = round(r["rel_error_vs_x_true"] / ref["rel_error_vs_x_true"], 6)
            r["equal_error"] = abs(r["error_ratio_vs_f32"] - 1.0) <= 0.01

    line = {
        "metric": "CGLS iters/s + GB/s vs HBM roofline, 512^3x720 views, BF16 vs FP32 at equal err",
        "value": round(value, 4), "unit": "CGLS iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 2), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": f"{args.config}: CGLS {args.iters} it, {g.nx}x{g.ny}x{g.nz} @{g.vx} mm, "
                               f"{g.n_views} views, {g.nu}x{g.nv} @{g.du} mm, SID {g.sid:g}, SDD {g.sdd:g}",
                   "iterations_per_step": args.iters, "relative_discrepancy": round(e_final, 6),
                   "rel_error_vs_x_true": round(rec_err, 6), "parallelism": "single GPU"},
        "roofline": roofline,
        "precision": precision,
        "tt_projector": tt,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
