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
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


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
    ap.add_argument("--cpu-views", type=int, default=8, help="views in the CPU-oracle sample")
    ap.add_argument("--nnz-views", type=int, default=90, help="views sampled to count nonzeros")
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
    ws = torch.empty(G.solver_workspace_bytes(tdt, "cgls"), dtype=torch.uint8, device=dev)
    out = torch.empty(g.vol_shape, dtype=torch.float32, device=dev)  # the iterate is always FP32
    torch.cuda.synchronize()
    log("[bench] inputs ready")

    for i in range(args.warmup):
        kct.cgls(G, b, args.iters, workspace=ws, out=out)
        log(f"[bench] warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for i in range(args.steps):
        _, info = kct.cgls(G, b, args.iters, workspace=ws, out=out)
        infos.append(info)
        log(f"[bench] step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    iters_total = sum(i.iterations for i in infos)
    value = iters_total / dt
    ms_per_step = 1e3 * dt / args.steps
    e_final = infos[-1].nb / infos[-1].nb0
    rec_err = (torch.linalg.vector_norm((out - xt).double()) / torch.linalg.vector_norm(xt.double())).item()

    # --- per-kernel timing of the projector pair (HIP events on the launch stream)
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

    # nonzeros of A (exact count of the oracle on evenly spaced views, scaled)
    import oracle
    step = max(1, g.n_views // args.nnz_views)
    sub = g.replace(n_views=len(range(0, g.n_views, step)), explicit_angles=g.angles()[::step])
    nnz = oracle.count_nnz(sub) * (g.n_views / sub.n_views)
    log(f"[bench] nonzeros per application ~ {nnz:.4g}")
    fwd_bytes = nnz * s_bytes + g.n_rays * s_bytes
    bwd_bytes = nnz * s_bytes + g.n_vox * s_bytes
    dominant = "backward" if t_bwd >= t_fwd else "forward"
    ach = (bwd_bytes / t_bwd if dominant == "backward" else fwd_bytes / t_fwd) / 1e9
    roofline = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dominant,
                "forward_ms": round(t_fwd * 1e3, 3), "backward_ms": round(t_bwd * 1e3, 3),
                "forward_GBs": round(fwd_bytes / t_fwd / 1e9, 1), "backward_GBs": round(bwd_bytes / t_bwd / 1e9, 1),
                "nnz_per_application": float(f"{nnz:.4g}")}

    cpu = None
    if not args.no_cpu:
        xs = x_true.astype(np.float64)
        cstep = max(1, g.n_views // args.cpu_views)
        idx = np.arange(0, g.n_views, cstep)[: args.cpu_views]
        subc = g.replace(n_views=len(idx), explicit_angles=g.angles()[idx])
        t = time.perf_counter()
        bs = oracle.project(subc, xs)
        t_a = time.perf_counter() - t
        t = time.perf_counter()
        oracle.backproject(subc, bs)
        t_at = time.perf_counter() - t
        per_iter = (t_a + t_at) * (g.n_views / subc.n_views)
        cpu = {"value": round(1.0 / per_iter, 6), "unit": "CGLS iters/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": f"one A and one A^T over {subc.n_views} of {g.n_views} views (full volume), "
                         f"{t_a + t_at:.1f} s, scaled by {g.n_views / subc.n_views:g}; vector updates excluded"}
        log(f"[bench] cpu oracle sample: A {t_a:.2f} s, A^T {t_at:.2f} s on {subc.n_views} views")

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
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
