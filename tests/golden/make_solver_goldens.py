"""Write the stored expected values of the full-size solver parity tests
(tests/test_gpu_goldens.py) from the FP64 oracle alone.

    python tests/golden/make_solver_goldens.py [case ...]

Cases (default: all):
  c1_cgls_k10      64^3, 90 views, CGLS 10 iterations (Gaussian noise)
  c3down_cgls_k10  128^3, 720 views, CGLS 10 iterations (transmission noise)
  c3down_cgls_k30  the same, 30 iterations
  c2_cgls_k40      256^3, 360 views, CGLS 40 iterations (transmission noise)
  c2_lsqr_k40      the same problem, LSQR 40 iterations
  c4i14_cgls_k3    instance 14 of the 48-instance batched workload (64^3, 165
                   views, 135 x 135 detector), CGLS 3 iterations (Gaussian noise)

For every case the data are b = noise(A_oracle x_true) rounded to float (the
single-precision input the library is given), and the file holds:
  b_sha256        hash of those float32 bytes (the test regenerates b and checks it)
  history         NB_k / NB0, k = 1..K, of the FP64 solve
  idx, x_idx      4096 fixed voxel indices and the FP64 iterate x_K there
  x_norm          |x_K| over the whole volume
  err_truth       |x_K - x_true| / |x_true| of the FP64 solve
  spread_alt      |x_K - x_K(other solver)| / |x_K|: CGLS against LSQR in FP64,
                  equal in exact arithmetic (the conditioning of the K-th iterate)
  spread32        |x_K - x_K(store32)| / |x_K|, and spread32_idx on the sampled
                  voxels: the same solver with its vectors stored in single
                  precision (the oracle's store32 option), i.e. how far
                  single-precision storage alone moves the K-th iterate
  history32       NB_k / NB0 of that single-precision-storage solve
  spread_f32_idx  |x_K - x_K(f32)| / |x_K| on the sampled voxels (spread_f32 over
                  the volume when the file is written in one run), history_f32,
                  err_truth_f32: the same solver in the precision
                  structure of a single-precision GPU path -- vectors stored in
                  float and the projector pair computed in float (the oracle's
                  "siddon32" operator with store32), scalars in double
  seconds         wall time of the FP64 solve, threads, CPU model

    python tests/golden/make_solver_goldens.py --add-f32 [case ...]

adds the spread_f32 fields to existing files (the FP64 results are kept; the
regenerated data must hash to the stored value).
A Markdown summary of the oracle timings goes to profiles/oracle_solver_timings.md.
"""
from __future__ import annotations

import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import kct_inputs as ki  # noqa: E402
import oracle  # noqa: E402

N_SAMPLES = 4096
SAMPLE_SEED = 20211026

CASES = {
    "c1_cgls_k10": ("c1", "cgls", 10),
    "c3down_cgls_k10": ("c3down", "cgls", 10),
    "c3down_cgls_k30": ("c3down", "cgls", 30),
    "c2_cgls_k40": ("c2", "cgls", 40),
    "c2_lsqr_k40": ("c2", "lsqr", 40),
    "c4i14_cgls_k3": ("c4i14", "cgls", 3),
}


def geometry(cfg: str):
    """A named configuration, or instance k of the batched workload ("c4i<k>")."""
    if cfg.startswith("c4i"):
        return ki.batch_instance(int(cfg[3:]))
    return ki.config(cfg)


def problem_data(cfg: str):
    """x_true and the float32 data of a configuration, from the oracle's
    projector: Gaussian noise (0.5 % of max b) for c1 and the batch instances
    (10 ellipsoids, seed 4000 + k), transmission noise at 1e4 photons per ray
    for the others."""
    g = geometry(cfg)
    if cfg.startswith("c4i"):
        seed, n_ell = 4000 + int(cfg[3:]), 10
    else:
        seed, n_ell = ki.SEEDS[cfg], ki.N_ELLIPSOIDS[cfg]
    x_true = ki.phantom(g, n_ell, seed)
    b = oracle.project(g, x_true.astype(np.float64))
    if cfg == "c1" or cfg.startswith("c4i"):
        b = ki.gaussian_noise(b, 0.005, seed + 1_000_000)
    else:
        b = ki.poisson_log_noise(b, 1e4, seed + 1_000_000)
    b32 = np.ascontiguousarray(b, dtype=np.float32)
    return g, x_true, b32


def b_hash(b32: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(b32, dtype=np.float32).tobytes()).hexdigest()


def sample_indices(n_vox: int) -> np.ndarray:
    rng = np.random.default_rng(SAMPLE_SEED)
    return np.sort(rng.choice(n_vox, size=min(N_SAMPLES, n_vox), replace=False)).astype(np.int64)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _solve(cache: dict, cfg: str, solver: str, K: int, store32: bool, projector: str = "siddon"):
    """One oracle solve, computed once per (configuration, solver, K, storage,
    operator) and shared by the cases that need it; returns (result, seconds)."""
    key = (cfg, solver, K, store32, projector)
    if key not in cache:
        g, _, b32 = cache[cfg]
        t = time.perf_counter()
        res = getattr(oracle, solver)(g, b32.astype(np.float64), K, store32=store32, projector=projector)
        secs = time.perf_counter() - t
        tag = "f32 " if projector == "siddon32" else ("store32 " if store32 else "FP64 ")
        print(f"[golden] {cfg}: {tag}{solver} K={K} in {secs:.1f} s", flush=True)
        cache[key] = (res, secs)
    return cache[key]


def _data_cached(cfg: str, cache: dict):
    if cfg not in cache:
        t = time.perf_counter()
        cache[cfg] = problem_data(cfg)
        print(f"[golden] {cfg}: data in {time.perf_counter() - t:.1f} s", flush=True)
    return cache[cfg]


def f32_fields(name: str, cache: dict, x_idx: np.ndarray, idx: np.ndarray, x=None) -> dict:
    """The single-precision-structure yardstick of a case: its spread from the
    FP64 iterate on the sampled voxels (x_idx = x_K[idx]) and, when the whole
    FP64 iterate x is at hand, over the volume."""
    cfg, solver, K = CASES[name]
    _, x_true, _ = _data_cached(cfg, cache)
    rf, _ = _solve(cache, cfg, solver, K, True, "siddon32")
    out = {"spread_f32_idx": rel(rf.x.ravel()[idx], x_idx), "history_f32": rf.history,
           "err_truth_f32": rel(rf.x, x_true)}
    if x is not None:
        out["spread_f32"] = rel(rf.x, x)
    return out


def run_case(name: str, cache: dict) -> dict:
    cfg, solver, K = CASES[name]
    g, x_true, b32 = _data_cached(cfg, cache)
    other = "lsqr" if solver == "cgls" else "cgls"
    res, secs = _solve(cache, cfg, solver, K, False)
    alt, _ = _solve(cache, cfg, other, K, False)
    r32, _ = _solve(cache, cfg, solver, K, True)
    idx = sample_indices(g.n_vox)
    x = res.x.ravel()
    out = {
        "config": cfg, "solver": solver, "K": K, "b_sha256": b_hash(b32),
        "history": res.history, "nb0": res.nb0, "nb": res.nb, "iterations": res.iterations,
        "idx": idx, "x_idx": x[idx], "x_norm": float(np.linalg.norm(x)),
        "err_truth": rel(x, x_true), "err_truth32": rel(r32.x, x_true),
        "spread_alt": rel(alt.x, x), "spread_alt_idx": rel(alt.x.ravel()[idx], x[idx]),
        "history_alt": alt.history,
        "spread32": rel(r32.x, x), "spread32_idx": rel(r32.x.ravel()[idx], x[idx]),
        "history32": r32.history,
        "seconds": secs, "threads": oracle.num_threads(), "cpu": cpu_model(),
    }
    out.update(f32_fields(name, cache, x[idx], idx, x))
    return out


def add_f32(name: str, cache: dict) -> dict:
    """Load a stored case, check its data, add the spread_f32 fields."""
    path = os.path.join(HERE, f"{name}.npz")
    with np.load(path, allow_pickle=False) as z:
        rec = {k: z[k][()] if z[k].ndim == 0 else z[k].copy() for k in z.files}
    cfg, _, _ = CASES[name]
    g, _, b32 = _data_cached(cfg, cache)
    if b_hash(b32) != str(rec["b_sha256"]):
        raise SystemExit(f"{name}: regenerated data differ from the stored input")
    # the FP64 iterate is stored on the sampled voxels only
    rec.update(f32_fields(name, cache, np.asarray(rec["x_idx"]), np.asarray(rec["idx"])))
    return rec


def save(name: str, rec: dict) -> str:
    path = os.path.join(HERE, f"{name}.npz")
    arrays = {k: np.asarray(v) for k, v in rec.items()}
    np.savez(path, **arrays)
    return path


def write_timings(recs: dict) -> None:
    path = os.path.join(ROOT, "profiles", "oracle_solver_timings.md")
    lines = ["# FP64 oracle: full solves (CPU)", "",
             "Written by `python tests/golden/make_solver_goldens.py` (plain C, FP64, OpenMP), the runs that "
             "produce the stored values of the full-size solver parity tests.", "",
             "| case | volume | views x detector | solver | K | wall s | s / iteration | threads | CPU |",
             "|---|---|---|---|---|---|---|---|---|"]
    for name, r in recs.items():
        g = geometry(str(r["config"]))
        lines.append(f"| {name} | {g.nx}^3 | {g.n_views} x {g.nu}x{g.nv} | {r['solver']} | {int(r['K'])} | "
                     f"{float(r['seconds']):.1f} | {float(r['seconds']) / int(r['K']):.2f} | {int(r['threads'])} | "
                     f"{r['cpu']} |")
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def main(argv):
    add = bool(argv) and argv[0] == "--add-f32"
    if add:
        argv = argv[1:]
    names = argv or list(CASES)
    for n in names:
        if n not in CASES:
            raise SystemExit(f"unknown case {n}; known: {', '.join(CASES)}")
    oracle.build(force=False)
    cache: dict = {}
    for name in names:
        rec = add_f32(name, cache) if add else run_case(name, cache)
        path = save(name, rec)
        summary = {k: (float(v) if isinstance(v, (float, np.floating)) else int(v) if isinstance(v, np.integer) else v)
                   for k, v in rec.items()
                   if k in ("K", "err_truth", "err_truth32", "err_truth_f32", "spread_alt", "spread32", "spread32_idx",
                            "spread_f32", "spread_f32_idx", "seconds")}
        print(f"[golden] wrote {os.path.relpath(path, ROOT)} {json.dumps(summary)}", flush=True)
    recs = {}
    for name in CASES:
        path = os.path.join(HERE, f"{name}.npz")
        if os.path.exists(path):
            with np.load(path, allow_pickle=False) as z:
                recs[name] = {k: z[k][()] for k in ("config", "solver", "K", "seconds", "threads", "cpu")}
    write_timings(recs)


if __name__ == "__main__":
    main(sys.argv[1:])
