"""Batched form: many independent CGLS reconstructions with their own
geometries, one launch per step for all instances (persistent work-queue
launches for the projector steps), the iteration replayed as a HIP graph,
through the C ABI (kct_batch_*).

Each instance keeps its own scalars and the tile decomposition of its own
solve, so with the default variants a batched solve returns exactly the bits of
the instance's separate kct_cgls_solve; graph replay and plain launches give
the same bits; the tuner may change an instance's forward or backprojection
variant, which only regroups partial sums (results within the FP32 solver
bound).
"""
import json
import os
import time

import numpy as np
import pytest

import kct_inputs as ki
import oracle
from tests.gpu_util import dev, geometry, rel, say, to_np, torch_mod

pytestmark = pytest.mark.gpu


def _problem(i, scale, torch, oracle_data=True):
    g = ki.batch_instance(i, scale)
    x_true = ki.phantom(g, 10, 4000 + i)
    if oracle_data:
        b = oracle.project(g, x_true.astype(np.float64))
    else:
        import paper_2110_13526_amd as kct
        G = geometry(g)
        b = kct.project(G, torch.from_numpy(x_true.astype(np.float32)).to(dev())).cpu().numpy()
    b = ki.gaussian_noise(b, 0.005, 4000 + i + 1_000_000).astype(np.float32)
    return g, x_true, b


@pytest.fixture(scope="module")
def small_batch():
    torch = torch_mod()
    probs = [_problem(i, 0.25, torch) for i in range(6)]
    geoms = [geometry(g) for g, _, _ in probs]
    bs = [torch.from_numpy(b).to(dev()) for _, _, b in probs]
    say("[batch] sizes " + ", ".join(f"{g.nx}^3/{g.n_views}x{g.nv}x{g.nu}" for g, _, _ in probs))
    return probs, geoms, bs


def test_batch_equals_separate_solves(small_batch):
    import paper_2110_13526_amd as kct
    torch = torch_mod()
    probs, geoms, bs = small_batch
    K = 6
    batch = kct.Batch(geoms)
    xs_g, inf_g = batch.cgls(bs, K, graph=True)
    xs_g = [x.clone() for x in xs_g]
    xs_e, inf_e = batch.cgls(bs, K, graph=False)
    xs_e = [x.clone() for x in xs_e]
    # replay again after unrelated eager work on the device
    junk = torch.randn(1 << 20, device=dev()).sum().item()
    xs_g2, _ = batch.cgls(bs, K, graph=True)
    for i, (G, b) in enumerate(zip(geoms, bs)):
        x1, info1 = kct.cgls(G, b, K)
        assert torch.equal(xs_g[i], x1), i
        assert torch.equal(xs_e[i], x1), i
        assert torch.equal(xs_g2[i], x1), i
        assert inf_g[i].iterations == info1.iterations == K
        assert inf_g[i].nb == info1.nb and inf_g[i].nb0 == info1.nb0
    assert np.isfinite(junk)
    # and one instance against the FP64 oracle
    g, x_true, b = probs[0]
    ref = oracle.cgls(g, b.astype(np.float64), K)
    assert rel(to_np(xs_g[0]), ref.x) < 1e-4
    batch.close()


def test_batch_tuner_and_cache(small_batch, tmp_path):
    import paper_2110_13526_amd as kct
    probs, geoms, bs = small_batch
    K = 6
    batch = kct.Batch(geoms)
    ref, _ = batch.cgls(bs, K)
    ref = [x.clone() for x in ref]
    cache = str(tmp_path / "tune.txt")
    batch.tune(cache=cache)
    lines = open(cache).read().split("\n")
    keys = {ln.split()[0] for ln in lines if ln.strip()}
    assert len(keys) == len({(g.nx, g.ny, g.nz, g.n_views, g.nv, g.nu) for g, _, _ in probs})
    assert all(ln.split()[1] in ("1", "2") and ln.split()[2] in ("0", "1") for ln in lines if ln.strip())
    xs, infos = batch.cgls(bs, K)
    for x, r in zip(xs, ref):
        assert rel(to_np(x), to_np(r)) < 1e-5
    # a second tuner reads the cache and appends nothing
    batch2 = kct.Batch(geoms)
    batch2.tune(cache=cache)
    assert open(cache).read().split("\n") == lines
    batch.close()
    batch2.close()


def test_batch_latencies(small_batch):
    """Per-instance completion times of a batched solve, on the device clock:
    positive, within the solve's wall time, and read again unchanged."""
    import paper_2110_13526_amd as kct
    torch = torch_mod()
    probs, geoms, bs = small_batch
    batch = kct.Batch(geoms)
    with pytest.raises(kct.KctError):
        batch.latencies()  # no solve yet
    torch.cuda.synchronize()
    t = time.perf_counter()
    batch.cgls(bs, 6)
    wall = time.perf_counter() - t
    lat = batch.latencies()
    say(f"[batch] latencies {['%.4f' % v for v in lat]} s, wall {wall:.4f} s")
    assert len(lat) == len(geoms)
    assert all(0.0 < v <= wall for v in lat)
    assert batch.latencies() == lat
    batch.close()


def test_batch_zero_iterations_returns_zeros(small_batch):
    """K = 0 returns x0 = 0 in every instance (the iterate is written even when
    the solve stops before its first step)."""
    import paper_2110_13526_amd as kct
    torch = torch_mod()
    probs, geoms, bs = small_batch
    batch = kct.Batch(geoms)
    outs = [torch.full(g.vol_shape, float("nan"), dtype=torch.float32, device=dev()) for g, _, _ in probs]
    xs, infos = batch.cgls(bs, 0, outs=outs)
    for x, inf in zip(xs, infos):
        assert inf.iterations == 0
        assert torch.count_nonzero(x).item() == 0
    batch.close()


def test_batch_argument_errors(small_batch):
    import paper_2110_13526_amd as kct
    torch = torch_mod()
    probs, geoms, bs = small_batch
    batch = kct.Batch(geoms)
    with pytest.raises(ValueError):
        batch.cgls(bs[:-1], 2)
    small = torch.empty(16, dtype=torch.uint8, device=dev())
    with pytest.raises(kct.KctError):
        batch.cgls(bs, 2, workspace=small)
    batch.close()


def test_batch_c4_full_size():
    """The batched workload at its full size: all 48 seeded instances (64^3 to
    192^3, 60-360 views, 96^2-288^2 detectors, SID 400-700 mm, SDD 800-1400 mm)
    in one batch, 3 CGLS iterations.  A subset (the smallest and the largest
    instances, and every eighth) is bitwise equal to its separate
    kct_cgls_solve; instance 14 is solved from the oracle's data and compared
    with the stored FP64 oracle result (tests/golden/c4i14_cgls_k3.npz) at the
    FP32 solver bound."""
    import paper_2110_13526_amd as kct
    from tests.golden import make_solver_goldens as mg
    torch = torch_mod()
    K = 3
    gold_i = 14
    gold = dict(np.load(os.path.join(os.path.dirname(__file__), "golden", "c4i14_cgls_k3.npz"), allow_pickle=False))
    say("[batch] c4: building 48 full-size instances")
    probs = []
    for i in range(48):
        if i == gold_i:
            g, x_true, b = mg.problem_data("c4i14")
            assert mg.b_hash(b) == str(gold["b_sha256"])
            probs.append((g, x_true, b))
        else:
            probs.append(_problem(i, 1.0, torch, oracle_data=False))
    geoms = [geometry(g) for g, _, _ in probs]
    bs = [torch.from_numpy(b).to(dev()) for _, _, b in probs]
    say(f"[batch] c4: {sum(g.n_vox for g, _, _ in probs) / 1e6:.1f} M voxels, "
        f"{sum(g.n_rays for g, _, _ in probs) / 1e6:.1f} M rays")
    batch = kct.Batch(geoms)
    xs, infos = batch.cgls(bs, K, graph=True)
    assert all(inf.iterations == K for inf in infos)
    sizes = [g.n_vox * g.n_views for g, _, _ in probs]
    subset = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), gold_i, *range(0, 48, 8)})
    for i in subset:
        x1, info1 = kct.cgls(geoms[i], bs[i], K)
        assert torch.equal(xs[i], x1), i
        assert infos[i].nb == info1.nb and infos[i].nb0 == info1.nb0, i
    idx = np.asarray(gold["idx"], dtype=np.int64)
    err = rel(to_np(xs[gold_i]).ravel()[idx], gold["x_idx"])
    say(f"[batch] c4: subset {subset} bitwise equal to separate solves; instance {gold_i} vs oracle rel {err:.3e}")
    assert err < 1e-4
    batch.close()


def test_batch_report_c4():
    """The batched workload: 48 seeded instances (64^3..192^3, 60-360 views,
    96^2..288^2 detectors, SID 400-700 mm, SDD 800-1400 mm), CGLS 20 iterations
    each, FP32.  The batched solve (tuned, graph replay) against the 48 separate
    solves one after another: per-instance latency inside the batch (device
    clock) and of the separate solves, p50 / p99, aggregate throughput, and the
    reconstruction error of both.  The batch must beat the separate solves at
    equal reconstruction error (median error against the phantoms within 1 %)."""
    import paper_2110_13526_amd as kct
    torch = torch_mod()
    K = 20
    say("[batch] c4 report: building 48 instances")
    probs = [_problem(i, 1.0, torch, oracle_data=False) for i in range(48)]
    geoms = [geometry(g) for g, _, _ in probs]
    bs = [torch.from_numpy(b).to(dev()) for _, _, b in probs]
    batch = kct.Batch(geoms)
    t = time.perf_counter()
    batch.tune()
    t_tune = time.perf_counter() - t
    batch.cgls(bs, 2)  # warm-up (records the graph)
    torch.cuda.synchronize()
    t = time.perf_counter()
    xs, infos = batch.cgls(bs, K, graph=True)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t
    lat_b = np.array(batch.latencies())
    errs_b = [rel(to_np(x), x_true) for x, (_, x_true, _) in zip(xs, probs)]
    # separate solves, one after another (each one's latency)
    lat = []
    errs_s = []
    for G, b in zip(geoms, bs):
        kct.cgls(G, b, 1)
    torch.cuda.synchronize()
    for (g, x_true, _), G, b in zip(probs, geoms, bs):
        t = time.perf_counter()
        x, _ = kct.cgls(G, b, K)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t)
        errs_s.append(rel(to_np(x), x_true))
    lat = np.array(lat)
    rep = {"instances": 48, "iterations": K, "batched_wall_s": t_batch, "tune_s": t_tune,
           "batched_latency_p50_s": float(np.percentile(lat_b, 50)),
           "batched_latency_p99_s": float(np.percentile(lat_b, 99)),
           "batched_instances_per_s": 48 / t_batch, "batched_iterations_per_s": 48 * K / t_batch,
           "separate_total_s": float(lat.sum()), "separate_p50_s": float(np.percentile(lat, 50)),
           "separate_p99_s": float(np.percentile(lat, 99)), "separate_instances_per_s": 48 / float(lat.sum()),
           "speedup_aggregate": float(lat.sum()) / t_batch,
           "voxels_total": int(sum(g.n_vox for g, _, _ in probs)), "rays_total": int(sum(g.n_rays for g, _, _ in probs)),
           "rel_error_vs_phantom_median_batched": float(np.median(errs_b)),
           "rel_error_vs_phantom_median_separate": float(np.median(errs_s)),
           "rel_error_max_ratio_batched_to_separate": float(max(b / s for b, s in zip(errs_b, errs_s)))}
    say("[batch] c4 " + json.dumps(rep))
    assert all(i.iterations == K for i in infos)
    assert rep["speedup_aggregate"] > 1.0
    assert abs(rep["rel_error_vs_phantom_median_batched"] / rep["rel_error_vs_phantom_median_separate"] - 1) <= 0.01
    assert np.all(lat_b > 0) and np.all(lat_b <= t_batch)
    batch.close()
