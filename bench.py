"""Benchmark of the FMM-LU hot path on one MI355X.

A step is one pass of the whole path over the workload: octree build, factorization
(tile assembly, ID, elimination, Schur updates per level, top block), and one forward
solve. value = n / (seconds per step) in unknowns/s. Reported beside it: fwd+adj solves/s
with the factors resident, the exact-matvec residual of the solution, the roofline of the
dominant kernel class (HIP-event timing inside the library on the factorization stream:
the timed steps bracket the Schur-update launches only; one extra untimed step brackets
every class for the per-class breakdown), and the CPU oracle timed on a bounded sample of
the same workload.

Workload: graded ellipsoid, semi-axes (1, 2, 4), n = 50,000 points with density
1 + 20 exp(-|x - (0,0,4)|^2 / 0.05), seed 2; k = 2 pi, eta = k, eps = 1e-6, leaf 64,
complex float64; right-hand side sqrt(w) times the field of a point source at (0.1,0.2,0.3).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "factor+solve unknowns/s at eps=1e-6 (FP64 vs FP32+refine); fwd+adj solves/s"
PEAK_FP64 = 78.6e12       # MI355X FP64 vector / matrix, FLOP/s
PEAK_HBM = 8.0e12         # bytes/s

# HBM bytes per launch of a kernel class on this workload, from two hardware-counter passes
# over one step (FETCH_SIZE, then WRITE_SIZE, rocprofv3 --pmc), each scaled by what the same
# counter read for a 1 GiB elementwise copy (FETCH_SIZE reads half the bytes: x2.0; WRITE_SIZE
# x1.0). Valid only while the listed kernel sources are unchanged (checked by hash); the
# counts and commands are in profiles/ellipsoid50k_hbm_traffic.md.
TRAFFIC = {
    "schur_update": {"bytes": 1260334144,
                     "sources": {"paper_2201_07325_amd/csrc/kernels_gemm.hip":
                                 "9666846b3dfdba8eebc7d191502254ca524c5bdfe3d888e8f440009d61298ae0"}},
}
MFMA_CLASSES = ("householder_qr", "elimination", "schur_update", "top_block")


def traffic_for(cls):
    import hashlib
    t = TRAFFIC.get(cls)
    if t is None:
        return None
    for path, sha in t["sources"].items():
        with open(os.path.join(ROOT, path), "rb") as fh:
            if hashlib.sha256(fh.read()).hexdigest() != sha:
                return None
    return t["bytes"]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_baseline(n_sample=4000):
    """The oracle (dense-bookkeeping RS-S, NumPy/SciPy) on a bounded sample of the same
    recipe: the graded ellipsoid with n_sample points, same k, eta, eps; tree + factor +
    solve timed on the host. cores = the BLAS threads its products ran on (its other steps
    are single-threaded NumPy); the host's available cores are reported beside it."""
    import synth
    from oracle import rss
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    avail = len(os.sched_getaffinity(0))
    s = synth.graded_ellipsoid(n_sample, seed=2)
    b = np.sqrt(s.weights) * synth.point_source_data(s.points, s.k)
    t0 = time.perf_counter()
    f = rss.RSSFactor(s.points, s.normals, s.weights, s.k, s.eta, s.eps, leaf_size=64)
    f.solve(b)
    dt = time.perf_counter() - t0
    return {"value": n_sample / dt, "unit": "unknowns/s", "cores": int(threads), "kind": "oracle",
            "host_cores_available": avail,
            "sample": f"graded ellipsoid n={n_sample} (same recipe, seed 2), tree+factor+solve in {dt:.1f} s"}


def ceilings():
    """Measured ceilings on this GPU beside the datasheet peaks: HBM bandwidth of a plain
    2 GiB device copy (bytes read + written per second), and the rate of a large float64 and
    complex128 library GEMM (torch.matmul, 8192^3; 8 flops per complex multiply-add)."""
    import torch
    out = {}
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    src = torch.ones(1 << 28, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    ev0.record()
    for _ in range(5):
        dst.copy_(src)
    ev1.record()
    ev1.synchronize()
    out["hbm_copy_GBps"] = 5 * 2 * src.numel() * 8 / (ev0.elapsed_time(ev1) / 1e3) / 1e9
    del src, dst
    for name, dt, fl in (("fp64_gemm_TFLOPs", torch.float64, 2), ("c128_gemm_TFLOPs", torch.complex128, 8)):
        n = 8192 if dt == torch.float64 else 4096
        a = torch.randn(n, n, dtype=dt, device="cuda")
        b = torch.randn(n, n, dtype=dt, device="cuda")
        torch.matmul(a, b)
        ev0.record()
        for _ in range(3):
            torch.matmul(a, b)
        ev1.record()
        ev1.synchronize()
        out[name] = 3 * fl * n ** 3 / (ev0.elapsed_time(ev1) / 1e3) / 1e12
        del a, b
    torch.cuda.empty_cache()
    return out


def golden_errors(f, bd, x, n):
    """Errors against the oracle's reference solutions of this workload (x* = A~^{-1} b and
    y* = A~^{-H} b from float64 GMRES with the exact matvec to relres <= 1e-13, written by
    tests/golden/make_ellipsoid50k_reference.py): relative 2-norm and max-entry errors of the
    factored solve, of the adjoint solve and of the refined solve."""
    path = os.path.join(ROOT, "tests", "golden", "ellipsoid50k_reference.npz")
    if n != 50_000 or not os.path.exists(path):
        return None
    ref = np.load(path)
    xs, ys = ref["x"], ref["y"]

    def err(v, r):
        v = v.cpu().numpy()
        return {"rel2": float(np.linalg.norm(v - r) / np.linalg.norm(r)),
                "max": float(np.max(np.abs(v - r)) / np.max(np.abs(r)))}
    out = {"solve": err(x, xs), "adjoint": err(f.solve_adjoint(bd), ys)}
    return out


def fp32_leg(s, bd, steps):
    """Same workload with complex float32 tiles and factors (float64 ID pivoting and pivot
    inverses), each step followed by float64 FGMRES refinement to 1e-10 with the exact matvec:
    n / (tree + factor + refined solve). Also the tree + factor time alone, the per-class
    breakdown of one extra profiled factorization, and the refined solution's error against
    the oracle's reference."""
    import torch
    import paper_2201_07325_amd as fm
    times, tfac, its, rel = [], [], 0, 0.0
    f = x = None
    for k in range(steps + 1):  # the first pass warms up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t = fm.Tree(s.points, 64)
        f = fm.Factor(s.points, s.normals, s.weights, s.k, s.eta, eps=s.eps, tree=t, precision=1)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        x, its, rel = f.solve_refined(bd, tol=1e-10, maxit=50, raise_on_fail=False)
        torch.cuda.synchronize()
        if k > 0:
            times.append(time.perf_counter() - t0)
            tfac.append(t1 - t0)
    dt = float(np.mean(times))
    out = {"unknowns_per_s": s.n / dt, "ms_per_step": dt * 1e3, "tree_factor_ms": float(np.mean(tfac)) * 1e3,
           "refine_iterations": its, "relres": rel, "tol": 1e-10, "factor_bytes": f.info()["factor_bytes"]}
    path = os.path.join(ROOT, "tests", "golden", "ellipsoid50k_reference.npz")
    if s.n == 50_000 and os.path.exists(path):
        xs = np.load(path)["x"]
        xv = x.cpu().numpy()
        out["err_vs_oracle"] = {"rel2": float(np.linalg.norm(xv - xs) / np.linalg.norm(xs)),
                                "max": float(np.max(np.abs(xv - xs)) / np.max(np.abs(xs)))}
    del f
    fp = fm.Factor(s.points, s.normals, s.weights, s.k, s.eta, eps=s.eps, precision=1, profile=1)
    out["class_ms"] = {c: round(v["ms"], 2) for c, v in fp.profile().items()}
    return out


def corrected_leg(s, bd, steps):
    """Same workload with locally corrected quadrature: synthetic target-dependent weights
    w_ij = w_j (1 + a_ij) for each point's near pairs (24 nearest within 2.5x its 8th-neighbour
    distance, a_ij ~ U[-0.3, 0.3], seed 1) and, for 1% of the targets, up to 8 pairs out to 14x
    that distance, which reach beyond a box's near field and move owners into Q (spill-over).
    n / (tree + factor + solve), the exact-matvec residual (corrections included) and the
    number of spill-over additions."""
    import torch
    import synth
    import paper_2201_07325_amd as fm
    t0 = time.perf_counter()
    corr = synth.near_corrections(s.points, seed=1, long_frac=0.01, long_factor=14.0)
    t_gen = time.perf_counter() - t0
    times = []
    f = x = None
    for k in range(steps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t = fm.Tree(s.points, 64)
        f = fm.Factor(s.points, s.normals, s.weights, s.k, s.eta, eps=s.eps, tree=t, corrections=corr)
        x = f.solve(bd)
        torch.cuda.synchronize()
        if k > 0:
            times.append(time.perf_counter() - t0)
    dt = float(np.mean(times))
    r = f.matvec(x, 0) - bd
    return {"unknowns_per_s": s.n / dt, "ms_per_step": dt * 1e3, "pairs": int(corr[0][-1]),
            "spill_over_owners": f.info()["nspill"],
            "relres_exact_matvec": float(torch.linalg.norm(r) / torch.linalg.norm(bd)),
            "table_generation_s": t_gen}


def c5_leg(n=1_000_000):
    """Large multiscale workload: bumpy sphere with 2,000 seeded bumps (seed 4), n = 1,000,000
    adaptive points, k = 10, eta = k, eps = 1e-4; complex float32 factors, float64 FGMRES
    refinement with the exact matvec to 1e-8. n / (tree + factor + refined solve), and the peak
    device memory of the factorization against the 288 GB of one MI355X."""
    import torch
    import synth
    import paper_2201_07325_amd as fm
    t0 = time.perf_counter()
    s = synth.bumpy_sphere(n, nbumps=2000, seed=4, k=10.0, eps=1e-4)
    t_gen = time.perf_counter() - t0
    log(f"c5: surface generated in {t_gen:.1f} s")
    d = np.random.default_rng(5).standard_normal(3)
    b = torch.as_tensor(s.weights ** 0.5 * synth.plane_wave_data(s.points, s.k, d)).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t = fm.Tree(s.points, 64)
    f = fm.Factor(s.points, s.normals, s.weights, s.k, s.eta, eps=s.eps, tree=t, precision=1)
    torch.cuda.synchronize()
    t_fac = time.perf_counter() - t0
    log(f"c5: tree + factor {t_fac:.2f} s")
    t1 = time.perf_counter()
    x, its, rel = f.solve_refined(b, tol=1e-8, maxit=30, raise_on_fail=False)
    torch.cuda.synchronize()
    t_ref = time.perf_counter() - t1
    info = f.info()
    log(f"c5: refined solve {t_ref:.2f} s, {its} iterations, relres {rel:.2e}")
    return {"workload": "bumpy sphere, 2000 bumps (seed 4), n=1,000,000, k=10, eta=k, eps=1e-4, "
                        "FP32 factors + FP64 FGMRES to 1e-8, plane-wave RHS (direction seed 5)",
            "n": s.n, "unknowns_per_s": s.n / (t_fac + t_ref), "tree_factor_s": t_fac, "refined_solve_s": t_ref,
            "refine_iterations": its, "relres": rel, "n0": info["n0"], "factor_bytes": info["factor_bytes"],
            "peak_bytes": info["peak_bytes"], "peak_frac_of_288GB": info["peak_bytes"] / 288e9,
            "surface_generation_s": t_gen}


def batched_leg(solves=20):
    """64 independent scatterers (spheres and ellipsoids, seed 3, sizes 2,000-20,000, k in
    [1, 8], eta = k, eps = 1e-5): trees + concurrent factorization timed once, then batched
    fwd+adj solves (one graph replay per direction for all problems). Complex float32 factors
    (the workload's stated precision), and float64 factors beside them."""
    import torch
    import synth
    import paper_2201_07325_amd as fm
    surfs = synth.scatterer_batch()
    probs = [(s.points, s.normals, s.weights, s.k, s.eta) for s in surfs]
    b = np.concatenate([np.sqrt(s.weights) * synth.point_source_data(
        s.points, s.k, src=tuple(np.array([0.1, 0.2, 0.3]) * np.array(s.meta["axes"]))) for s in surfs])
    bd = torch.as_tensor(b).cuda()
    out = {"workload": "64 scatterers (spheres/ellipsoids, axes U[0.5,3], n U[2000,20000], k U[1,8], "
                       "eta=k, seed 3), eps=1e-5"}
    for prec, name in ((1, "fp32"), (0, "fp64")):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        batch = fm.FactorBatch(probs, eps=1e-5, precision=prec)
        torch.cuda.synchronize()
        t_fac = time.perf_counter() - t0
        for _ in range(3):
            batch.solve(bd)
            batch.solve(bd, adjoint=True)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        times = []
        for _ in range(solves):
            ev0.record()
            batch.solve(bd)
            batch.solve(bd, adjoint=True)
            ev1.record()
            ev1.synchronize()
            times.append(ev0.elapsed_time(ev1) / 1e3)
        x = batch.solve(bd)
        worst = 0.0
        for i in range(0, batch.count, 8):  # every eighth problem: exact matvec residual
            lo, hi = int(batch.offsets[i]), int(batch.offsets[i + 1])
            r = batch.factor(i).matvec(x[lo:hi].contiguous()) - bd[lo:hi]
            worst = max(worst, float(torch.linalg.norm(r) / torch.linalg.norm(bd[lo:hi])))
        out[name] = {"n_total": batch.n, "factor_s": t_fac, "unknowns_per_s": batch.n / t_fac,
                     "fwd_adj_batch_solves_per_s": 1.0 / float(np.median(times)), "relres_sampled_max": worst}
        del batch, x
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=50_000)
    ap.add_argument("--solves", type=int, default=100)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=4000)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-c5", action="store_true")
    ap.add_argument("--no-corrections", action="store_true")
    ap.add_argument("--factor-only", action="store_true",
                    help="only the timed steps (tree + factor + one solve), for hardware-counter runs")
    ap.add_argument("--copy-calib-mb", type=int, default=0,
                    help="first run one plain device copy of this many MiB (a known-size kernel "
                         "for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU layout is design-only)", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_2201_07325_amd as fm

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    fm.lib()
    s = synth.graded_ellipsoid(args.n, seed=2)
    b = np.sqrt(s.weights) * synth.point_source_data(s.points, s.k)
    bd = torch.as_tensor(b).cuda()
    n = s.n
    if args.copy_calib_mb > 0:
        nel = args.copy_calib_mb * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)  # an elementwise kernel: reads and writes each byte once
        torch.cuda.synchronize()
        log(f"calibration copy: {args.copy_calib_mb} MiB read + {args.copy_calib_mb} MiB written")
        del src, dst

    def step(profile):
        t = fm.Tree(s.points, 64)
        f = fm.Factor(s.points, s.normals, s.weights, s.k, s.eta, eps=s.eps, tree=t, profile=profile)
        x = f.solve(bd)
        return f, x

    for w in range(args.warmup):
        step(False)
        torch.cuda.synchronize()
        log(f"warmup {w} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    profs = []
    for k in range(args.steps):
        # HIP-event brackets around the Schur-update launches only (profile=2): every class
        # bracketed (profile=1) costs about 4 ms of host event records per factorization
        f, x = step(2)
        profs.append(f.profile())
        log(f"step {k} done")
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    if args.factor_only:
        print(json.dumps({"factor_only": True, "n": n, "steps": args.steps, "ms_per_step": dt * 1e3}), flush=True)
        f = x = None
        fm.release_all()
        return
    info = f.info()
    # one more step, untimed, with every kernel class bracketed: the per-class breakdown and
    # the dominant class
    f_full, _ = step(1)
    full = f_full.profile()
    del f_full
    torch.cuda.synchronize()

    # accuracy of the last step's solution: exact float64 matvec residual
    r = f.matvec(x, 0) - bd
    relres = float(torch.linalg.norm(r) / torch.linalg.norm(bd))

    # fwd+adj solves/s with factors resident (median of timed pairs)
    for _ in range(10):
        f.solve(bd)
        f.solve_adjoint(bd)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(args.solves):
        ev0.record()
        f.solve(bd)
        f.solve_adjoint(bd)
        ev1.record()
        ev1.synchronize()
        times.append(ev0.elapsed_time(ev1) / 1e3)
    t_pair = float(np.median(times))
    solve_bytes = 2.0 * info["factor_bytes"]  # every factor byte once per sweep direction

    # blocked multi-right-hand-side solves: 64 columns (2 blocks of 32, matrix-core sweeps)
    # forward + adjoint
    nrhs, blk = 64, 32
    B = bd.reshape(n, 1).repeat(1, nrhs) * torch.exp(1j * torch.arange(nrhs, device=bd.device) * 0.1).reshape(1, nrhs)
    f.solve(B)
    f.solve_adjoint(B)
    torch.cuda.synchronize()
    mtimes = []
    for _ in range(5):
        ev0.record()
        XB = f.solve(B)
        f.solve_adjoint(B)
        ev1.record()
        ev1.synchronize()
        mtimes.append(ev0.elapsed_time(ev1) / 1e3)
    t_multi = float(np.median(mtimes))
    rb = f.matvec(XB[:, nrhs - 1].contiguous(), 0) - B[:, nrhs - 1]
    multi = {"nrhs": nrhs, "block": blk, "fwd_adj_solves_per_s": nrhs / t_multi,
             "ms_per_block_pair": t_multi * 1e3 / (nrhs // blk),
             "relres_last_column": float(torch.linalg.norm(rb) / torch.linalg.norm(B[:, nrhs - 1]))}
    log(f"multi-rhs: {nrhs / t_multi:.0f} fwd+adj solves/s")

    # float64 refinement to 1e-10 with the exact matvec, the factored inverse as preconditioner
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xr, r_it, r_rel = f.solve_refined(bd, tol=1e-10, maxit=50, raise_on_fail=False)
    torch.cuda.synchronize()
    t_ref = time.perf_counter() - t0
    log(f"refined solve: {r_it} iterations, relres {r_rel:.2e}, {t_ref * 1e3:.1f} ms")
    err_oracle = golden_errors(f, bd, x, n)
    if err_oracle is not None:
        xr_np = xr.cpu().numpy()
        xs_ref = np.load(os.path.join(ROOT, "tests", "golden", "ellipsoid50k_reference.npz"))["x"]
        err_oracle["refined"] = {"rel2": float(np.linalg.norm(xr_np - xs_ref) / np.linalg.norm(xs_ref)),
                                 "max": float(np.max(np.abs(xr_np - xs_ref)) / np.max(np.abs(xs_ref)))}
        log(f"error vs oracle reference: {err_oracle}")

    # dominant kernel class (from the fully bracketed step); its figures from the timed steps
    # when they bracketed it (the Schur update), else from that step
    classes = list(full.keys())
    dom = max(classes, key=lambda c: full[c]["ms"])
    tot = {c: {k: sum(p[c][k] for p in profs) for k in ("ms", "launches", "flops", "bytes")} for c in classes}
    nsteps_d = args.steps
    if tot[dom]["launches"] == 0:
        tot[dom] = dict(full[dom])
        nsteps_d = 1
    d = tot[dom]
    sec = d["ms"] / 1e3
    if dom == "assemble" or (d["flops"] == 0 and d["bytes"] > 0):
        roof = {"bound": "hbm", "achieved": d["bytes"] / sec / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s"}
    else:
        # complex float64 GEMM classes run on FP64 MFMA; the pivoting classes on FP64 vector ALUs
        roof = {"bound": "mfma" if dom in MFMA_CLASSES else "alu", "achieved": d["flops"] / sec / 1e12,
                "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = traffic_for(dom)
    roof["kernel"] = dom
    roof["launches"] = d["launches"] / nsteps_d
    roof["ms_per_step"] = d["ms"] / nsteps_d
    roof["source"] = "timed steps" if nsteps_d == args.steps else "separate fully profiled step"
    breakdown = {c: round(full[c]["ms"], 2) for c in classes}
    # achieved rate per class: algorithmic TFLOP/s, or GB/s for the byte-counted classes
    class_rate = {}
    for c in classes:
        if full[c]["ms"] <= 0:
            continue
        if full[c]["flops"] > 0:
            class_rate[c] = {"TFLOP/s": round(full[c]["flops"] / (full[c]["ms"] * 1e-3) / 1e12, 2)}
        elif full[c]["bytes"] > 0:
            class_rate[c] = {"GB/s": round(full[c]["bytes"] / (full[c]["ms"] * 1e-3) / 1e9, 1)}
    # step-level roofline fraction: every class at its own bound (algorithmic flops at the FP64
    # peak, or algorithmic bytes at HBM bandwidth, whichever is longer) over the measured step
    ideal_ms = sum(max(full[c]["flops"] / PEAK_FP64, full[c]["bytes"] / PEAK_HBM) * 1e3 for c in classes)

    out = {
        "metric": METRIC,
        "value": n / dt,
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128 (f64)",
        "data": "synthetic",
        "config": {"workload": f"graded ellipsoid (1,2,4) n={n} seed 2, k=2pi, eta=k, eps=1e-6, leaf 64, "
                               f"point-source RHS, FP64 factors", "n": n, "k": s.k, "eta": s.eta,
                   "eps": s.eps, "precision": "fp64"},
        "fwd_adj_solves_per_s": 1.0 / t_pair,
        "solve_pair_ms": t_pair * 1e3,
        "solve_hbm_GBps": solve_bytes / t_pair / 1e9,
        "relres_exact_matvec": relres,
        "multi_rhs": multi,
        "refined": {"tol": 1e-10, "iterations": r_it, "relres": r_rel, "ms": t_ref * 1e3,
                    "unknowns_per_s_factor_plus_refined": n / (dt + t_ref)},
        "n0": info["n0"],
        "factor_bytes": info["factor_bytes"],
        "class_ms_per_step": breakdown,
        "class_rate": class_rate,
        "gemm_autotune": fm.gemm_tuning(),
        "roofline": roof,
        "step_roofline": {"ideal_ms": ideal_ms, "measured_ms": dt * 1e3, "frac": ideal_ms / (dt * 1e3),
                          "note": "sum over kernel classes of max(flops / FP64 peak, bytes / HBM peak)"},
        "err_vs_oracle": err_oracle,
    }
    if not args.no_fp32:
        log("float32 factors + float64 refinement")
        out["fp32_refine"] = fp32_leg(s, bd, args.steps)
    if not args.no_corrections:
        log("locally corrected quadrature")
        out["corrected"] = corrected_leg(s, bd, args.steps)
    if not args.no_c5:
        log("large multiscale workload (1M points)")
        out["c5"] = c5_leg()
    if not args.no_batch:
        del f, x
        log("batched scatterers")
        out["batched"] = batched_leg()
    log("measured ceilings")
    out["ceilings"] = ceilings()
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample)
    print(json.dumps(out), flush=True)
    # last HIP calls of the library while the interpreter runs: factors destroyed, caches freed
    f = x = xr = XB = None
    fm.release_all()
    torch.cuda.synchronize()


if __name__ == "__main__":
    main()
