"""Benchmark of the multigroup discrete-ordinates dose solve on one MI355X.

Workload: water cylinder (35 cm diameter) in air on a 64 x 64 x 16 grid of
0.6 cm voxels, one collimated point source 54 cm from the axis (20 deg fan x
10 deg cone), 19 groups over 10-120 keV with Kramers 120 kVp weights, S8
level-symmetric quadrature (80 directions), P3 scattering, source iteration
to 1e-6 per group.  A step is one whole solve (ray trace, first-collision
source, every group's source iterations with sweeps and moment maps, dose
tally) with every input already resident on the device, plus the dose
written to a device buffer.

Prints one JSON line.  Metric: sweep cell x angle x group updates per second
over the whole solve, for the fastest precision whose dose stays within 1e-4
(L2, relative) of the FP64 solve.  Also reports the sweep kernel's achieved
HBM bandwidth (algorithmic bytes / measured kernel time) and the FP64 CPU
oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sweep cell·angle·group updates/s + ms/solve at ≤1e-4 rel dose err vs FP64"
HBM_PEAK_GBS = 8000.0


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(prob, groups=None):
    """FP64 oracle on the first `groups` groups of the same workload (all of
    them by default; groups only couple downward, so a prefix is exactly the
    first part of the full solve), all host threads it is given."""
    import numpy as np

    import oracle
    from paper_1811_12391_amd import inputs as I

    xs = prob.xs
    groups = prob.G if groups is None else groups
    sub = xs if groups == prob.G else I.XSTables(edges=xs.edges[: groups + 1], sigma_t=xs.sigma_t[:, :groups].copy(),
                     sigma_s=xs.sigma_s[:, :, :groups, :groups].copy(), kerma=xs.kerma[:, :groups].copy(),
                     cutoff=xs.cutoff[:, :groups].copy(), names=xs.names, Z=xs.Z)
    threads = oracle.default_threads()
    oracle.lib()
    t0 = time.perf_counter()
    r = oracle.solve(prob.phantom, sub, prob.dirs, prob.weights, prob.L, prob.src_pos, prob.src_axis,
                     prob.fan_deg, prob.cone_deg, prob.group_w[:groups], tol=prob.tol, threads=threads)
    dt = time.perf_counter() - t0
    upd = float(r.iters.sum()) * prob.phantom.C * prob.N
    return {"value": upd / dt, "unit": "updates/s", "cores": threads, "kind": "oracle",
            "sample": (f"the whole solve, all {prob.G} groups" if groups == prob.G else
                       f"first {groups} of {prob.G} groups of the same solve")
                      + f" ({int(r.iters.sum())} source iterations, {dt:.1f} s wall, FP64 C oracle, "
                        f"OpenMP over directions/voxels)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precisions", default="fp64,fp32,fp32_bf16map")
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4", "c5"],
                    help="configuration to time (the headline metric is quoted on c2; the others are for profiling)")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the batched axial-scan and adjoint forms (reported beside the headline)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 256 MiB device copy (reference dispatch for HBM byte counters)")
    ap.add_argument("--schedule", default=None, metavar="BK:SYNC",
                    help="pin the sweep schedule of the timed solves (z layers per workgroup : wave "
                         "coupling) instead of autotuning; for counter runs, where the profiler's "
                         "serialisation can change the tuner's choice")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): sharding the solve over several "
              "GPUs (right-hand sides, then z slabs) is not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1811_12391_amd import dctsn, inputs as I

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.copy_calibration:
        src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    prob = I.make_problem(args.workload)
    C, G, N = prob.phantom.C, prob.G, prob.N
    solver = dctsn.Solver(prob, device=0, stream=ct_stream(stream))
    dose_dev = torch.empty(C, dtype=torch.float64, device="cuda")

    def run(precision, steps, warmup, tag, fixed=None):
        kw = dict(precision=precision, tol=prob.tol, fixed_iters=fixed, autotune=True)
        if args.schedule:
            bk, sync = (int(x) for x in args.schedule.split(":"))
            kw.update(autotune=False, sweep_bk=bk, sweep_sync=sync)
        for _ in range(warmup):
            solver.solve(**kw)
            dctsn.dose_dev(solver.h, dose_dev, summed=True)
        torch.cuda.synchronize()
        stats = []
        t0 = time.perf_counter()
        for _ in range(steps):
            # HIP events around every PROFILE_EVERY-th sweep launch (a sample
            # over all groups; fewer events disturb the timed solve less)
            stats.append(solver.solve(profile=PROFILE_EVERY, **kw))
            dctsn.dose_dev(solver.h, dose_dev, summed=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        dose = dose_dev.cpu().numpy().copy()
        upd = float(np.mean([s.sweep_updates for s in stats]))
        res = {
            "precision": precision,
            "ms_per_step": 1e3 * wall / steps,
            "updates_per_s": upd * steps / wall,
            "device_ms_per_solve": float(np.mean([s.solve_ms for s in stats])),
            "sweep_ms_timed_per_solve": float(np.mean([s.sweep_ms for s in stats])),
            "sweep_launches_per_solve": float(np.mean([s.sweep_launches_all for s in stats])),
            "sweep_launches_timed_per_solve": float(np.mean([s.sweep_launches for s in stats])),
            "sweep_updates_per_solve": upd,
            "iterations": int(stats[-1].iters.sum()),
            "iters_per_group": stats[-1].iters[0].tolist(),
            "fixed_iters": fixed is not None,
            "iteration_sets": int(stats[-1].iteration_sets),
            "sweep_schedule": {"z_layers_per_workgroup": int(stats[-1].sweep_bk),
                               "wave_coupling": {1: "lds_counters", 2: "barrier",
                                                  3: "pipelined_blocks", 4: "layered_waves_4",
                                                  5: "layered_waves_2"}[int(stats[-1].sweep_sync)]},
            "dose": dose,
        }
        _log(f"[bench] {tag}: {res['ms_per_step']:.2f} ms/solve wall, {res['device_ms_per_solve']:.2f} ms device, "
             f"sweep {1e3 * res['sweep_ms_timed_per_solve'] / res['sweep_launches_timed_per_solve']:.1f} us per launch "
             f"({res['sweep_launches_timed_per_solve']:.0f} of {res['sweep_launches_per_solve']:.0f} timed), "
             f"{res['updates_per_s']:.3e} updates/s")
        return res

    precs = [p for p in args.precisions.split(",") if p]
    results = {}
    for p in precs:
        fixed = None
        if p == "fp32_bf16map":
            # bf16 map inputs leave a rounding floor above tol 1e-6; run them at
            # the iteration counts the FP32 solve needed
            src = results.get("fp32") or results.get("fp64")
            fixed = np.array(src["iters_per_group"], dtype=np.int32) if src else np.full(G, 12, np.int32)
        results[p] = run(p, args.steps, args.warmup, p, fixed)
    ref = results["fp64"]["dose"] if "fp64" in results else None
    for p, r in results.items():
        if ref is not None:
            r["dose_l2_rel_err_vs_fp64"] = float(np.linalg.norm(r["dose"] - ref) / np.linalg.norm(ref))
    # headline: fastest precision meeting the dose-error bar
    ok = [p for p, r in results.items() if r.get("dose_l2_rel_err_vs_fp64", 0.0) <= 1e-4]
    best = max(ok, key=lambda p: results[p]["updates_per_s"])
    hb = results[best]
    s = 8 if best == "fp64" else 4
    # algorithmic bytes of the sweep: read q, write psi per update, plus the
    # two class copies of sigma_t per cell per launch
    launches = hb["sweep_launches_per_solve"]
    bytes_per_solve = hb["sweep_updates_per_solve"] * 2 * s + launches * 2 * C * s
    avg_launch_ms = hb["sweep_ms_timed_per_solve"] / hb["sweep_launches_timed_per_solve"]
    achieved = bytes_per_solve / launches / (avg_launch_ms * 1e-3) / 1e9
    line = {
        "metric": METRIC,
        "value": hb["updates_per_s"],
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": hb["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp32_bf16map": "f32+bf16"}[best],
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload],
                   "voxels": C, "groups": G, "directions": N, "legendre_order": prob.L, "sources": prob.B,
                   "precision": best},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(best) if args.workload == "c2" else None,
                     "kernel": "k_sweep", "avg_launch_ms": avg_launch_ms,
                     "bytes_per_launch": bytes_per_solve / launches},
        "variants": {p: {k: v for k, v in r.items() if k != "dose"} for p, r in results.items()},
    }
    if not args.no_forms:
        solver.close()
        solver = None
        line["forms"] = other_forms(args)
    if not args.no_cpu_baseline:
        _log("[bench] timing the FP64 CPU oracle on a bounded sample")
        line["cpu_baseline"] = cpu_baseline(prob)
    if solver is not None:
        solver.close()
    print(json.dumps(line), flush=True)


def other_forms(args):
    """The batched, superposed and differentiated forms of the solve, each
    against the same form in FP64 on the GPU: the 36-source axial scan (FP32,
    autotuned, graph replay), the 16-beam CT scan superposed into one
    collided solve (FP32 at the FP64 solve's iteration counts), and the
    ROI-dose gradient on the 64x64x16 abdomen (FP32 forward + adjoint)."""
    import numpy as np
    import torch

    from paper_1811_12391_amd import dctsn, inputs as I

    out = {}
    # axial scan: 36 right-hand sides in one solve
    prob = I.make_problem("c4")
    s = dctsn.Solver(prob)
    try:
        s.solve(precision="fp64", tol=prob.tol)
        ref = s.dose(summed=True)
        kw = dict(precision="fp32", tol=prob.tol, autotune=True, use_graph=True, chunk=8)
        s.solve(**kw)
        torch.cuda.synchronize()
        reps = max(1, min(args.steps, 3))
        t0 = time.perf_counter()
        for _ in range(reps):
            st = s.solve(**kw)
        wall = (time.perf_counter() - t0) / reps
        d = s.dose(summed=True)
        upd = float(st.iters.sum()) * prob.phantom.C * prob.N
        out["axial_scan_batched"] = {
            "workload": "c2 cylinder, 36 sources every 10 deg on a 54 cm circle, 19 groups, S6 (48 dirs), P3",
            "precision": "fp32", "ms_per_solve": 1e3 * wall, "updates_per_s": upd / wall,
            "sweep_schedule": {"z_layers_per_workgroup": int(st.sweep_bk), "coupling": int(st.sweep_sync)},
            "summed_dose_l2_rel_err_vs_fp64_gpu": float(np.linalg.norm(d - ref) / np.linalg.norm(ref)),
        }
        _log(f"[bench] axial scan (36 sources) fp32: {1e3 * wall:.1f} ms/solve, {upd / wall:.3e} updates/s")
    finally:
        s.close()
    # CT scan as 16 concurrent cone beams superposed into one collided solve,
    # beside one beam alone and the 16 beams as separate right-hand sides
    prob = I.make_problem("ct16")
    one = I.Problem("ct16_one", prob.phantom, prob.xs, prob.dirs, prob.weights, prob.L, prob.src_pos[:1],
                    prob.src_axis[:1], prob.fan_deg, prob.cone_deg, prob.group_w)
    reps = max(1, min(args.steps, 3))

    def timed(p, **kw):
        s = dctsn.Solver(p)
        try:
            s.solve(**kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                st = s.solve(**kw)
            wall = (time.perf_counter() - t0) / reps
            return wall, st, s.dose(summed=True)
        finally:
            s.close()

    base = dict(autotune=True, use_graph=True, chunk=8)
    _, st64, ref = timed(prob, precision="fp64", tol=prob.tol, superpose=16, **base)
    # the three FP32 timings run the FP64 solve's per-group iteration counts,
    # so they do the same work (superposed, one beam, 16 separate)
    fi = st64.iters[0].astype(np.int32)
    w_sup, st, d = timed(prob, precision="fp32", fixed_iters=fi, superpose=16, **base)
    w_one, st1, _ = timed(one, precision="fp32", fixed_iters=fi, **base)
    w_sep, _, d_sep = timed(prob, precision="fp32", fixed_iters=fi, **base)
    upd = float(st.iters.sum()) * prob.phantom.C * prob.N
    out["ct_scan_superposed"] = {
        "workload": "c2 cylinder, 16 cone beams of 30 x 30 deg every 22.5 deg on a 54 cm circle, superposed "
                    "into one collided solve, 19 groups, S6 (48 dirs), P3",
        "precision": "fp32", "fixed_iters_from_fp64": fi.tolist(), "ms_per_solve": 1e3 * w_sup,
        "updates_per_s": upd / w_sup, "one_beam_ms_per_solve": 1e3 * w_one,
        "sixteen_separate_rhs_ms_per_solve": 1e3 * w_sep,
        "dose_l2_rel_err_vs_fp64_gpu": float(np.linalg.norm(d - ref) / np.linalg.norm(ref)),
        "superposed_vs_separate_dose_l2_rel_diff": float(np.linalg.norm(d - d_sep) / np.linalg.norm(d_sep)),
    }
    _log(f"[bench] CT scan, 16 beams superposed fp32: {1e3 * w_sup:.1f} ms/solve (one beam {1e3 * w_one:.1f} ms, "
         f"16 separate {1e3 * w_sep:.1f} ms)")
    # ROI-dose gradient
    prob = I.make_problem("c5")
    ph = prob.phantom
    roi = np.zeros((ph.nz, ph.ny, ph.nx))
    roi[6:10, 27:37, 27:37] = 1.0 / 400.0
    roi = roi.reshape(-1)
    s = dctsn.Solver(prob)
    try:
        s.solve(precision="fp64", tol=prob.tol, keep_adjoint=True)
        a64 = s.adjoint(roi, tol=prob.tol)
        res = {}
        for rep in range(2):
            t0 = time.perf_counter()
            st = s.solve(precision="fp32", tol=prob.tol, keep_adjoint=True, autotune=True)
            t1 = time.perf_counter()
            a32 = s.adjoint(roi, tol=prob.tol)
            t2 = time.perf_counter()
            res = {"forward_ms": 1e3 * (t1 - t0), "adjoint_ms": 1e3 * (t2 - t1)}
        l2 = lambda x, y: float(np.linalg.norm(x - y) / np.linalg.norm(y))
        out["roi_dose_gradient"] = {
            "workload": "64x64x16 abdomen, 19 groups, S6, P3, mean dose in the centred 10x10x4 ROI",
            "precision": "fp32", **res,
            "d_density_l2_rel_err_vs_fp64_gpu": l2(a32.d_density, a64.d_density),
            "d_group_w_l2_rel_err_vs_fp64_gpu": l2(a32.d_group_w, a64.d_group_w),
            "roi_dose_rel_err_vs_fp64_gpu": abs(a32.R - a64.R) / abs(a64.R),
        }
        _log(f"[bench] ROI gradient fp32: forward {res['forward_ms']:.1f} ms, adjoint {res['adjoint_ms']:.1f} ms")
    finally:
        s.close()
    return out


WORKLOADS = {
    "c1": "water cylinder d=35cm in air, 24x24x8 voxels @1.5cm, 1 point source 54cm (20x10 deg), 4 groups "
          "10-120keV Kramers, S4 (24 dirs), P1, tol 1e-6",
    "c2": "water cylinder d=35cm in air, 64x64x16 voxels @0.6cm, 1 point source 54cm (20x10 deg), 19 groups "
          "10-120keV Kramers, S8 (80 dirs), P3, tol 1e-6",
    "c3": "seeded abdomen phantom, 128x128x32 voxels @0.3cm, 1 point source 54cm (20x10 deg), 19 groups, "
          "S8 (80 dirs), P3, tol 1e-6",
    "c4": "water cylinder d=35cm in air, 64x64x16 voxels @0.6cm, 36 sources every 10 deg on a 54cm circle, "
          "19 groups, S6 (48 dirs), P3, tol 1e-6",
    "c5": "seeded abdomen phantom, 64x64x16 voxels @0.6cm, 1 point source 54cm, 19 groups, S6 (48 dirs), P3, "
          "tol 1e-6",
}
COPY_BYTES = 256 << 20
PROFILE_EVERY = 4
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_sweep_c2_hbm_traffic.txt")
SWEEP_SRC = os.path.join(ROOT, "paper_1811_12391_amd", "csrc", "k_sweep.hip")


def measured_traffic(precision):
    """HBM bytes per sweep launch (FETCH_SIZE + WRITE_SIZE, scaled by the
    same counters on a plain copy of known size) from the committed counter
    summary, or None when there is none for this precision or the sweep
    source has changed since the counters were taken."""
    import hashlib

    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    with open(SWEEP_SRC, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    if kv.get("k_sweep_sha256") != sha:
        return None
    v = kv.get(f"bytes_per_launch_{precision}")
    return float(v) if v is not None else None


def ct_stream(stream):
    import ctypes

    return ctypes.c_void_p(stream.cuda_stream)


if __name__ == "__main__":
    main()
