"""Benchmark of the multigroup discrete-ordinates dose solve on one MI355X.

Headline workload: the axial scan -- water cylinder (35 cm diameter) in air on
a 64 x 64 x 16 grid of 0.6 cm voxels, 36 collimated point sources (20 deg fan
x 10 deg cone) every 10 deg on a 54 cm circle solved together as 36
right-hand sides, 19 groups over 10-120 keV with Kramers 120 kVp weights, S6
level-symmetric quadrature (48 directions), P3 scattering, source iteration to
1e-6 per group and per source.  A step is one whole solve (ray traces,
first-collision sources, every group's source iterations with sweeps and
moment maps, dose tally) with every input already resident on the device,
plus the summed dose written to a device buffer.

Prints one JSON line.  Metric: sweep cell x angle x group updates per second
over the whole solve, for the fastest precision whose dose stays within 1e-4
(L2, relative) of the FP64 solve of the same workload on the GPU.  Also
reports the sweep kernel's achieved HBM bandwidth (algorithmic bytes /
measured kernel time, HIP events on the solver's stream), the other workloads
(the 128 x 128 x 32 abdomen, the single-source cylinder, the superposed CT
scan, the ROI-dose gradient) and the FP64 CPU oracle timed on a bounded
sample of the headline workload.
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
BAR = 1e-4


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(prob, sources=None, threads=None):
    """FP64 oracle on the first `sources` sources of the same workload (every
    source's solve is independent of the others, so a prefix of the sources
    is a prefix of the whole job), on `threads` host threads (default: all
    it is given)."""
    import oracle

    k = prob.B if sources is None else min(sources, prob.B)
    threads = threads or oracle.default_threads()
    oracle.lib()
    t0 = time.perf_counter()
    r = oracle.solve(prob.phantom, prob.xs, prob.dirs, prob.weights, prob.L, prob.src_pos[:k], prob.src_axis[:k],
                     prob.fan_deg, prob.cone_deg, prob.group_w, tol=prob.tol, threads=threads)
    dt = time.perf_counter() - t0
    upd = float(r.iters.sum()) * prob.phantom.C * prob.N
    return {"value": upd / dt, "unit": "updates/s", "cores": threads, "kind": "oracle",
            "sample": (f"whole solves of the first {k} of the {prob.B} sources" if k < prob.B else
                       f"the whole solve, all {prob.B} source(s)")
                      + f" ({int(r.iters.sum())} source iterations, {dt:.1f} s wall, FP64 C oracle, "
                        + ("OpenMP over directions/voxels)" if threads > 1 else "one thread)")}


def sweep_roofline(res, C, workload):
    """Achieved HBM bandwidth of the sweep kernel: algorithmic bytes (read q,
    write psi per cell-direction update, plus the two class copies of sigma_t
    per launch) over the average launch time from HIP events."""
    s = 8 if res["precision"] == "fp64" else 4
    launches = res["sweep_launches_per_solve"]
    bytes_per_solve = res["sweep_updates_per_solve"] * 2 * s + launches * 2 * C * s
    avg_launch_ms = res["sweep_ms_timed_per_solve"] / res["sweep_launches_timed_per_solve"]
    achieved = bytes_per_solve / launches / (avg_launch_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(workload, res["precision"], streams=res.get("rhs_streams", 1),
                                        coupling=res.get("sweep_sync")),
            "kernel": "k_sweep", "avg_launch_ms": avg_launch_ms, "bytes_per_launch": bytes_per_solve / launches}


def fused_roofline(res, prob, workload):
    """Achieved HBM bandwidth of the fused iteration kernel (direction->moment
    map, combine, moment->direction map): algorithmic bytes per cell of one
    right-hand side and iteration -- read psi and write q (N values each), read
    the group source ext and write the moments (Nm values each), read the old
    phi_00, the material byte and the FP64 density -- over the average launch
    time from HIP events."""
    if not res.get("fused_maps") or not res.get("fused_launches_timed_per_solve"):
        return None
    s = 8 if res["precision"] == "fp64" else 4
    N, Nm = prob.N, (prob.L + 1) ** 2
    cell_iters = res["sweep_updates_per_solve"] / N
    launches = res["iteration_sets"] * res.get("rhs_streams", 1)   # one fused launch per set and stream
    bytes_per_solve = cell_iters * ((2 * N + 2 * Nm + 1) * s + 9)
    avg_launch_ms = res["fused_ms_timed_per_solve"] / res["fused_launches_timed_per_solve"]
    achieved = bytes_per_solve / launches / (avg_launch_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(workload, res["precision"], "k_dcm", res.get("rhs_streams", 1)),
            "kernel": "k_dcm", "avg_launch_ms": avg_launch_ms, "bytes_per_launch": bytes_per_solve / launches}


def timed_solves(solver, prob, precision, steps, warmup, tag, dose_dev, fixed=None, schedule=None, **extra):
    extra.setdefault("fuse_maps", FUSE.get(_ARGS_FUSE[0], 0))
    """warmup + steps solves (stream launches; HIP events around every
    PROFILE_EVERY-th sweep launch), each followed by the summed dose into a
    device buffer; wall time of the timed steps."""
    import numpy as np
    import torch

    from paper_1811_12391_amd import dctsn

    kw = dict(precision=precision, tol=prob.tol, fixed_iters=fixed, autotune=True, **extra)
    if schedule:
        parts = [int(x) for x in schedule.split(":")]
        kw.update(autotune=False, sweep_bk=parts[0], sweep_sync=parts[1])
        if len(parts) > 2:
            kw["sweep_rhs_chain" if parts[1] >= 9 else "sweep_chain"] = parts[2]
    for _ in range(warmup):
        solver.solve(**kw)
        dctsn.dose_dev(solver.h, dose_dev, summed=True)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(steps):
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
        "fused_ms_timed_per_solve": float(np.mean([s.fused_ms for s in stats])),
        "fused_launches_timed_per_solve": float(np.mean([s.fused_launches for s in stats])),
        "sweep_updates_per_solve": upd,
        "iterations": int(stats[-1].iters.sum()),
        "iters_per_group_max_over_sources": stats[-1].iters.max(0).tolist(),
        "fixed_iters": fixed is not None,
        "iteration_sets": int(stats[-1].iteration_sets),
        "sweep_schedule": {"z_layers_per_workgroup": int(stats[-1].sweep_bk),
                           "wave_coupling": COUPLINGS.get(int(stats[-1].sweep_sync), str(stats[-1].sweep_sync)),
                           "chained_directions": int(stats[-1].sweep_chain),
                           "chained_sources": int(stats[-1].sweep_rhs_chain),
                           "streams": int(stats[-1].rhs_streams)},
        "rhs_streams": int(stats[-1].rhs_streams),
        "sweep_sync": int(stats[-1].sweep_sync),
        "fused_maps": bool(stats[-1].fused_maps),
        "dose": dose,
    }
    _log(f"[bench] {tag}: {res['ms_per_step']:.2f} ms/solve wall, {res['device_ms_per_solve']:.2f} ms device, "
         f"sweep {1e3 * res['sweep_ms_timed_per_solve'] / res['sweep_launches_timed_per_solve']:.1f} us per launch "
         f"({res['sweep_launches_timed_per_solve']:.0f} of {res['sweep_launches_per_solve']:.0f} timed), "
         f"{res['updates_per_s']:.3e} updates/s")
    return res


def run_workload(name, precisions, steps, warmup, schedule=None):
    """Every precision of one workload; dose error of each against the FP64
    GPU solve of the same workload (when FP64 is among them)."""
    import numpy as np
    import torch

    from paper_1811_12391_amd import dctsn, inputs as I

    prob = I.make_problem(name)
    C, G = prob.phantom.C, prob.G
    stream = torch.cuda.current_stream()
    solver = dctsn.Solver(prob, device=0, stream=ct_stream(stream))
    dose_dev = torch.empty(C, dtype=torch.float64, device="cuda")
    results = {}
    try:
        for p in precisions:
            fixed = None
            if p == "fp32_bf16map":
                # bf16 map inputs leave a rounding floor above tol 1e-6; run them at
                # the iteration counts the FP32 solve needed
                src = results.get("fp32") or results.get("fp64")
                fixed = (np.array(src["iters_per_group_max_over_sources"], dtype=np.int32) if src
                         else np.full(G, 12, np.int32))
            results[p] = timed_solves(solver, prob, p, steps, warmup, f"{name} {p}", dose_dev, fixed, schedule)
            if results[p]["rhs_streams"] == 2:
                # the same solve on one stream: the kernels' own rates, without the
                # other half's launches beside them
                results[p]["one_stream"] = timed_solves(solver, prob, p, steps, warmup, f"{name} {p} one stream",
                                                        dose_dev, fixed, schedule, rhs_streams=1)
    finally:
        solver.close()
    ref = results["fp64"]["dose"] if "fp64" in results else None
    for r in results.values():
        if ref is not None:
            r["dose_l2_rel_err_vs_fp64"] = float(np.linalg.norm(r["dose"] - ref) / np.linalg.norm(ref))
        for rr in [r] + ([r["one_stream"]] if "one_stream" in r else []):
            kernels = [sweep_roofline(rr, C, name)]
            fr = fused_roofline(rr, prob, name)
            if fr is not None:
                kernels.append(fr)
            for k in kernels:
                k["streams"] = rr["rhs_streams"]
            # the dominant kernel: the longest average launch
            rr["roofline_kernels"] = kernels
            rr["roofline"] = max(kernels, key=lambda k: k["avg_launch_ms"])
        if "one_stream" in r:
            r["one_stream"].pop("dose", None)
            # both kernels' algorithmic bytes over the device time of the solve: what
            # the two streams move together
            tot = sum(k["bytes_per_launch"] * n for k, n in
                      zip(r["roofline_kernels"], (r["sweep_launches_per_solve"],
                                                  r["iteration_sets"] * r["rhs_streams"])))
            ach = tot / (r["device_ms_per_solve"] * 1e-3) / 1e9
            r["roofline_aggregate"] = {"kernels": "k_sweep + k_dcm", "bytes_per_solve": tot,
                                       "device_ms_per_solve": r["device_ms_per_solve"], "achieved": ach,
                                       "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS}
    return prob, results


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precisions", default="fp64,fp32")
    ap.add_argument("--workload", default="c4", choices=["c1", "c2", "c3", "c4", "c5"],
                    help="configuration of the headline line (the metric is quoted on c4, the largest "
                         "single-GPU job; the others are for profiling)")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the other workloads and forms reported beside the headline")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 256 MiB device copy (reference dispatch for HBM byte counters)")
    ap.add_argument("--fuse", default="auto", choices=["auto", "on", "off"],
                    help="maps and combine as one kernel per iteration (auto: by shape)")
    ap.add_argument("--schedule", default=None, metavar="BK:SYNC",
                    help="pin the sweep schedule of the timed solves (z layers per workgroup : wave "
                         "coupling [: chained directions, or chained sources for couplings 9 / 10]) instead "
                         "of autotuning; for counter runs, where "
                         "the profiler's serialisation can change the tuner's choice")
    args = ap.parse_args()
    _ARGS_FUSE[0] = args.fuse
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): sharding the solve over several "
              "GPUs (right-hand sides, then z slabs) is not built", file=sys.stderr)
        sys.exit(2)

    import torch

    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    precs = [p for p in args.precisions.split(",") if p]
    prob, results = run_workload(args.workload, precs, args.steps, args.warmup, args.schedule)
    C, G, N = prob.phantom.C, prob.G, prob.N
    # headline: fastest precision meeting the dose-error bar
    ok = [p for p, r in results.items() if r.get("dose_l2_rel_err_vs_fp64", 0.0) <= BAR]
    best = max(ok, key=lambda p: results[p]["updates_per_s"])
    hb = results[best]
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
        "dtype": {"fp64": "f64", "fp32": "f32", "fp32_bf16map": "f32+bf16", "fp32_bf16x3": "f32+bf16x3"}[best],
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload],
                   "voxels": C, "groups": G, "directions": N, "legendre_order": prob.L, "sources": prob.B,
                   "precision": best},
        "roofline": hb["roofline"],
        "roofline_kernels": hb["roofline_kernels"],
        # with the sources in two halves on two streams the launches above overlap the
        # other half's; the same solve on one stream gives the kernels' own rates
        "roofline_one_stream": hb.get("one_stream", {}).get("roofline"),
        "roofline_aggregate": hb.get("roofline_aggregate"),
        "variants": {p: {k: v for k, v in r.items() if k != "dose"} for p, r in results.items()},
    }
    if not args.no_forms:
        line["forms"] = other_forms(args)
    if not args.no_cpu_baseline:
        _log("[bench] timing the FP64 CPU oracle on a bounded sample")
        line["cpu_baseline"] = cpu_baseline(prob, CPU_SOURCES.get(args.workload))
        if args.workload in CPU_SOURCES_1T:
            # the same oracle on one core: the single-threaded form of the baseline
            _log("[bench] timing the FP64 CPU oracle on one thread")
            line["cpu_baseline_single_thread"] = cpu_baseline(prob, CPU_SOURCES_1T[args.workload], threads=1)
    print(json.dumps(line), flush=True)


def other_forms(args):
    """The other workloads and forms of the solve, each against the same
    workload in FP64 on the GPU: the 128 x 128 x 32 abdomen (one source, S8,
    converged FP32 solve), the single-source 64 x 64 x 16 cylinder (S8; FP64,
    FP32 and bf16 map inputs), the headline workload replayed from a HIP
    graph, the 16-beam CT scan superposed into one collided solve (FP32 at
    the FP64 solve's iteration counts), and the ROI-dose gradient on the
    64 x 64 x 16 abdomen (FP32 forward + adjoint)."""
    import numpy as np
    import torch

    from paper_1811_12391_amd import dctsn, inputs as I

    out = {}

    def summary(name, results):
        return {"workload": WORKLOADS[name],
                "variants": {p: {k: v for k, v in r.items() if k != "dose"} for p, r in results.items()}}

    reps = max(1, min(args.steps, 3))
    for name, precs in (("c3", ["fp64", "fp32"]), ("c2", ["fp64", "fp32", "fp32_bf16map", "fp32_bf16x3"])):
        _, res = run_workload(name, precs, reps, 1)
        out[name] = summary(name, res)
    # the headline workload with its iteration sets replayed from a HIP graph
    prob = I.make_problem(args.workload)
    s = dctsn.Solver(prob)
    try:
        kw = dict(precision="fp32", tol=prob.tol, autotune=True, use_graph=True, chunk=8)
        s.solve(**kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            st = s.solve(**kw)
        wall = (time.perf_counter() - t0) / reps
        upd = float(st.iters.sum()) * prob.phantom.C * prob.N
        out["headline_graph_replay"] = {
            "workload": WORKLOADS[args.workload], "precision": "fp32", "ms_per_solve": 1e3 * wall,
            "updates_per_s": upd / wall, "iteration_sets": int(st.iteration_sets),
            "sweep_schedule": {"z_layers_per_workgroup": int(st.sweep_bk),
                               "wave_coupling": COUPLINGS.get(int(st.sweep_sync), str(st.sweep_sync))},
        }
        _log(f"[bench] {args.workload} fp32 graph replay: {1e3 * wall:.1f} ms/solve, {upd / wall:.3e} updates/s")
    finally:
        s.close()
    # within-group acceleration (Anderson, depth 2) against plain source
    # iteration, on the strongly scattering 4-group cylinder and on the headline
    # workload; and a scan solved position by position, cold and warm started
    def accel_case(name, precision, reps_):
        p_ = I.make_problem(name)
        s_ = dctsn.Solver(p_)
        res_ = {}
        try:
            for m in (0, 2):
                kw = dict(precision=precision, tol=p_.tol, autotune=True, accel_depth=m)
                s_.solve(**kw)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps_):
                    st = s_.solve(**kw)
                wall = (time.perf_counter() - t0) / reps_
                res_[m] = (wall, st, s_.dose(summed=True))
        finally:
            s_.close()
        (w0, st0, d0), (w2, st2, d2) = res_[0], res_[2]
        return {"workload": WORKLOADS[name], "precision": precision,
                "plain": {"ms_per_solve": 1e3 * w0, "iterations": int(st0.iters.sum()),
                          "fused_maps": bool(st0.fused_maps)},
                "anderson_depth_2": {"ms_per_solve": 1e3 * w2, "iterations": int(st2.iters.sum()),
                                     "fused_maps": bool(st2.fused_maps)},
                "summed_dose_l2_rel_diff": float(np.linalg.norm(d2 - d0) / np.linalg.norm(d0))}

    out["accelerated_c1_fp64"] = accel_case("c1", "fp64", reps)
    out["accelerated_c4_fp32"] = accel_case("c4", "fp32", 1)
    for k_, v_ in (("c1", out["accelerated_c1_fp64"]), ("c4", out["accelerated_c4_fp32"])):
        _log(f"[bench] {k_} accelerated: plain {v_['plain']['iterations']} iterations "
             f"{v_['plain']['ms_per_solve']:.1f} ms, Anderson {v_['anderson_depth_2']['iterations']} iterations "
             f"{v_['anderson_depth_2']['ms_per_solve']:.1f} ms")
    prob = I.make_problem("c4")
    scan = {}
    for warm in (False, True):
        one = I.Problem("c4_one", prob.phantom, prob.xs, prob.dirs, prob.weights, prob.L, prob.src_pos[:1],
                        prob.src_axis[:1], prob.fan_deg, prob.cone_deg, prob.group_w)
        s = dctsn.Solver(one)
        try:
            s.solve(precision="fp32", tol=prob.tol, autotune=True)
            torch.cuda.synchronize()
            n_it, t0 = 0, time.perf_counter()
            for p_ in range(prob.B):
                dctsn.set_source(s.h, 1, prob.src_pos[p_:p_ + 1], prob.src_axis[p_:p_ + 1], prob.fan_deg,
                                 prob.cone_deg, prob.group_w)
                st = s.solve(precision="fp32", tol=prob.tol, autotune=True, warm_start=warm)
                n_it += int(st.iters.sum())
            wall = time.perf_counter() - t0
        finally:
            s.close()
        scan["warm" if warm else "cold"] = {"ms_total": 1e3 * wall, "iterations": n_it}
    out["sequential_scan_warm_start"] = {
        "workload": "the 36 positions of the axial scan solved one after the other (one source per solve), "
                    "FP32, S6, P3, tol 1e-6", **scan}
    _log(f"[bench] sequential scan: cold {scan['cold']['iterations']} iterations {scan['cold']['ms_total']:.0f} ms, "
         f"warm {scan['warm']['iterations']} iterations {scan['warm']['ms_total']:.0f} ms")
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
# sources of the headline workload the CPU oracle solves for its baseline
# (about 10-20 s of host time)
CPU_SOURCES = {"c4": 6}
CPU_SOURCES_1T = {"c4": 1}   # about 25 s of one core
COUPLINGS = {1: "lds_counters", 2: "barrier", 3: "pipelined_blocks", 4: "layered_waves_4", 5: "layered_waves_2",
             6: "chained_directions_1", 7: "chained_directions_2", 8: "chained_directions_4",
             9: "chained_sources_2", 10: "chained_sources_1"}
FUSE = {"auto": 0, "on": 1, "off": -1}
_ARGS_FUSE = ["auto"]
SWEEP_SRC = os.path.join(ROOT, "paper_1811_12391_amd", "csrc", "k_sweep.hip")
FUSED_SRC = os.path.join(ROOT, "paper_1811_12391_amd", "csrc", "k_source.hip")


def measured_traffic(workload, precision, kernel="k_sweep", streams=1, coupling=None):
    """HBM bytes per sweep launch (FETCH_SIZE + WRITE_SIZE, scaled by the
    same counters on a plain copy of known size) from the committed counter
    summary of that workload, or None when there is none for this precision,
    the kernel's source has changed since the counters were taken, or they
    were taken with launches over a different share of the right-hand sides
    (one or two streams) or, for the sweep, another wave coupling."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    src = SWEEP_SRC if kernel == "k_sweep" else FUSED_SRC
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    if kv.get(f"{kernel}_sha256") != sha or int(kv.get("streams", "1")) != streams:
        return None
    if coupling is not None and "coupling" in kv and int(kv["coupling"]) != coupling:
        return None
    v = kv.get(f"bytes_per_launch_{precision}")
    return float(v) if v is not None else None


def ct_stream(stream):
    import ctypes

    return ctypes.c_void_p(stream.cuda_stream)


if __name__ == "__main__":
    main()
