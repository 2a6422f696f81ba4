#!/usr/bin/env python3
"""Benchmark of the spin-F ground-state hot path on one MI355X.

Workload: spin-3, 3D, 128^3 grid on [-8,8]^3, V = (x^2 + y^2 + 4 z^2)/2,
beta = (500, 5, -5, 2), M = 0.2 (synthetic seeded inputs; no dataset).

A step is one Riemannian Hessian-vector product of the regularised Newton
model at a fixed point u, exactly as one truncated-CG iteration issues it:
the three spectral-Laplacian axis passes, the pointwise spin-3 Hessian terms,
the FP64 reductions for the tangent-space projection and <Z, HZ>, the
projection, and the host read-back of <Z, HZ>.  The headline value is HVPs/s
in mixed precision (c64 fields, FP64 reductions); the FP64 figure, both
rooflines, time-to-ground-state for both precisions (full newton_solve:
retraction, RGBB, ARNT, energies and gradients) and the CPU oracle timing
ride on the same JSON line.

The batched form (64 spin-1 2D problems of uneven grids in one gpe_batch:
one batched HVP pass against the same HVPs one by one, and with
--batch-solve the lock-step Newton solve against one-by-one solves) rides on
the same line under "batched".

    python bench.py [--gpus 1] [--steps 200] [--warmup 10] [--no-solve] [--no-cpu]
                    [--no-batch] [--batch-solve]
"""

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published

# VALU lane-operation peak of MI355X without packed FP32: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# (the published 78.6 TFLOP/s FP64 / non-packed FP32 vector rate, an FMA counting as 2 flops).
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12

# Per-launch counters of the dominant HVP kernel from rocprofv3 runs recorded in
# profiles/hvp_spin3_128_*.md: HBM bytes (FETCH_SIZE / WRITE_SIZE, copy-kernel
# calibrated) and VALU instructions (SQ_INSTS_VALU, per wavefront; x64 lanes),
# by schedule variant; valid only while the kernel sources hash to `src_hash`.
MEASURED = {
    "src_hash": "bad9f4f2b2109094",
    "hvp_xpass": {
        "traffic": {"fp64": {"0": 1106788223, "1": 1097933451, "2": 1088466717},
                    "mixed": {"0": 482389904, "1": 480248912, "2": 479403257}},
        "valu": {"fp64": {"0": 61161472, "1": 63971328, "2": 61128704},
                 "mixed": {"0": 64700416, "1": 63512576, "2": 60817408}},
    },
}


def kernel_src_hash():
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1907_01194_amd", "csrc")
    for f in ("lap.hip", "fft.h", "spin.h", "common.h"):
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=128, help="grid points per axis")
    ap.add_argument("--no-solve", action="store_true", help="skip time-to-ground-state")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle timing")
    ap.add_argument("--solve-time", type=float, default=45.0,
                    help="wall-clock cap per solve of the benchmark physics (s)")
    ap.add_argument("--precisions", default="mixed,fp64")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-HVP measurement")
    ap.add_argument("--batch-solve", action="store_true",
                    help="also time the lock-step batched solve of the 64 problems against one-by-one solves")
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--paper-tables", action="store_true",
                    help="only reproduce the ARNT rows of the Sec. 7.1 tables (every magnetization, R1/R2/R3)")
    ap.add_argument("--solve-only", action="store_true",
                    help="only the paper's spin-3 128^3 ground-state solve (for profiling the whole solve)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy kernel (reference for HBM counters)")
    return ap.parse_args()


def copy_calibration(log):
    """A plain device-to-device copy kernel of known size: read 256 MiB, write
    256 MiB, ten times.  Profiled with the same counters as the HVP kernels it
    gives the scale factor between counter readings and bytes."""
    import torch
    n = 1 << 26                                    # 64 Mi floats = 256 MiB
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty(n, dtype=torch.float32, device="cuda")
    for _ in range(10):
        torch.add(a, 1.0, out=b)                   # elementwise kernel: 256 MiB in, 256 MiB out
    torch.cuda.synchronize()
    log("copy calibration: 10 launches, %d bytes read and %d bytes written per launch" % (4 * n, 4 * n))


def kernel_bytes(kind, K, npts, cb, rb):
    """Algorithmic HBM bytes of one launch of each HVP kernel kind:
    cb = bytes per complex element, rb = bytes per real; one field = K*npts*cb."""
    f = K * npts * cb
    return {
        "hvp_xpass": 4 * f + npts * rb,  # read X, Z, LX, V; write W
        "lap_axis_y": 3 * f,             # read Z and W, write W
        "lap_axis_z": 4 * f,             # read Z, W and X (projection), write HZ
        "project": 3 * f,                # 1-D only: read X and W, write HZ
        "finalize": 0,
    }.get(kind)


def time_hvps(spec, prec, w, noise, steps, warmup, log):
    import torch
    from paper_1907_01194_amd.binding import Problem, R1
    gp = Problem(spec, prec)
    X = torch.from_numpy(w).cuda()
    u = gp.retract(X, None, 0.0, R1)                       # u = psi(w), on the manifold
    xi = gp.project(u, torch.from_numpy(noise).cuda())     # tangent direction
    nrm = np.sqrt(gp.constraints(xi)[0])
    xi /= nrm
    gp.set_point(u)
    Z = xi.to(gp.work_dtype).contiguous()
    HZ = gp.empty(work=True)
    for _ in range(warmup):
        gp.hvp_dot(Z, 1e-2, out=HZ)
    torch.cuda.synchronize()
    # the handle runs on torch's current stream, so these events bracket its work
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    # (1) the timed region: `steps` HVPs, nothing else on the stream
    e0.record(stream)
    t0 = time.perf_counter()
    kappa = 0.0
    for _ in range(steps):
        _, kappa = gp.hvp_dot(Z, 1e-2, out=HZ)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / steps
    # (2) the same HVPs again with the library's HIP events around every launch
    # (on the handle's stream): per-kernel durations for the breakdown and the roofline
    gp.timing(True)
    for _ in range(steps):
        gp.hvp_dot(Z, 1e-2, out=HZ)
    torch.cuda.synchronize()
    kt = gp.timing_read()
    gp.timing(False)
    sched = gp.schedule()
    log("%s: x-pass schedule variant %d (autotuned; us per variant %s)" % (prec, sched[0], sched[1]))
    log("%s: %.1f us per HVP (events), %.1f us (wall), kappa=%.6e; per-kernel pass (events around each launch):"
        % (prec, 1e3 * ms, 1e6 * wall / steps, kappa))
    for k, (c, t) in sorted(kt.items(), key=lambda x: -x[1][1]):
        log("   %-12s %6d launches  %9.1f us avg" % (k, c, 1e3 * t / c))
    del gp
    torch.cuda.empty_cache()
    return ms, kt, sched


def roofline(spec, prec, ms, kt, variant):
    """Roofline of the dominant kernel and of the whole HVP.  The fused x pass
    is VALU-bound when its counters are on record (its VALU lane-operation rate
    against VALU_PEAK_TOPS is then the headline fraction; its HBM rate rides
    along), else it is reported against HBM."""
    K = spec.K
    npts = int(np.prod(spec.n))
    cb, rb = (16, 8) if prec == "fp64" else (8, 4)
    # dominant kernel = largest total time among the HVP kernels
    cand = {k: v for k, v in kt.items() if kernel_bytes(k, K, npts, cb, rb)}
    dom = max(cand, key=lambda k: cand[k][1])
    cnt, tot = cand[dom]
    per_launch_s = tot / cnt / 1e3
    b = kernel_bytes(dom, K, npts, cb, rb)
    achieved = b / per_launch_s / 1e9
    hvp_bytes = 3 * K * npts * cb + npts * rb             # read X, Z, V; write HZ
    hvp_gbs = hvp_bytes / (ms / 1e3) / 1e9
    traffic = valu = None
    if npts == 128 ** 3 and K == 7 and kernel_src_hash() == MEASURED["src_hash"]:
        rec = MEASURED.get(dom, {})
        traffic = rec.get("traffic", {}).get(prec, {}).get(str(variant))
        valu = rec.get("valu", {}).get(prec, {}).get(str(variant))
    hbm = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic}
    if valu:
        ops = valu * 64
        tops = ops / per_launch_s / 1e12
        kern = {"bound": "alu", "achieved": round(tops, 2), "peak": round(VALU_PEAK_TOPS, 2),
                "unit": "TOP/s (VALU lane operations)", "frac": round(tops / VALU_PEAK_TOPS, 4),
                "traffic": traffic, "valu_lane_ops_per_launch": ops, "hbm": hbm}
    else:
        kern = dict(hbm)
    kern.update({"name": dom, "schedule_variant": variant, "bytes_per_launch": b,
                 "us_per_launch": round(per_launch_s * 1e6, 2)})
    return {
        "kernel": kern,
        "hvp": {"bound": "hbm", "achieved": round(hvp_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(hvp_gbs / HBM_PEAK_GBS, 4), "compulsory_bytes": hvp_bytes,
                "us_per_hvp": round(ms * 1e3, 2)},
    }


def time_solve(spec, prec, w, limit, log):
    """Time-to-ground-state: newton_solve from w (device-resident before the
    clock starts) to ||grad|| <= 1e-6, or until `limit` seconds."""
    import torch
    from paper_1907_01194_amd.binding import Problem
    gp = Problem(spec, prec)
    X = torch.from_numpy(w).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    X, st = gp.newton_solve(X, check=False, tol=1e-6, time_limit=limit)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log("solve %s %s: E=%.12f |g|=%.2e conv=%d rgbb=%d outer=%d cg=%d hvp=%d %.1fs" % (
        spec.name, prec, st["E"], st["gnorm"], st["converged"], st["rgbb_iters"], st["outer"], st["cg_total"],
        st["hvp_calls"], wall))
    del gp
    torch.cuda.empty_cache()
    return {"seconds": round(wall, 3), "E": st["E"], "gnorm": st["gnorm"], "converged": bool(st["converged"]),
            "rgbb_iters": st["rgbb_iters"], "outer": st["outer"], "cg_total": st["cg_total"],
            "hvp_calls": st["hvp_calls"], "t_rgbb": round(st["t_rgbb"], 3), "t_arnt": round(st["t_arnt"], 3)}


def batch_measure(count, steps, solve, log):
    """Batched form: `count` spin-1 2D problems of uneven grids (64^2, 128^2,
    256^2) and parameters in one gpe_batch.  Times one batched Riemannian HVP
    pass over all problems (one launch per kernel stage) against the same HVPs
    issued problem by problem, and optionally the lock-step Newton solve of
    all problems against solving them one at a time."""
    import torch
    from paper_1907_01194_amd import workloads as W
    from paper_1907_01194_amd.binding import Batch, Problem
    specs = W.spin1_2d_batch(count=count, seed=5)
    t0 = time.perf_counter()
    b = Batch(specs, "mixed")
    t_create = time.perf_counter() - t0
    sched = b.schedule()
    X0 = [torch.from_numpy(W.initial_state(sp, 60 + i)).cuda() for i, sp in enumerate(specs)]
    Z = []
    for i, (p, sp) in enumerate(zip(b.problems, specs)):
        u = p.retract(X0[i], None)
        d = p.project(u, torch.from_numpy(W.random_direction(sp, 200 + i)).cuda())
        d /= float(d.abs().pow(2).sum().sqrt())
        p.set_point(u)
        Z.append(d.to(p.work_dtype).contiguous())
    sig = [1e-2] * count
    HZ = [p.empty(work=True) for p in b.problems]
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    for _ in range(5):
        b.hvp(Z, True, sig, HZ)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        b.hvp(Z, True, sig, HZ)
    e1.record(stream)
    torch.cuda.synchronize()
    batched_ms = e0.elapsed_time(e1) / steps
    for p, z, h in zip(b.problems, Z, HZ):
        p.hvp_dot(z, 1e-2, out=h)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        for p, z, h in zip(b.problems, Z, HZ):
            p.hvp_dot(z, 1e-2, out=h)
    e1.record(stream)
    torch.cuda.synchronize()
    seq_ms = e0.elapsed_time(e1) / steps
    pts = sum(int(np.prod(sp.n)) for sp in specs)
    sizes = {}
    for sp in specs:
        sizes[sp.n[0]] = sizes.get(sp.n[0], 0) + 1
    log("batch of %d (%s): %.1f us per batched HVP pass, %.1f us one by one; x-pass variant %d %s" % (
        count, sizes, 1e3 * batched_ms, 1e3 * seq_ms, sched[0], sched[1]))
    out = {"workload": "%d spin-1 2D problems, n^2 with n in {64,128,256}, [-12,12]^2, lattice V, "
                       "beta=(100, U[-1,1]), M=U[0,0.9], seed 5" % count,
           "grid_counts": {str(k): v for k, v in sorted(sizes.items())}, "grid_points": pts,
           "precision": "mixed", "create_s": round(t_create, 3),
           "xpass_schedule": {"variant": sched[0], "us_per_variant": [round(x, 1) for x in sched[1]]},
           "batched_pass_us": round(1e3 * batched_ms, 2), "sequential_pass_us": round(1e3 * seq_ms, 2),
           "hvp_per_s_batched": round(count / (batched_ms / 1e3), 1),
           "hvp_per_s_sequential": round(count / (seq_ms / 1e3), 1),
           "speedup": round(seq_ms / batched_ms, 2)}
    if solve:
        Xb = [x.clone() for x in X0]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = b.newton_solve(Xb, check=False, tol=1e-6)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        conv = sum(int(s["converged"]) for s in st)
        log("batched solve: %.2f s, %d/%d converged, max hvp %d" % (tb, conv, count, max(s["hvp_calls"] for s in st)))
        ts, E1 = 0.0, []
        for i, sp in enumerate(specs):
            p = Problem(sp, "mixed")
            x = X0[i].clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, s1 = p.newton_solve(x, check=False, tol=1e-6)
            torch.cuda.synchronize()
            ts += time.perf_counter() - t0
            E1.append(s1["E"])
            p.close()
        dE = max(abs(a["E"] - e) / abs(e) for a, e in zip(st, E1))
        log("one-by-one solves: %.2f s; max relative energy difference %.2e" % (ts, dE))
        out["solve"] = {"tol": 1e-6, "batched_s": round(tb, 3), "sequential_s": round(ts, 3),
                        "speedup": round(ts / tb, 2), "converged": conv,
                        "max_hvp_calls": max(s["hvp_calls"] for s in st),
                        "total_hvp_calls": sum(s["hvp_calls"] for s in st),
                        "max_rel_energy_diff_vs_sequential": dE}
    b.close()
    torch.cuda.empty_cache()
    return out


def paper_tables(log):
    """ARNT on the Sec. 7.1 workloads (Tables 1-1-2 .. 1-3-3): every printed
    magnetization with the three retractions, FP64, one mesh, ||grad|| <= 1e-6,
    the paper's initial data.  Energies against the printed ones; times are this
    GPU's (the paper's: MATLAB on a 12-core Xeon, all meshes)."""
    import torch
    from paper_1907_01194_amd import workloads as W
    from paper_1907_01194_amd.binding import Problem
    rows = []
    for table, t in W.PAPER_TABLES.items():
        for M, E_paper in t["E"].items():
            spec, X0 = W.paper_table_case(table, M)
            for retr in (1, 2, 3):
                gp = Problem(spec, "fp64")
                X = torch.from_numpy(X0).cuda()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, st = gp.newton_solve(X, check=False, tol=1e-6, retraction=retr, time_limit=120.0)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                gp.close()
                del X
                torch.cuda.empty_cache()
                inner = st["cg_total"] / max(st["outer"], 1)
                rows.append({"table": table, "M": M, "retraction": "R%d" % retr, "E": st["E"], "E_paper": E_paper,
                             "dE": st["E"] - E_paper, "gnorm": st["gnorm"], "converged": bool(st["converged"]),
                             "outer": st["outer"], "avg_inner": round(inner, 1), "rgbb_iters": st["rgbb_iters"],
                             "seconds": round(dt, 3)})
                log("table %s M=%g R%d: E=%.6f (paper %.4f, diff %+.1e) |g|=%.1e iter %d (%.0f) %.2fs" % (
                    table, M, retr, st["E"], E_paper, st["E"] - E_paper, st["gnorm"], st["outer"], inner, dt))
    return rows


def cpu_baseline(spec, w, noise, log):
    """The oracle (FP64, NumPy/scipy) per Riemannian HVP on the same workload."""
    here = os.path.dirname(os.path.abspath(__file__))
    sys.path.insert(0, here)
    import oracle
    import oracle.energy as oe
    oe.FFT_WORKERS = os.cpu_count()
    prob = oracle.make_problem(spec.F, spec.n, spec.lo, spec.hi, spec.V, spec.beta, spec.M, spec.p, spec.q)
    u = oracle.retraction.psi(prob, w, 1)
    xi = oracle.project(prob, u, noise)
    xi /= np.sqrt(oracle.inner(xi, xi))
    ag, bg = oracle.proj_coeffs(prob, u, oracle.grad(prob, u))
    oracle.rhess(prob, u, xi, ag, bg, 1e-2)                   # warm-up
    reps = 2
    t0 = time.perf_counter()
    for _ in range(reps):
        oracle.rhess(prob, u, xi, ag, bg, 1e-2)
    dt = (time.perf_counter() - t0) / reps
    log("cpu oracle: %.2f s per HVP" % dt)
    return {"value": round(1.0 / dt, 4), "unit": "HVP/s", "cores": os.cpu_count(), "kind": "oracle",
            "sample": "%d Riemannian HVPs (spin-3 128^3, FP64 NumPy/scipy.fft) after 1 warm-up, "
                      "scipy.fft workers=%d" % (reps, os.cpu_count())}


def paper_case_solves(n, precs, log):
    """The paper's spin-3 128^3 workload (Sec. 7.3 Table 4-1 3D / Table 1-3-3, Case II, M = 0.5)
    from the paper's initial data, solved to ||grad|| <= 1e-6 in each precision."""
    from paper_1907_01194_amd import workloads as W
    ps = W.spin3_3d_paper(n, "II", 0.5)
    pw = W.paper_initial(ps, W.paper_U(3, None, ps.M, 0))
    entry = {"workload": ps.name, "initial": "U phi0, U seeded uniform in R^7 (Sec. 7)", "tol": 1e-6,
             "paper_energy": 42.9822,
             "paper_context": {"seconds": 1050.1, "hardware": "MATLAB R2018b, 12-core Xeon E5-2680 v3",
                               "source": "Sec. 7.1 Table 1-3-3, ARNT with R1, M = 0.5, all meshes"}}
    for prec in precs:
        entry[prec] = time_solve(ps, prec, pw, 300.0, log)
        entry[prec]["energy_err_vs_paper"] = abs(entry[prec]["E"] - 42.9822)
    return entry


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the benchmark runs on one GPU only (the workload is one spin-3 128^3 grid; "
              "--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    log = lambda m: print(m, file=sys.stderr, flush=True)
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(log)
        return
    if args.paper_tables:
        rows = paper_tables(log)
        print(json.dumps({"paper_tables": rows, "precision": "fp64", "tol": 1e-6}), flush=True)
        return
    from paper_1907_01194_amd import workloads as W
    precs = args.precisions.split(",")
    if args.solve_only:
        print(json.dumps({"time_to_ground_state": {"paper_case": paper_case_solves(args.n, precs, log)}}), flush=True)
        return
    spec = W.spin3_3d(args.n)
    w = W.initial_state(spec, 3)
    noise = W.random_direction(spec, 103)
    res = {}
    for prec in precs:
        ms, kt, sched = time_hvps(spec, prec, w, noise, args.steps, args.warmup, log)
        res[prec] = {"ms_per_hvp": ms, "hvp_per_s": 1e3 / ms, "roofline": roofline(spec, prec, ms, kt, sched[0]),
                     "kernels_us": {k: round(1e3 * t / c, 2) for k, (c, t) in kt.items()},
                     "xpass_schedule": {"variant": sched[0], "us_per_variant": [round(x, 1) for x in sched[1]]}}
    solves = {}
    if not args.no_solve:
        solves["paper_case"] = paper_case_solves(args.n, precs, log)
        # (b) the benchmark physics (beta = (500, 5, -5, 2), gamma = (1, 1, 2)) from the same
        #     kind of initial data, capped: its soft modes make the Newton iteration slow
        bw = W.paper_initial(spec, W.paper_U(3, None, spec.M, 3))
        entry = {"workload": spec.name, "initial": "U phi0, U seeded uniform in R^7 (Sec. 7)", "tol": 1e-6,
                 "time_cap_s": args.solve_time}
        for prec in precs:
            entry[prec] = time_solve(spec, prec, bw, args.solve_time, log)
        solves["benchmark_physics"] = entry
    batch = None if args.no_batch else batch_measure(args.batch_count, 50, args.batch_solve, log)
    cpu = None if args.no_cpu else cpu_baseline(spec, w, noise, log)
    head = precs[0]
    out = {
        "metric": "HVPs/s + time-to-ground-state, spin-3 128^3, mixed vs FP64, same GPU",
        "value": round(res[head]["hvp_per_s"], 2),
        "unit": "HVP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res[head]["ms_per_hvp"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64+f64-reductions" if head == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": spec.name, "F": spec.F, "grid": list(spec.n), "box": [spec.lo[0], spec.hi[0]],
                   "potential": "0.5*(x^2+y^2+4z^2)", "beta": list(spec.beta), "M": spec.M,
                   "precision": head},
        "roofline": res[head]["roofline"]["kernel"],
        "hvp_roofline": res[head]["roofline"]["hvp"],
        "cpu_baseline": cpu,
        "precisions": {p: {"hvp_per_s": round(r["hvp_per_s"], 2), "ms_per_hvp": round(r["ms_per_hvp"], 4),
                           "roofline": r["roofline"], "kernels_us": r["kernels_us"],
                           "xpass_schedule": r["xpass_schedule"]} for p, r in res.items()},
        "time_to_ground_state": solves or None,
        "batched": batch,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
