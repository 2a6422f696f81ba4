#!/usr/bin/env python3
"""Benchmark of the spin-F ground-state hot path on one MI355X.

Workload: spin-3, 3D, 128^3 grid on [-8,8]^3, V = (x^2 + y^2 + 4 z^2)/2,
beta = (500, 5, -5, 2), M = 0.2 (synthetic seeded inputs; no dataset).

A step is one Riemannian Hessian-vector product of the regularised Newton
model at a fixed point u (Sec. 3 HVP formula, Lemma 4.2): the three
spectral-Laplacian axis passes, the pointwise spin-3 Hessian terms, the FP64
reductions of the tangent-space projection and the projection itself.  Steps
run back to back on one stream with nothing read back (as the device-resident
CG issues them); the same loop with the host read-back of <Z, HZ> after every
HVP is reported beside it.  The headline value is FP64 HVPs/s; mixed
precision (c64 fields, FP64 reductions) rides on the same line, with the
whole HVP's HBM roofline at its compulsory bytes for both, the dominant
kernel's own figures, time-to-ground-state for both precisions (full
newton_solve: retraction, RGBB, ARNT, energies and gradients) with the time
each takes to reach 1e-5 relative energy, the configurations' other solves,
the batched form (64 spin-1 2D problems of uneven grids in one gpe_batch: one
batched HVP pass against the same HVPs one by one, and the lock-step Newton
solve against one-by-one solves) and the CPU oracle's timings.

    python bench.py [--gpus 1] [--steps 200] [--warmup 100] [--no-solve] [--no-cpu]
                    [--no-batch] [--no-batch-solve] [--no-batch-sequential] [--batch-only]
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

# Per-launch HBM bytes of the HVP's kernels from rocprofv3 counter runs recorded
# in profiles/ (FETCH_SIZE + WRITE_SIZE, copy-kernel calibrated) and the x pass's
# VALU instructions (SQ_INSTS_VALU, per wavefront; x64 lanes), by precision and
# schedule variant; valid only while the kernel sources hash to `src_hash`.
MEASURED = {
    "src_hash": "b9479596af174dd3",
    "traffic": {
        "fp64": {
            "0": {
                "hvp_xpass": 960321477,
                "lap_axis_y": 705329830,
                "lap_axis_z": 939946766
            },
            "1": {
                "hvp_xpass": 958474865,
                "lap_axis_y": 705329830,
                "lap_axis_z": 939946766
            },
            "2": {
                "hvp_xpass": 957689317,
                "lap_axis_y": 705329830,
                "lap_axis_z": 939946766
            }
        },
        "mixed": {
            "0": {
                "hvp_xpass": 479323960,
                "lap_axis_y": 352821879,
                "lap_axis_z": 469991312
            },
            "1": {
                "hvp_xpass": 478860473,
                "lap_axis_y": 352821879,
                "lap_axis_z": 469991312
            },
            "2": {
                "hvp_xpass": 478603403,
                "lap_axis_y": 352821879,
                "lap_axis_z": 469991312
            }
        }
    },
    "valu": {
        "fp64": {
            "0": 67518464,
            "1": 67493888,
            "2": 64040960
        },
        "mixed": {
            "0": 67600384,
            "1": 67371008,
            "2": 64229376
        }
    }
}


def kernel_src_hash():
    """Hash of the sources of the kernels an HVP launches (the x, y and z passes):
    lap.hip and every library header it includes, directly or not."""
    import hashlib
    import re
    d = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1907_01194_amd", "csrc")
    todo, seen = ["lap.hip"], []
    while todo:
        f = todo.pop()
        if f in seen or not os.path.exists(os.path.join(d, f)):
            continue
        seen.append(f)
        todo += re.findall(r'#include "([^"]+)"', open(os.path.join(d, f)).read())
    h = hashlib.sha256()
    for f in sorted(seen):
        h.update(f.encode())
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--n", type=int, default=128, help="grid points per axis")
    ap.add_argument("--no-solve", action="store_true", help="skip time-to-ground-state")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle timing")
    ap.add_argument("--solve-time", type=float, default=120.0,
                    help="wall-clock cap per solve of the benchmark physics (s)")
    ap.add_argument("--precisions", default="fp64,mixed", help="the first is the headline")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched measurements")
    ap.add_argument("--no-batch-solve", action="store_true", help="skip the lock-step batched solve")
    ap.add_argument("--no-batch-sequential", action="store_true",
                    help="skip the one-by-one solves the batched solve is compared with")
    ap.add_argument("--oracle-solves", action="store_true",
                    help="also time the oracle's spin-2 2D 256^2 solve (minutes on the host)")
    ap.add_argument("--variant", type=int, default=None, help="force the x-pass schedule variant")
    ap.add_argument("--trace-solve", action="store_true",
                    help="only the benchmark-physics solves, printing their per-iteration traces")
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--paper-tables", action="store_true",
                    help="only reproduce the ARNT rows of the Sec. 7.1 tables (every magnetization, R1/R2/R3)")
    ap.add_argument("--tables", default="", help="with --paper-tables: comma list of tables (default: all)")
    ap.add_argument("--table-cap", type=float, default=120.0, help="with --paper-tables: seconds per solve")
    ap.add_argument("--table-mg", type=int, default=0,
                    help="with --paper-tables: coarser meshes of the cascadic hierarchy (0: one mesh)")
    ap.add_argument("--solve-only", action="store_true",
                    help="only the paper's spin-3 128^3 ground-state solve (for profiling the whole solve)")
    ap.add_argument("--batch-only", action="store_true",
                    help="only the batched measurements (for profiling the batched kernels)")
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


def hvp_bytes(K, npts, cb, rb):
    """Compulsory bytes of one Riemannian HVP: read X, Z and V once, write HZ once."""
    return 3 * K * npts * cb + npts * rb


def time_hvps(spec, prec, w, noise, steps, warmup, log, variant=None):
    """Time `steps` back-to-back Riemannian HVPs (nothing read back) with HIP
    events on the handle's stream (torch's current stream), then the same with
    the host read-back of <Z, HZ> after each, then a pass with the library's
    events around every launch for the per-kernel breakdown."""
    import torch
    from paper_1907_01194_amd.binding import Problem, R1
    gp = Problem(spec, prec)
    if variant is not None:
        gp.set_schedule(variant)
    X = torch.from_numpy(w).cuda()
    u = gp.retract(X, None, 0.0, R1)                       # u = psi(w), on the manifold
    xi = gp.project(u, torch.from_numpy(noise).cuda())     # tangent direction
    nrm = np.sqrt(gp.constraints(xi)[0])
    xi /= nrm
    gp.set_point(u)
    Z = xi.to(gp.work_dtype).contiguous()
    HZ = gp.empty(work=True)
    for _ in range(warmup):
        gp.hvp(Z, True, 1e-2, out=HZ)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    # (1) the timed region: `steps` HVPs back to back, nothing else on the stream
    e0.record(stream)
    t0 = time.perf_counter()
    for _ in range(steps):
        gp.hvp(Z, True, 1e-2, out=HZ)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / steps
    # five more repetitions of the same (reported beside the timed region: their median)
    reps = []
    for _ in range(5):
        e0.record(stream)
        for _ in range(steps):
            gp.hvp(Z, True, 1e-2, out=HZ)
        e1.record(stream)
        torch.cuda.synchronize()
        reps.append(e0.elapsed_time(e1) / steps)
    # (2) with the read-back of kappa = <Z, HZ> after every HVP (one synchronisation each)
    e0.record(stream)
    kappa = 0.0
    for _ in range(steps):
        _, kappa = gp.hvp_dot(Z, 1e-2, out=HZ)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_dot = e0.elapsed_time(e1) / steps
    # (3) the library's HIP events around every launch: per-kernel durations
    gp.timing(True)
    for _ in range(steps):
        gp.hvp(Z, True, 1e-2, out=HZ)
    torch.cuda.synchronize()
    kt = gp.timing_read()
    gp.timing(False)
    sched = gp.schedule()
    log("%s: x-pass schedule variant %d (%s; us per variant %s)" % (
        prec, sched[0], "forced" if variant is not None else "autotuned", sched[1]))
    log("%s: %.1f us per HVP back to back (events), %.1f us (wall); %.1f us with the kappa read-back, "
        "kappa=%.6e; per-kernel pass (events around each launch):" % (prec, 1e3 * ms, 1e6 * wall / steps,
                                                                     1e3 * ms_dot, kappa))
    for k, (c, t) in sorted(kt.items(), key=lambda x: -x[1][1]):
        log("   %-12s %6d launches  %9.1f us avg" % (k, c, 1e3 * t / c))
    log("%s: five more repetitions: %s us per HVP (median %.1f)" % (
        prec, ", ".join("%.1f" % (1e3 * r) for r in reps), 1e3 * float(np.median(reps))))
    gp.close()
    del gp
    torch.cuda.empty_cache()
    return ms, ms_dot, kt, sched, reps


def roofline(spec, prec, ms, kt, variant, steps):
    """HBM roofline of the whole Riemannian HVP at its compulsory bytes (read
    X, Z, V; write HZ) against the measured time per HVP, and the dominant
    kernel's own figures (algorithmic bytes per launch over its average launch
    duration; VALU lane operations when its counters are on record)."""
    K = spec.K
    npts = int(np.prod(spec.n))
    cb, rb = (16, 8) if prec == "fp64" else (8, 4)
    hb = hvp_bytes(K, npts, cb, rb)
    hvp_gbs = hb / (ms / 1e3) / 1e9
    valid = npts == 128 ** 3 and K == 7 and MEASURED["src_hash"] == kernel_src_hash()
    tr = MEASURED["traffic"].get(prec, {}).get(str(variant)) if valid else None
    traffic = None
    if tr:
        # kernel launches per HVP from the per-launch timing pass
        traffic = int(sum(tr.get(k, 0) * c / steps for k, (c, _) in kt.items()))
    cand = {k: v for k, v in kt.items() if kernel_bytes(k, K, npts, cb, rb)}
    dom = max(cand, key=lambda k: cand[k][1])
    cnt, tot = cand[dom]
    per_launch_s = tot / cnt / 1e3
    b = kernel_bytes(dom, K, npts, cb, rb)
    achieved = b / per_launch_s / 1e9
    kern = {"name": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": tr.get(dom) if tr else None,
            "bytes_per_launch": b, "us_per_launch": round(per_launch_s * 1e6, 2), "schedule_variant": variant}
    valu = MEASURED["valu"].get(prec, {}).get(str(variant)) if valid else None
    if valu and dom == "hvp_xpass":
        ops = valu * 64
        tops = ops / per_launch_s / 1e12
        kern["valu"] = {"bound": "alu", "achieved": round(tops, 2), "peak": round(VALU_PEAK_TOPS, 2),
                        "unit": "TOP/s (VALU lane operations, non-packed)", "frac": round(tops / VALU_PEAK_TOPS, 4),
                        "lane_ops_per_launch": ops}
    return {"bound": "hbm", "achieved": round(hvp_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(hvp_gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
            "name": "riemannian_hvp (all its kernels, back to back)", "compulsory_bytes": hb,
            "us_per_hvp": round(ms * 1e3, 2), "dominant_kernel": kern}


def time_solve(spec, prec, w, limit, log, tol=1e-6, trace=0, mg=0):
    """Time-to-ground-state: newton_solve from w (device-resident before the
    clock starts) to ||grad|| <= tol, or until `limit` seconds; on one mesh, or
    after mg coarser meshes of the cascadic hierarchy (Algorithm 1)."""
    import torch
    from paper_1907_01194_amd.binding import Problem
    gp = Problem(spec, prec)
    X = torch.from_numpy(w).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    X, st = gp.newton_solve(X, check=False, tol=tol, time_limit=limit, trace=trace, mg_levels=mg)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log("solve %s %s%s: E=%.12f |g|=%.2e conv=%d rgbb=%d outer=%d cg=%d hvp=%d %.1fs" % (
        spec.name, prec, " mg=%d" % st["mg_levels"] if mg else "", st["E"], st["gnorm"], st["converged"],
        st["rgbb_iters"], st["outer"], st["cg_total"], st["hvp_calls"], wall))
    gp.close()
    del gp
    torch.cuda.empty_cache()
    out = {"seconds": round(wall, 3), "E": st["E"], "gnorm": st["gnorm"], "converged": bool(st["converged"]),
           "rgbb_iters": st["rgbb_iters"], "outer": st["outer"], "cg_total": st["cg_total"],
           "hvp_calls": st["hvp_calls"], "t_rgbb": round(st["t_rgbb"], 3), "t_arnt": round(st["t_arnt"], 3)}
    if mg:
        out.update({"mg_levels": st["mg_levels"], "t_coarse": round(st["t_coarse"], 3),
                    "finest_mesh": {"outer": st["outer"], "cg_total": st["cg_total"], "hvp_calls": st["hvp_calls"]}})
    if trace:
        out["_trace"] = st["trace"]
    return out


def time_to_accuracy(entry, precs, rel=1e-5):
    """Seconds (and HVPs) each precision's solve needs to bring E within `rel`
    of the best energy any of them reached (from the solves' traces)."""
    Es = [entry[p]["E"] for p in precs if p in entry]
    Eref = min(Es)
    out = {"relative_energy": rel, "E_ref": Eref, "E_ref_from": "lowest final energy of the solves"}
    for p in precs:
        tr = entry[p].pop("_trace", None)
        hit = None
        if tr is not None:
            for row in tr:
                if abs(row[1] - Eref) <= rel * abs(Eref):
                    hit = row
                    break
        t0 = entry[p].get("t_coarse", 0.0)   # a cascadic trace covers the finest mesh only
        out[p] = None if hit is None else {"seconds": round(t0 + float(hit[0]), 3), "hvp_calls": int(hit[3])}
    return out


def batch_measure(count, steps, solve, sequential, log):
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
    def timed(fn):
        for _ in range(20):
            fn()
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    def seq(dot):
        for p, z, h in zip(b.problems, Z, HZ):
            if dot:
                p.hvp_dot(z, 1e-2, out=h)
            else:
                p.hvp(z, True, 1e-2, out=h)

    # back to back without kappa (no read-back), and with each pass's kappas on the host
    batched_ms = timed(lambda: b.hvp(Z, True, sig, HZ, kappa=False))
    batched_k_ms = timed(lambda: b.hvp(Z, True, sig, HZ))
    seq_ms = timed(lambda: seq(False))
    seq_k_ms = timed(lambda: seq(True))
    pts = sum(int(np.prod(sp.n)) for sp in specs)
    sizes = {}
    for sp in specs:
        sizes[sp.n[0]] = sizes.get(sp.n[0], 0) + 1
    log("batch of %d (%s): %.1f us per batched HVP pass (%.1f with kappa read-back), %.1f us one by one "
        "(%.1f); x-pass variant %d %s" % (count, sizes, 1e3 * batched_ms, 1e3 * batched_k_ms, 1e3 * seq_ms,
                                           1e3 * seq_k_ms, sched[0], sched[1]))
    out = {"workload": "%d spin-1 2D problems, n^2 with n in {64,128,256}, [-12,12]^2, lattice V, "
                       "beta=(100, U[-1,1]), M=U[0,0.9], seed 5" % count,
           "grid_counts": {str(k): v for k, v in sorted(sizes.items())}, "grid_points": pts,
           "precision": "mixed", "create_s": round(t_create, 3),
           "xpass_schedule": {"variant": sched[0], "us_per_variant": [round(x, 1) for x in sched[1]]},
           "batched_pass_us": round(1e3 * batched_ms, 2), "sequential_pass_us": round(1e3 * seq_ms, 2),
           "batched_pass_kappa_readback_us": round(1e3 * batched_k_ms, 2),
           "sequential_pass_kappa_readback_us": round(1e3 * seq_k_ms, 2),
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
        for i, sp in enumerate(specs if sequential else []):
            p = Problem(sp, "mixed")
            x = X0[i].clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, s1 = p.newton_solve(x, check=False, tol=1e-6)
            torch.cuda.synchronize()
            ts += time.perf_counter() - t0
            E1.append(s1["E"])
            p.close()
        out["solve"] = {"tol": 1e-6, "batched_s": round(tb, 3), "converged": conv,
                        "max_hvp_calls": max(s["hvp_calls"] for s in st),
                        "total_hvp_calls": sum(s["hvp_calls"] for s in st)}
        # the same batch through the cascadic hierarchy (two coarser meshes per problem, each level in lock step)
        Xc = [x.clone() for x in X0]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, stc = b.newton_solve(Xc, check=False, tol=1e-6, mg_levels=2)
        torch.cuda.synchronize()
        tc = time.perf_counter() - t0
        convc = sum(int(s["converged"]) for s in stc)
        dEc = max(abs(a["E"] - c["E"]) / abs(a["E"]) for a, c in zip(st, stc))
        log("batched cascadic solve: %.2f s (coarse levels %.2f s), %d/%d converged, max finest-mesh hvp %d, "
            "max relative energy difference to the one-mesh solves %.1e" % (
                tc, stc[0]["t_coarse"], convc, count, max(s["hvp_calls"] for s in stc), dEc))
        out["solve_cascadic"] = {"tol": 1e-6, "mg_levels": stc[0]["mg_levels"], "batched_s": round(tc, 3),
                                 "coarse_levels_s": round(stc[0]["t_coarse"], 3), "converged": convc,
                                 "max_hvp_calls_finest_mesh": max(s["hvp_calls"] for s in stc),
                                 "total_hvp_calls_finest_mesh": sum(s["hvp_calls"] for s in stc),
                                 "max_rel_energy_diff_vs_one_mesh": dEc}
        if sequential:
            dE = max(abs(a["E"] - e) / abs(e) for a, e in zip(st, E1))
            log("one-by-one solves: %.2f s; max relative energy difference %.2e" % (ts, dE))
            out["solve"].update({"sequential_s": round(ts, 3), "speedup": round(ts / tb, 2),
                                 "max_rel_energy_diff_vs_sequential": dE})
    b.close()
    torch.cuda.empty_cache()
    return out


def paper_tables(log, tables=None, cap=120.0, mg=0):
    """ARNT on the Sec. 7.1 workloads (Tables 1-1-2 .. 1-3-3): every printed
    magnetization with the three retractions, FP64, ||grad|| <= 1e-6, the
    paper's initial data, on one mesh (mg = 0) or after mg coarser meshes of the
    cascadic hierarchy (Algorithm 1).  Energies against the printed ones; times
    are this GPU's (the paper's: MATLAB on a 12-core Xeon, all meshes)."""
    import torch
    from paper_1907_01194_amd import workloads as W
    from paper_1907_01194_amd.binding import Problem
    rows = []
    for table, t in W.PAPER_TABLES.items():
        if tables and table not in tables:
            continue
        for M, E_paper in t["E"].items():
            spec, X0 = W.paper_table_case(table, M)
            for retr in (1, 2, 3):
                gp = Problem(spec, "fp64")
                X = torch.from_numpy(X0).cuda()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, st = gp.newton_solve(X, check=False, tol=1e-6, retraction=retr, time_limit=cap, mg_levels=mg)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                gp.close()
                del X
                torch.cuda.empty_cache()
                inner = st["cg_total"] / max(st["outer"], 1)
                rows.append({"table": table, "M": M, "retraction": "R%d" % retr, "mg_levels": st["mg_levels"],
                             "E": st["E"], "E_paper": E_paper,
                             "dE": st["E"] - E_paper, "gnorm": st["gnorm"], "converged": bool(st["converged"]),
                             "outer": st["outer"], "avg_inner": round(inner, 1), "rgbb_iters": st["rgbb_iters"],
                             "seconds": round(dt, 3)})
                log("table %s M=%g R%d mg=%d: E=%.6f (paper %.4f, diff %+.1e) |g|=%.1e iter %d (%.0f) %.2fs" % (
                    table, M, retr, st["mg_levels"], st["E"], E_paper, st["E"] - E_paper, st["gnorm"], st["outer"],
                    inner, dt))
    return rows


def cpu_baseline(spec, w, noise, log, reps=5):
    """The oracle (FP64, NumPy/scipy.fft on every host core) per Riemannian HVP
    on the same workload: the median of `reps` timed HVPs after one warm-up."""
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
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        oracle.rhess(prob, u, xi, ag, bg, 1e-2)
        ts.append(time.perf_counter() - t0)
    dt = float(np.median(ts))
    log("cpu oracle: %.2f s per HVP (median of %d: %s)" % (dt, reps, ", ".join("%.2f" % t for t in ts)))
    return {"value": round(1.0 / dt, 4), "unit": "HVP/s", "cores": os.cpu_count(), "kind": "oracle",
            "sample": "median of %d Riemannian HVPs (spin-3 128^3, FP64 NumPy/scipy.fft, workers=%d) after "
                      "1 warm-up" % (reps, os.cpu_count()),
            "seconds_per_hvp": round(dt, 3), "seconds_each": [round(t, 3) for t in ts]}


def oracle_hvp_seconds(spec, seed, reps=3):
    """The oracle's median time per Riemannian HVP (all host cores for
    scipy.fft) at a point of `spec` built from its seeded initial state."""
    here = os.path.dirname(os.path.abspath(__file__))
    sys.path.insert(0, here)
    import oracle
    import oracle.energy as oe
    from paper_1907_01194_amd import workloads as W
    oe.FFT_WORKERS = os.cpu_count()
    prob = oracle.make_problem(spec.F, spec.n, spec.lo, spec.hi, spec.V, spec.beta, spec.M, spec.p, spec.q)
    u = oracle.retraction.psi(prob, W.initial_state(spec, seed), 1)
    xi = oracle.project(prob, u, W.random_direction(spec, 100 + seed))
    xi /= np.sqrt(oracle.inner(xi, xi))
    ag, bg = oracle.proj_coeffs(prob, u, oracle.grad(prob, u))
    oracle.rhess(prob, u, xi, ag, bg, 1e-2)
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        oracle.rhess(prob, u, xi, ag, bg, 1e-2)
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def oracle_solves(log):
    """The oracle's own time-to-ground-state on the small configurations (all
    host cores for scipy.fft): spin-1 1D 128 to ||grad|| <= 1e-8 and spin-2 2D
    256^2 to 1e-6, from the same seeded initial states as the GPU solves."""
    here = os.path.dirname(os.path.abspath(__file__))
    sys.path.insert(0, here)
    import oracle
    import oracle.energy as oe
    from paper_1907_01194_amd import workloads as W
    oe.FFT_WORKERS = os.cpu_count()
    out = {}
    for key, spec, seed, tol in (("spin1-1d-128", W.spin1_1d(), 1, 1e-8), ("spin2-2d-256", W.spin2_2d(), 2, 1e-6)):
        prob = oracle.make_problem(spec.F, spec.n, spec.lo, spec.hi, spec.V, spec.beta, spec.M, spec.p, spec.q)
        t0 = time.perf_counter()
        _, st = oracle.solve(prob, W.initial_state(spec, seed), oracle.SolveOpts(tol=tol))
        dt = time.perf_counter() - t0
        log("oracle solve %s: %.2f s E=%.12f |g|=%.2e conv=%d hvp=%d" % (key, dt, st.E, st.gnorm, st.converged,
                                                                          st.hvp_calls))
        out[key] = {"seconds": round(dt, 3), "E": st.E, "gnorm": st.gnorm, "converged": bool(st.converged),
                    "hvp_calls": st.hvp_calls, "tol": tol, "cores": os.cpu_count()}
    return out


def oracle_solves_small(log):
    """The oracle's spin-1 1D 128 solve (a fraction of a second)."""
    here = os.path.dirname(os.path.abspath(__file__))
    sys.path.insert(0, here)
    import oracle
    import oracle.energy as oe
    from paper_1907_01194_amd import workloads as W
    oe.FFT_WORKERS = os.cpu_count()
    spec = W.spin1_1d()
    prob = oracle.make_problem(spec.F, spec.n, spec.lo, spec.hi, spec.V, spec.beta, spec.M, spec.p, spec.q)
    t0 = time.perf_counter()
    _, st = oracle.solve(prob, W.initial_state(spec, 1), oracle.SolveOpts(tol=1e-8))
    dt = time.perf_counter() - t0
    log("oracle solve spin1-1d-128: %.2f s E=%.12f |g|=%.2e" % (dt, st.E, st.gnorm))
    return {"spin1-1d-128": {"seconds": round(dt, 3), "E": st.E, "gnorm": st.gnorm, "converged": bool(st.converged),
                             "hvp_calls": st.hvp_calls, "tol": 1e-8, "cores": os.cpu_count()}}


def config_solves(log):
    """GPU time-to-ground-state of the small configurations (FP64), from the
    same seeded initial states as the oracle's solves."""
    from paper_1907_01194_amd import workloads as W
    out = {}
    for key, spec, seed, tol in (("spin1-1d-128", W.spin1_1d(), 1, 1e-8), ("spin2-2d-256", W.spin2_2d(), 2, 1e-6)):
        out[key] = time_solve(spec, "fp64", W.initial_state(spec, seed), 120.0, log, tol=tol)
        out[key]["tol"] = tol
    return out


def paper_case_solves(n, precs, log, mg=0):
    """The paper's spin-3 128^3 workload (Sec. 7.3 Table 4-1 3D / Table 1-3-3, Case II, M = 0.5)
    from the paper's initial data, solved to ||grad|| <= 1e-6 in each precision."""
    from paper_1907_01194_amd import workloads as W
    ps = W.spin3_3d_paper(n, "II", 0.5)
    pw = W.paper_initial(ps, W.paper_U(3, None, ps.M, 0))
    entry = {"workload": ps.name, "initial": "U phi0, U seeded uniform in R^7 (Sec. 7)", "tol": 1e-6,
             "paper_energy": 42.9822,
             "paper_context": {"seconds": 1050.1, "hardware": "MATLAB R2018b, 12-core Xeon E5-2680 v3",
                               "source": "Sec. 7.1 Table 1-3-3, ARNT with R1, M = 0.5, all meshes"}}
    if mg:
        entry["meshes"] = "cascadic: %s" % " -> ".join("%d^3" % (n >> (mg - i)) for i in range(mg + 1))
    for prec in precs:
        entry[prec] = time_solve(ps, prec, pw, 300.0, log, mg=mg)
        entry[prec]["energy_err_vs_paper"] = abs(entry[prec]["E"] - 42.9822)
    return entry


def benchmark_physics_solves(spec, precs, limit, log, trace=4000, mg=0):
    """The benchmark physics (beta = (500, 5, -5, 2), gamma = (1, 1, 2)) from the
    Sec. 7 kind of initial data, each precision to ||grad|| <= 1e-6 or the
    time cap (on one mesh, or after mg coarser meshes of the cascadic
    hierarchy), with the time each takes to reach 1e-5 relative energy."""
    from paper_1907_01194_amd import workloads as W
    bw = W.paper_initial(spec, W.paper_U(3, None, spec.M, 3))
    entry = {"workload": spec.name, "initial": "U phi0, U seeded uniform in R^7 (Sec. 7)", "tol": 1e-6,
             "time_cap_s": limit, "meshes": "one (%d^3)" % spec.n[0] if not mg else
             "cascadic: %s" % " -> ".join("%d^3" % (spec.n[0] >> (mg - i)) for i in range(mg + 1))}
    for prec in precs:
        entry[prec] = time_solve(spec, prec, bw, limit, log, trace=trace, mg=mg)
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
        rows = paper_tables(log, [t for t in args.tables.split(",") if t], args.table_cap, args.table_mg)
        print(json.dumps({"paper_tables": rows, "precision": "fp64", "tol": 1e-6, "cap_s": args.table_cap,
                          "mg_levels": args.table_mg}), flush=True)
        return
    if args.batch_only:
        print(json.dumps({"batched": batch_measure(args.batch_count, 200, not args.no_batch_solve,
                                                   not args.no_batch_sequential, log)}), flush=True)
        return
    from paper_1907_01194_amd import workloads as W
    from paper_1907_01194_amd.binding import TRACE_NAMES
    precs = args.precisions.split(",")
    if args.solve_only:
        print(json.dumps({"time_to_ground_state": {"paper_case": paper_case_solves(args.n, precs, log)}}), flush=True)
        return
    spec = W.spin3_3d(args.n)
    if args.trace_solve:
        entry = benchmark_physics_solves(spec, precs, args.solve_time, log)
        for p in precs:
            tr = entry[p]["_trace"]
            log("trace %s (%s):" % (p, " ".join(TRACE_NAMES)))
            for row in tr:
                log("  " + " ".join("%.6g" % v for v in row))
        entry["to_1e-5_relative_energy"] = time_to_accuracy(entry, precs)
        print(json.dumps({"benchmark_physics": entry}), flush=True)
        return
    w = W.initial_state(spec, 3)
    noise = W.random_direction(spec, 103)
    res = {}
    for prec in precs:
        ms, ms_dot, kt, sched, reps = time_hvps(spec, prec, w, noise, args.steps, args.warmup, log, args.variant)
        res[prec] = {"ms_per_hvp": ms, "hvp_per_s": 1e3 / ms, "ms_per_hvp_with_kappa_readback": ms_dot,
                     "ms_per_hvp_repetitions": [round(r, 4) for r in reps],
                     "ms_per_hvp_median_of_5": round(float(np.median(reps)), 4),
                     "roofline": roofline(spec, prec, ms, kt, sched[0], args.steps),
                     "kernels_us": {k: round(1e3 * t / c, 2) for k, (c, t) in kt.items()},
                     "kernel_launches_per_hvp": {k: round(c / args.steps, 2) for k, (c, t) in kt.items()},
                     "xpass_schedule": {"variant": sched[0], "forced": args.variant is not None,
                                        "us_per_variant": [round(x, 1) for x in sched[1]]}}
    solves = {}
    if not args.no_solve:
        solves["paper_case"] = paper_case_solves(args.n, precs, log)
        entry = benchmark_physics_solves(spec, precs, args.solve_time, log)
        entry["to_1e-5_relative_energy"] = time_to_accuracy(entry, precs)
        solves["benchmark_physics"] = entry
        # Algorithm 1's cascadic outer loop: three coarser meshes (16^3 .. 64^3) first
        solves["paper_case_cascadic"] = paper_case_solves(args.n, precs, log, mg=3)
        cas = benchmark_physics_solves(spec, precs, args.solve_time, log, mg=3)
        cas["to_1e-5_relative_energy"] = time_to_accuracy(cas, precs)
        solves["benchmark_physics_cascadic"] = cas
        solves["configs"] = config_solves(log)
    batch = None if args.no_batch else batch_measure(args.batch_count, 200, not args.no_batch_solve,
                                                     not args.no_batch_sequential, log)
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(spec, w, noise, log)
        orc = {}
        if args.oracle_solves:
            orc = oracle_solves(log)
        else:
            orc = {k: v for k, v in oracle_solves_small(log).items()}
        c2 = solves.get("configs", {}).get("spin2-2d-256") if solves else None
        if c2 and "spin2-2d-256" not in orc:
            t2 = oracle_hvp_seconds(W.spin2_2d(), 2)
            log("cpu oracle: %.4f s per HVP at spin-2 2D 256^2" % t2)
            orc["spin2-2d-256 (estimate)"] = {
                "kind": "estimate: oracle seconds per HVP (median of 3) x the GPU FP64 solve's HVP count (not run; "
                        "bench.py --oracle-solves runs it)",
                "seconds": round(t2 * c2["hvp_calls"], 1), "seconds_per_hvp": round(t2, 4),
                "hvp_calls": c2["hvp_calls"]}
        fp = solves.get("benchmark_physics", {}).get("fp64") if solves else None
        if fp:
            orc["spin3-3d-128 (estimate)"] = {
                "kind": "estimate: oracle seconds per HVP x the GPU FP64 solve's HVP count (not run)",
                "seconds": round(cpu["seconds_per_hvp"] * fp["hvp_calls"], 1), "hvp_calls": fp["hvp_calls"]}
        cpu["time_to_ground_state"] = orc
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
        "dtype": "f64" if head == "fp64" else "c64+f64-reductions",
        "data": "synthetic",
        "config": {"workload": spec.name, "F": spec.F, "grid": list(spec.n), "box": [spec.lo[0], spec.hi[0]],
                   "potential": "0.5*(x^2+y^2+4z^2)", "beta": list(spec.beta), "M": spec.M,
                   "precision": head},
        "roofline": res[head]["roofline"],
        "cpu_baseline": cpu,
        "precisions": {p: {"hvp_per_s": round(r["hvp_per_s"], 2), "ms_per_hvp": round(r["ms_per_hvp"], 4),
                           "ms_per_hvp_with_kappa_readback": round(r["ms_per_hvp_with_kappa_readback"], 4),
                           "ms_per_hvp_median_of_5": r["ms_per_hvp_median_of_5"],
                           "ms_per_hvp_repetitions": r["ms_per_hvp_repetitions"],
                           "roofline": r["roofline"], "kernels_us": r["kernels_us"],
                           "kernel_launches_per_hvp": r["kernel_launches_per_hvp"],
                           "xpass_schedule": r["xpass_schedule"]} for p, r in res.items()},
        "time_to_ground_state": solves or None,
        "batched": batch,
        "kernel_src_hash": kernel_src_hash(),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
