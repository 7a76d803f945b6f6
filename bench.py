#!/usr/bin/env python3
"""Throughput benchmark of the HLBM step on one MI355X.

One bench step = one base-level step of the whole hybrid update: the base grid
once, the refinement box twice, and per finest step the coupling of
eqs. (4)-(9), n finite-volume sub-steps and the wall force.  Workload: NACA
0012 at Re = 5000, 8 deg, chord 512, 8192 x 4096 base cells (spacing 2) with a
2048 x 1024 box of unit spacing, O-mesh 2048 x 128 (synthetic geometry, no
dataset).  value = structured node updates (all levels) per second of the
whole step, in MLUPS, with FP32-shifted populations; the FP64 run is reported
beside it.  The roofline object covers the dominant kernel, timed with HIP
events on the library's stream during the timed region.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def progress(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)
METRIC = "MLUPS & HBM GB/s % peak, FP32 vs FP64 at stated Cd error; adjoint/forward time"


def run_precision(w, precision, steps, warmup, hlbm, torch):
    progress(f"create precision={precision}")
    sim = hlbm.HLBM.from_workload(w, precision=precision)
    progress("warmup")
    per = 2 ** w.n_refine
    info = sim.info
    sim.step(per * warmup)
    torch.cuda.synchronize()
    progress("timed region")
    t0 = time.perf_counter()
    sim.step(per * steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    progress(f"timed {steps} steps in {t1 - t0:.3f} s")
    # per-kernel breakdown: the same number of steps with every launch
    # bracketed by HIP events (the brackets add launch gaps; not used for value)
    # (with the running means of the wall coefficients, eqs. (12)-(13), switched on)
    sim.wall_stats_begin()
    sim.profile(True)
    sim.profile_read()
    sim.step(per * steps)
    prof = sim.profile_read()
    sim.profile(False)
    wall = sim.wall_stats()
    cd, cl = sim.history(sim.t - per * (warmup + 2 * steps), sim.t)
    # back-to-back launches of single kernels (pure kernel time per launch)
    pure = {"fv_substep": sim.kernel_bench("fv_substep", 400) if info.n_mesh_nodes else None}
    for l in range(info.n_levels):
        pure[f"collide_l{l}"] = sim.kernel_bench(f"collide_l{l}", 20)
    progress("kernel timings done")
    struct_updates = sum(int(info.active_nodes[l]) << l for l in range(info.n_levels))
    fv_updates = per * info.n_sub * int(info.n_mesh_nodes)
    return dict(sim=sim, info=info, prof=prof, pure=pure, t=t1 - t0,
                struct_updates=struct_updates, fv_updates=fv_updates, cd=cd, cl=cl, wall=wall)


def kernel_bytes(info, k):
    if k.startswith("collide_l"):
        return int(info.k1_bytes[int(k[-1])])
    if k == "fv_substep":      # one launch takes fv_fuse sub-steps
        return int(info.fv_bytes) * max(1, int(info.fv_fuse))
    return None


def kernel_table(r):
    info = r["info"]
    rows = {}
    for k, (ms, n) in r["prof"].items():
        if n == 0:
            continue
        by = kernel_bytes(info, k)
        avg_us = 1e3 * ms / n
        rows[k] = {"launches": n, "event_avg_us": round(avg_us, 3), "share": None, "alg_bytes": by}
        if k in r["pure"] and r["pure"][k]:
            pu = 1e3 * r["pure"][k]
            rows[k]["avg_us"] = round(pu, 3)
            rows[k]["gbs"] = round(by / (pu * 1e-6) / 1e9, 1)
    tot = sum(v["event_avg_us"] * v["launches"] for v in rows.values())
    for v in rows.values():
        v["share"] = round(v["event_avg_us"] * v["launches"] / tot, 4)
    return rows


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "hlbm_step_naca_re5000_c512_fp32_hbm_traffic.md")
# the forward kernels are the text of kernels.hip before this line
ADJOINT_MARKER = "// ---- Discrete adjoint kernels (reverse mode, FP64) ----"


def measured_traffic(kernel, fv_fuse=None):
    """Calibrated HBM bytes per launch from the committed counter summary, or
    None when the forward kernels (or, for the FV launch, its number of
    sub-steps) changed since the counters were taken."""
    import hashlib
    import re
    try:
        text = open(TRAFFIC_SUMMARY).read()
        rec = json.loads(re.search(r"```json\n(.*?)\n```", text, re.S).group(1))
        src = open(os.path.join(ROOT, "paper_2006_10487_amd", "csrc", "kernels.hip")).read()
        fwd = src[:src.index(ADJOINT_MARKER)]
        if hashlib.sha256(fwd.encode()).hexdigest() != rec["forward_kernels_sha256"]:
            return None
        if kernel == "fv_substep" and rec[kernel].get("fv_fuse") != fv_fuse:
            return None
        return round(rec[kernel]["traffic_bytes"])
    except (OSError, ValueError, KeyError, AttributeError):
        return None


def roofline(rows, k, note, traffic=None, info=None):
    v = rows[k]
    out = {"bound": "hbm", "kernel": k, "achieved": v["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(v["gbs"] / HBM_PEAK_GBS, 4), "traffic": traffic,
           "alg_bytes_per_launch": v["alg_bytes"], "avg_launch_us": v["avg_us"], "note": note}
    if k == "fv_substep" and info is not None:
        # what this implementation's layout moves if nothing stays on chip between sub-steps
        # (records with stored moments, padded neighbour table), for comparison with traffic
        out["layout_bytes_per_launch"] = int(info.fv_layout_bytes) * max(1, int(info.fv_fuse))
    return out


def adjoint_cost(hlbm, torch, workloads, t_end=25000, ckpt=500, fd=False):
    """(objective run + discrete adjoint) time over a plain forward of the same steps.

    Workload: Re = 1000, c = 128, 5 deg, eight seeded Hicks-Henne bumps
    (1024x512 base grid, one 384x192 box, 512x64 mesh), FP64, J = mean C_D over
    finest steps [0.8 t_end, t_end), checkpoints every `ckpt` steps; gradient
    w.r.t. angle of attack, tau and the eight bump amplitudes (the mesh carries
    the bump tangent as its shape derivatives).  With fd, central differences
    (h = 1e-6) of the GPU forward check dJ/d alpha and two amplitudes."""
    w = workloads.naca_re1000_c128_bumps()
    tan = w.omesh.bump_tangent(workloads.HH_PEAKS)
    progress(f"adjoint cost, {t_end} finest steps")
    sim = hlbm.HLBM.from_workload(w, precision=hlbm.FP64, history_len=t_end + 8, dxy_dshape=tan)
    sim.step(20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(t_end)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    progress(f"forward {t_fwd:.2f} s")
    spec = dict(t_end=t_end, t0=t_end * 4 // 5, t1=t_end, ckpt_every=ckpt, w_cd=1.0, w_cl=0.0)
    out = {"workload": w.name, "finest_steps": t_end, "window": [spec["t0"], spec["t1"]], "ckpt_every": ckpt,
           "precision": "fp64", "forward_s": round(t_fwd, 4)}
    # workspace and transposed tables once, outside the timed runs
    sim.reserve_objective(**spec, mesh_grad=True)
    warm = dict(spec, t_end=2 * ckpt, t0=ckpt, t1=2 * ckpt)
    sim.run_objective(**warm, mesh_grad=True)
    sim.adjoint()
    for mesh_grad in (False, True):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        J = sim.run_objective(**spec, mesh_grad=mesh_grad)
        t1 = time.perf_counter()
        g = sim.adjoint()
        t2 = time.perf_counter()
        key = "with_shape" if mesh_grad else "aoa_tau"
        out[key] = {"ratio": round((t2 - t0) / t_fwd, 3), "objective_run_s": round(t1 - t0, 4),
                    "adjoint_s": round(t2 - t1, 4), "J": J, "grad_aoa_tau": [float(g[0]), float(g[1])]}
        if mesh_grad:
            out[key]["grad_bumps"] = [float(v) for v in g[2:]]
        progress(f"{key}: ratio {out[key]['ratio']}")
    sim.close()
    out["ratio"] = out["with_shape"]["ratio"]
    if fd:
        out["central_fd"] = adjoint_fd(hlbm, torch, workloads, w, spec, out["with_shape"])
    out["note"] = ("gradient of the windowed mean C_D w.r.t. angle of attack, tau and the 8 bump amplitudes; "
                   "ratio = (objective run + adjoint) / plain forward of the same finest steps")
    return out


def adjoint_fd(hlbm, torch, workloads, w, spec, adj, h=1e-6):
    """Central differences of the GPU forward (FP64) for alpha and bumps 2 and 5."""
    amps0 = workloads.hh_amplitudes(0)

    def J(aoa=None, amps=None):
        ww = w if amps is None else workloads.naca_re1000_c128_bumps(amps)
        sim = hlbm.HLBM.from_workload(ww, precision=hlbm.FP64, history_len=spec["t_end"] + 8,
                                      aoa_rad=ww.aoa_rad if aoa is None else aoa)
        sim.step(spec["t_end"])
        cd, _ = sim.history(spec["t0"], spec["t1"])
        sim.close()
        return float(np.mean(cd))

    res = {"h": h}
    fd_a = (J(aoa=w.aoa_rad + h) - J(aoa=w.aoa_rad - h)) / (2 * h)
    res["aoa"] = {"fd": fd_a, "adjoint": adj["grad_aoa_tau"][0],
                  "rel_diff": abs(fd_a - adj["grad_aoa_tau"][0]) / abs(fd_a)}
    progress(f"fd alpha {res['aoa']}")
    for m in (2, 5):
        ap, am = amps0.copy(), amps0.copy()
        ap[m] += h
        am[m] -= h
        fd_m = (J(amps=ap) - J(amps=am)) / (2 * h)
        res[f"bump{m}"] = {"fd": fd_m, "adjoint": adj["grad_bumps"][m],
                           "rel_diff": abs(fd_m - adj["grad_bumps"][m]) / abs(fd_m)}
        progress(f"fd bump {m} {res[f'bump{m}']}")
    return res


def oracle_legs(preset, legs):
    """Runs the FP64 oracle in a child process on a workload preset: per (threads,
    finest steps) leg its wall time (create excluded)."""
    import subprocess
    cmd = [sys.executable, "-m", "oracle.oracle", preset] + [str(v) for leg in legs for v in leg]
    out = subprocess.run(cmd, cwd=ROOT, check=True, capture_output=True, text=True).stdout
    return json.loads(out.strip().splitlines()[-1])


def gpu_seconds_per_step(hlbm, torch, w, precision, finest_steps):
    sim = hlbm.HLBM.from_workload(w, precision=precision)
    info = sim.info
    sim.step(2 ** w.n_refine * 4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(finest_steps)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / finest_steps
    sim.close()
    return dt, info


def cpu_baseline(hlbm, torch, workloads, preset, w, r32, base_steps, c0_steps):
    """The oracle as it stands, on the host cores: the bench workload (base_steps
    base steps with all threads, one base step with one thread) and the Re = 100
    workload (c0_steps finest steps with all threads and with one)."""
    per = 2 ** w.n_refine
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    progress(f"oracle legs on the bench workload ({threads} threads, then 1)")
    big = oracle_legs(preset, [(threads, per * base_steps), (1, per)])
    su = r32["struct_updates"]                      # structured node updates per base step (all levels)
    fvu = r32["fv_updates"]                         # FV node-substeps per base step
    legs = []
    for leg in big["legs"]:
        n_base = leg["finest_steps"] / per
        legs.append({"workload": w.name, "threads": leg["threads"], "finest_steps": leg["finest_steps"],
                     "seconds": round(leg["seconds"], 3),
                     "mlups": round(su * n_base / leg["seconds"] / 1e6, 2),
                     "fv_msubsteps_per_s": round(fvu * n_base / leg["seconds"] / 1e6, 2)})
    w0 = workloads.naca_re100_c40()
    progress(f"oracle legs on the Re 100 workload ({c0_steps} steps, {threads} threads, then 1)")
    small = oracle_legs("naca_re100_c40", [(threads, c0_steps), (1, c0_steps)])
    g_dt, info0 = gpu_seconds_per_step(hlbm, torch, w0, hlbm.FP64, c0_steps)
    su0 = int(info0.active_nodes[0])
    fvu0 = int(info0.n_sub) * int(info0.n_mesh_nodes)
    for leg in small["legs"]:
        legs.append({"workload": w0.name, "threads": leg["threads"], "finest_steps": leg["finest_steps"],
                     "seconds": round(leg["seconds"], 3),
                     "mlups": round(su0 * leg["finest_steps"] / leg["seconds"] / 1e6, 2),
                     "fv_msubsteps_per_s": round(fvu0 * leg["finest_steps"] / leg["seconds"] / 1e6, 2)})
    gpu_c0 = {"workload": w0.name, "precision": "fp64", "finest_steps": c0_steps,
              "ms_per_finest_step": round(1e3 * g_dt, 4), "mlups": round(su0 / g_dt / 1e6, 2),
              "fv_msubsteps_per_s": round(fvu0 / g_dt / 1e6, 2)}
    main_leg = legs[0]
    return {"value": main_leg["mlups"], "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{base_steps} base steps = {per * base_steps} finest steps of the same workload in FP64 "
                      f"with {threads} OpenMP threads (structured levels, {int(r32['info'].n_sub)} FV sub-steps "
                      f"per finest step, coupling, forces), {main_leg['seconds']} s wall",
            "seconds": main_leg["seconds"], "legs": legs, "gpu_same_legs_re100_fp64": gpu_c0}


def drift(hlbm, torch, w, finest_steps):
    """C_D and C_L of the bench workload over `finest_steps` finest steps in FP32-shifted
    and FP64 storage: means over the second half and their differences.  A third
    run in FP64 with the angle of attack moved by 1e-9 rad measures how far the
    flow itself carries a perturbation of that size (its deterministic effect on
    the means is ~1e-9): FP32 deviations of the same size are flow sensitivity."""
    out = {"finest_steps": finest_steps, "window": [finest_steps // 2, finest_steps]}
    hist = {}
    for name, prec, da in (("fp64", hlbm.FP64, 0.0), ("fp32", hlbm.FP32_SHIFTED, 0.0),
                           ("fp64_aoa_plus_1e-9", hlbm.FP64, 1e-9)):
        sim = hlbm.HLBM.from_workload(w, precision=prec, history_len=finest_steps + 8, check_every=1000,
                                      aoa_rad=w.aoa_rad + da)
        progress(f"drift run {name}")
        sim.step_logged(finest_steps, name)
        hist[name] = sim.history(0, finest_steps)
        sim.close()
    h = slice(finest_steps // 2, finest_steps)
    for name in ("fp64", "fp32", "fp64_aoa_plus_1e-9"):
        cd, cl = hist[name]
        out[name] = {"cd_mean": float(np.mean(cd[h])), "cl_mean": float(np.mean(cl[h])),
                     "cd_min": float(np.min(cd[h])), "cd_max": float(np.max(cd[h])),
                     "cl_min": float(np.min(cl[h])), "cl_max": float(np.max(cl[h]))}
    d, s_, pt = out["fp64"], out["fp32"], out["fp64_aoa_plus_1e-9"]
    norm = max(abs(d["cl_mean"]), abs(d["cd_mean"]))
    out["cd_mean_rel_err"] = abs(s_["cd_mean"] - d["cd_mean"]) / abs(d["cd_mean"])
    out["cl_mean_err_over_max_abs_cl_cd"] = abs(s_["cl_mean"] - d["cl_mean"]) / norm
    out["fp64_sensitivity_cd_rel"] = abs(pt["cd_mean"] - d["cd_mean"]) / abs(d["cd_mean"])
    out["fp64_sensitivity_cl_over_max_abs_cl_cd"] = abs(pt["cl_mean"] - d["cl_mean"]) / norm
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100, help="timed base steps")
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="naca_re5000_c512")
    ap.add_argument("--cpu-steps", type=int, default=16, help="base steps of the oracle sample (~10 s on 16 cores)")
    ap.add_argument("--cpu-c0-steps", type=int, default=2000,
                    help="finest steps of the oracle legs on the Re 100 workload (its stated run)")
    ap.add_argument("--drift-steps", type=int, default=0,
                    help="also run the bench workload this many finest steps in both precisions and compare "
                         "the means of C_D and C_L over the second half")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint cost measurement")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only the adjoint cost measurement (prints its JSON object; for profiling)")
    ap.add_argument("--adjoint-steps", type=int, default=25000,
                    help="finest steps of the adjoint cost run (the adjoint workload's length is 25,000)")
    ap.add_argument("--adjoint-fd", action="store_true",
                    help="also check the adjoint gradient against central differences of the GPU forward")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of MIB MiB five times (calibrates HBM byte counters)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (--gpus {a.gpus} requested); "
              "the multi-GPU decomposition is a design note, not an implementation.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2006_10487_amd import hlbm, workloads

    w = workloads.PRESETS[a.workload]()
    per = 2 ** w.n_refine
    if a.adjoint_only:
        print(json.dumps(adjoint_cost(hlbm, torch, workloads, a.adjoint_steps, fd=a.adjoint_fd)))
        return
    r32 = run_precision(w, hlbm.FP32_SHIFTED, a.steps, a.warmup, hlbm, torch)
    k32 = kernel_table(r32)
    t32 = r32["t"]
    value = r32["struct_updates"] * a.steps / t32 / 1e6
    res = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(1e3 * t32 / a.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "base_cells": [w.nx_cells, w.ny_cells], "boxes": w.patches,
                   "mesh_nodes": int(r32["info"].n_mesh_nodes), "n_sub": int(r32["info"].n_sub),
                   "re": w.re, "aoa_deg": w.aoa_deg, "chord": w.chord,
                   "finest_steps_per_step": per, "fv_fuse": int(r32["info"].fv_fuse),
                   "fv_tiles": int(r32["info"].fv_tiles), "fv_tile_nodes": int(r32["info"].fv_tile_nodes),
                   "precision": "fp32_shifted_fp64_forces"},
    }
    dom = max(k32, key=lambda k: k32[k]["share"])
    res["roofline"] = roofline(k32, dom, "dominant kernel by time share; algorithmic bytes per launch (FV: per "
                                         "node-sub-step 9 populations in and out, own coefficients and row "
                                         "pointer, column and (G_x, G_y, C) per neighbour entry; fv_fuse "
                                         "sub-steps per launch) over the mean of back-to-back launches timed "
                                         "with HIP events; traffic = calibrated FETCH_SIZE + WRITE_SIZE bytes "
                                         "per launch",
                               measured_traffic(dom, int(r32["info"].fv_fuse))
                               if w.name == "naca0012_re5000_c512_8192x4096_r1" else None,
                               info=r32["info"])
    res["roofline_base_grid"] = roofline(k32, "collide_l0", "base-level fused stream-collide (72 B per node)",
                                         measured_traffic("collide_l0") if w.name == "naca0012_re5000_c512_8192x4096_r1" else None)
    res["kernels_fp32"] = k32
    if "wall_stats" in k32:
        n_wall = int(r32["wall"][1].size)
        ws = k32["wall_stats"]
        res["wall_stats"] = {
            "kernel": "wall_stats", "bound": "latency", "n_wall": n_wall, "launches": ws["launches"],
            "event_avg_us": ws["event_avg_us"], "share_of_step": ws["share"],
            "alg_bytes_per_launch": n_wall * (12 * 4 + 16 + 48),
            "steps_averaged": r32["wall"][0],
            "note": "running means of C_p, C_f, C_n at the wall nodes (eqs. (12)-(13)), one launch per finest "
                    "step while switched on; a few hundred KB per launch, so launch latency bounds it"}
    res["fv_msubsteps_per_s"] = round(r32["fv_updates"] * a.steps / t32 / 1e6, 1)
    if not a.no_fp64:
        r64 = run_precision(w, hlbm.FP64, a.steps, a.warmup, hlbm, torch)
        k64 = kernel_table(r64)
        res["fp64"] = {"value": round(r64["struct_updates"] * a.steps / r64["t"] / 1e6, 1),
                       "ms_per_step": round(1e3 * r64["t"] / a.steps, 4),
                       "roofline_base_grid": roofline(k64, "collide_l0", "FP64, 144 B per node"),
                       "kernels": k64}
        n = min(len(r32["cd"]), len(r64["cd"]))
        cd32, cd64 = r32["cd"][:n], r64["cd"][:n]
        cl32, cl64 = r32["cl"][:n], r64["cl"][:n]
        res["fp32_vs_fp64"] = {
            "finest_steps": int(n),
            "window": "every finest step of the two bench runs from the initial state: the impulsive start, "
                      "not a settled flow (--drift-steps compares the means of a longer run)",
            "cd_mean_fp64": float(np.mean(cd64)), "cl_mean_fp64": float(np.mean(cl64)),
            "cd_mean_rel_err": float(abs(np.mean(cd32) - np.mean(cd64)) / abs(np.mean(cd64))),
            "cl_mean_err_over_max_abs_cl_cd": float(abs(np.mean(cl32) - np.mean(cl64)) /
                                                    max(abs(np.mean(cl64)), abs(np.mean(cd64)))),
            "cd_max_rel_err_per_step": float(np.max(np.abs(cd32 - cd64) / np.abs(cd64))),
        }
        r64["sim"].close()
    if a.copy_probe:
        n = a.copy_probe * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        res["copy_probe_bytes_each_way"] = n * 4
        del src, dst
    if not a.no_adjoint:
        res["adjoint_over_forward"] = adjoint_cost(hlbm, torch, workloads, a.adjoint_steps, fd=a.adjoint_fd)
    if a.drift_steps:
        res["fp32_vs_fp64_drift"] = drift(hlbm, torch, w, a.drift_steps)
    if not a.no_cpu:
        res["cpu_baseline"] = cpu_baseline(hlbm, torch, workloads, a.workload, w, r32, a.cpu_steps, a.cpu_c0_steps)
    r32["sim"].close()
    print(json.dumps(res))


if __name__ == "__main__":
    main()
