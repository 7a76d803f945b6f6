"""Measured cost of the hybrid scheme against an equivalent uniform-grid LBM (eq. (14)).

eq. (14) models G = T_h / T_eq = (1 + chi s' n) / g, with T_h the time of a
hybrid iteration and T_eq that of a standard LBM resolving the body as finely
as the unstructured mesh does.  Here both times are measured on the GPU:

* T_h: one base-level step of the workload (every level, the coupling and the
  n FV sub-steps of each finest step), from a timed run of hlbm_step;
* T_eq: one base-level step (the same physical time) of the equivalent LBM
  (workloads.equivalent_lbm): the same structured levels plus one more nested
  box of half the finest spacing over the finest box (inset by a margin), no
  mesh, the profile resolved on that box by halfway bounce-back with the
  force by momentum exchange every finest step.  Its finest spacing is half a
  lattice unit, the wall spacing of the workloads' meshes.  The same grid
  without the body is timed too (t_eq_nobody): the cost of the body itself.

The model's inputs are measured on the same runs: chi = FV node updates over
structured node updates per base step (without n), g = structured node
updates of the equivalent LBM over those of the hybrid grid, s' = time per FV
node sub-step over time per structured node update (back-to-back kernel
timings of the finest collide-stream and the FV sub-step).

    python -m paper_2006_10487_amd.speedup --workload naca_re5000_c512 --steps 20

prints one JSON object.  With --accuracy-steps N (and optionally --aoa) both
schemes also run N finest steps of the hybrid scheme (2N of the equivalent
LBM, the same physical time) from the initial state, and the object gains the
mean C_D and C_L of each over the second half.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import sys
import time

from . import hlbm, workloads


def updates_per_base_step(info) -> int:
    """Structured node updates of one base step (level l steps 2^l times)."""
    return sum(int(info.active_nodes[l]) << l for l in range(info.n_levels))


def time_base_steps(sim, per: int, steps: int, warmup: int) -> float:
    import torch
    sim.step(per * warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(per * steps)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def mean_forces(w, prec, finest_steps):
    """Mean C_D, C_L over the second half of finest_steps steps from the initial state."""
    import torch
    sim = hlbm.HLBM.from_workload(w, precision=prec, history_len=finest_steps + 8)
    per = 2 ** (sim.info.n_levels - 1)
    n = finest_steps // per * per
    done, t0 = 0, time.perf_counter()
    while done < n:
        k = min(4000 // per * per, n - done)
        sim.step(k)
        done += k
        print(f"[speedup] {w.name}: {done}/{n} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    cd, cl = sim.history(n // 2, n)
    sim.close()
    return {"finest_steps": n, "cd_mean": float(cd.mean()), "cl_mean": float(cl.mean()),
            "cl_amplitude": float(0.5 * (cl.max() - cl.min())), "seconds": round(time.perf_counter() - t0, 2)}


def compare_forces(w, prec, steps):
    """The hybrid scheme and the body-resolved equivalent LBM over the same physical time."""
    h = mean_forces(w, prec, steps)
    e = mean_forces(workloads.equivalent_lbm(w), prec, 2 * steps)
    return {"aoa_deg": w.aoa_deg, "window": "second half", "hybrid": h, "equivalent_lbm": e,
            "cd_rel_diff": (h["cd_mean"] - e["cd_mean"]) / e["cd_mean"]}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--workload", default="naca_re5000_c512")
    ap.add_argument("--steps", type=int, default=20, help="timed base steps")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--fp64", action="store_true", help="FP64 populations (default FP32-shifted)")
    ap.add_argument("--accuracy-steps", type=int, default=0,
                    help="also compare mean C_D, C_L over the second half of this many hybrid finest steps")
    ap.add_argument("--aoa", type=float, default=None, help="angle of attack in degrees (default: the workload's)")
    a = ap.parse_args(argv)
    prec = hlbm.FP64 if a.fp64 else hlbm.FP32_SHIFTED
    w = workloads.PRESETS[a.workload]()
    if a.aoa is not None:
        w = dataclasses.replace(w, aoa_deg=a.aoa)
    sim = hlbm.HLBM.from_workload(w, precision=prec)
    info = sim.info
    L = info.n_levels - 1
    t_h = time_base_steps(sim, 2 ** L, a.steps, a.warmup)
    t_collide = sim.kernel_bench(f"collide_l{L}", 50) * 1e-3
    t_fv = sim.kernel_bench("fv_substep", 200) * 1e-3 / max(1, int(info.fv_fuse))   # per sub-step
    n_fin = int(info.active_nodes[L])
    n_mesh = int(info.n_mesh_nodes)
    n_sub = int(info.n_sub)
    ups_h = updates_per_base_step(info)
    sim.close()

    e = workloads.equivalent_lbm(w)
    sim = hlbm.HLBM.from_workload(e, precision=prec)
    einfo = sim.info
    t_eq = time_base_steps(sim, 2 ** (einfo.n_levels - 1), a.steps, a.warmup)
    ups_eq = updates_per_base_step(einfo)
    n_solid, n_bounce = int(einfo.n_solid), int(einfo.n_bounce)
    cd_eq = float(sim.history()[0][-1])
    sim.close()
    sim = hlbm.HLBM.from_workload(workloads.equivalent_lbm(w, body=False), precision=prec)
    t_eq_nobody = time_base_steps(sim, 2 ** (sim.info.n_levels - 1), a.steps, a.warmup)
    sim.close()

    fv_ups = n_mesh * (2 ** L)                       # FV node updates per base step, without n
    chi = fv_ups / ups_h
    g = ups_eq / ups_h
    s_prime = (t_fv / n_mesh) / (t_collide / n_fin)
    out = {
        "workload": w.name, "equivalent": e.name, "precision": "fp64" if a.fp64 else "fp32_shifted",
        "t_h_ms_per_base_step": round(1e3 * t_h, 4), "t_eq_ms_per_base_step": round(1e3 * t_eq, 4),
        "t_eq_nobody_ms_per_base_step": round(1e3 * t_eq_nobody, 4),
        "G_measured": round(t_h / t_eq, 4),
        "equivalent_body": {"solid_nodes": n_solid, "bounce_back_nodes": n_bounce, "cd_last": cd_eq},
        "model": {"chi": chi, "n": n_sub, "s_prime": round(s_prime, 3), "g": round(g, 4),
                  "G": round((1.0 + chi * s_prime * n_sub) / g, 4)},
        "structured_updates_per_base_step": {"hybrid": ups_h, "equivalent": ups_eq},
        "mesh_nodes": n_mesh, "finest_collide_us": round(1e6 * t_collide, 3), "fv_substep_us": round(1e6 * t_fv, 3),
        "paper": {"chi": 1.5e-4, "g": 1.6, "n": 10, "s_prime": "3-5", "G": 0.63},
    }
    if a.accuracy_steps > 0:
        out["accuracy"] = compare_forces(w, prec, a.accuracy_steps)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
