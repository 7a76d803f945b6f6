"""FP64 against FP32-shifted storage on one workload preset over a long run.

For each precision: time means of C_D and C_L over the second half of the run,
their extremes there, and the Strouhal number of the lift signal; then the
FP32-shifted deviations (C_D relative, C_L relative to max(|C_L|, C_D), which
stays meaningful where C_L vanishes by symmetry) and per-tenth maxima of the
step-by-step C_D difference.

    python -m paper_2006_10487_amd.precision --workload naca_re1e4_c256 --f2c-filter --steps 100000

prints one JSON object.
"""
from __future__ import annotations

import argparse
import inspect
import json
import sys
import time

import numpy as np

from . import hlbm, workloads


def run(w, steps: int, precision: int):
    sim = hlbm.HLBM.from_workload(w, precision=precision, history_len=steps + 8, check_every=1000)
    t0 = time.perf_counter()
    sim.step_logged(steps, w.name, chunk=10000)
    dt = time.perf_counter() - t0
    cd, cl = sim.history(0, steps)
    sim.close()
    return cd, cl, dt


def summary(cd, cl, w):
    h = slice(len(cd) // 2, len(cd))
    return {"cd_mean": float(np.mean(cd[h])), "cl_mean": float(np.mean(cl[h])),
            "cd_min": float(np.min(cd[h])), "cd_max": float(np.max(cd[h])),
            "cl_min": float(np.min(cl[h])), "cl_max": float(np.max(cl[h])),
            "st": hlbm.strouhal(cl[h], w.chord, w.u_inf)}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--workload", default="naca_re1e4_c256", choices=sorted(workloads.PRESETS))
    ap.add_argument("--steps", type=int, default=0, help="finest steps (0: the preset's own)")
    ap.add_argument("--f2c-filter", action="store_true", help="filtered fine -> coarse transfer")
    a = ap.parse_args(argv)
    make = workloads.PRESETS[a.workload]
    kw = {"f2c_filter": True} if a.f2c_filter else {}
    if kw and "f2c_filter" not in inspect.signature(make).parameters:
        raise SystemExit(f"{a.workload} takes no f2c_filter")
    w = make(**kw)
    steps = a.steps or w.steps
    steps -= steps % (2 ** w.n_refine)
    out = {"workload": w.name, "finest_steps": steps, "window": [steps // 2, steps],
           "re": w.re, "aoa_deg": w.aoa_deg, "f2c_filter": bool(w.f2c_filter)}
    cd64, cl64, t64 = run(w, steps, hlbm.FP64)
    cd32, cl32, t32 = run(w, steps, hlbm.FP32_SHIFTED)
    s64, s32 = summary(cd64, cl64, w), summary(cd32, cl32, w)
    norm = max(abs(s64["cl_mean"]), abs(s64["cd_mean"]))
    d = np.abs(cd32 - cd64) / np.abs(cd64).max()
    tenth = max(1, steps // 10)
    out.update({"fp64": dict(s64, seconds=round(t64, 2)), "fp32": dict(s32, seconds=round(t32, 2)),
                "cd_mean_rel_err": abs(s32["cd_mean"] - s64["cd_mean"]) / abs(s64["cd_mean"]),
                "cl_mean_err_over_max_abs_cl_cd": abs(s32["cl_mean"] - s64["cl_mean"]) / norm,
                "st_rel_err": (abs(s32["st"] - s64["st"]) / s64["st"]) if np.isfinite(s64["st"]) else None,
                "cd_step_diff_over_max_cd_per_tenth": [float(f"{d[i:i + tenth].max():.2e}")
                                                        for i in range(0, steps, tenth)]})
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
