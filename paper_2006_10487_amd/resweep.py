"""Reynolds-number sweep at zero incidence (Sec. 6.2) in FP64 and FP32-shifted.

Workload ``workloads.naca_re_sweep(re)`` (c = 512, two structured levels, thin
O-mesh band; ``--f2c-filter`` for the filtered fine -> coarse transfer).  Each
run starts from the uniform state and lasts ``passes`` chord-transit times;
C_D, C_L and the Strouhal number of the lift are taken over the last 40 % of
it.  The paper's drag at these Reynolds numbers (its table of C_D against Re,
computed at c = 1024) is printed beside as context.

    python -m paper_2006_10487_amd.resweep --re 1000,2000,5000,10000 --passes 20

prints one JSON object per Reynolds number.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import hlbm, workloads

PAPER_CD = {1000: 0.119, 2000: 0.084, 5000: 0.052, 10000: 0.037}


def run(re: float, passes: float, precision: int, mesh: dict):
    w = workloads.naca_re_sweep(re, **mesh)
    per = 2 ** w.n_refine
    steps = int(round(passes * w.chord / w.u_inf / per)) * per
    sim = hlbm.HLBM.from_workload(w, precision=precision, history_len=steps + 8, check_every=2000)
    n_sub = int(sim.info.n_sub)
    t0 = time.perf_counter()
    sim.step_logged(steps, w.name)
    dt = time.perf_counter() - t0
    cd, cl = sim.history()
    sim.close()
    win = slice(steps - (2 * steps) // 5, steps)
    return (w, steps, n_sub, dt, float(np.mean(cd[win])), float(np.mean(cl[win])),
            hlbm.strouhal(cl[win], w.chord, w.u_inf))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--re", default="1000,2000,5000,10000")
    ap.add_argument("--passes", type=float, default=20.0, help="chord-transit times per run")
    ap.add_argument("--no-fp64", action="store_true", help="FP32-shifted runs only")
    ap.add_argument("--ns", type=int, default=1280, help="surface points of the O-mesh")
    ap.add_argument("--d-out", type=float, default=0.19, help="outer ellipse beyond the chord, in chords")
    ap.add_argument("--nl", type=int, default=64, help="O-mesh layers")
    ap.add_argument("--h1", type=float, default=0.8, help="first layer height (lu)")
    ap.add_argument("--f2c-filter", action="store_true", help="filtered fine -> coarse transfer")
    a = ap.parse_args(argv)
    mesh = dict(ns=a.ns, d_out=a.d_out, nl=a.nl, h1=a.h1, f2c_filter=a.f2c_filter)
    for re in [float(x) for x in a.re.split(",")]:
        out = {"re": re, "passes": a.passes}
        try:
            w, steps, n_sub, t32, cd32, cl32, st32 = run(re, a.passes, hlbm.FP32_SHIFTED, mesh)
            out.update({"workload": w.name, "finest_steps": steps, "n_sub": n_sub, "mesh_nodes": int(w.mesh_xy.shape[0]),
                        "fp32_shifted": {"cd": cd32, "cl": cl32, "st": st32, "seconds": round(t32, 2)},
                        "paper_cd_c1024": PAPER_CD.get(int(re))})
            if not a.no_fp64:
                _, _, _, t64, cd64, cl64, st64 = run(re, a.passes, hlbm.FP64, mesh)
                out["fp64"] = {"cd": cd64, "cl": cl64, "st": st64, "seconds": round(t64, 2)}
                out["cd_rel_err"] = abs(cd32 - cd64) / abs(cd64)
                out["cl_abs_err"] = abs(cl32 - cl64)
                out["st_rel_err"] = (abs(st32 - st64) / st64) if (math.isfinite(st32) and math.isfinite(st64)) else None
        except hlbm.HLBMError as e:
            out["error"] = str(e)
        print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
