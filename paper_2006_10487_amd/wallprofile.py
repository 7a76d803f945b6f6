"""Mean pressure and skin-friction coefficients on the airfoil and the separation
point (eqs. (12)-(13), Sec. 6) for the Re = 1000, c = 128 workload.

Runs `steps` finest steps from the uniform state, averages C_p and C_f at the
wall nodes over the second half (hlbm_wall_stats), and reports per surface the
distributions along x/c (C_f positive for attached flow) and the separation
point: the first zero of C_f with negative slope on the upper surface.

    python -m paper_2006_10487_amd.wallprofile --aoa 8 --steps 40000 --ns 2048

prints one JSON object (distributions sampled at 21 stations per surface).
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

from . import hlbm, workloads


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--aoa", type=float, default=8.0)
    ap.add_argument("--steps", type=int, default=40000)
    ap.add_argument("--ns", type=int, default=2048, help="surface points of the O-mesh")
    ap.add_argument("--band", type=float, default=workloads.RE1000_C128_DOUT)
    ap.add_argument("--nl", type=int, default=64)
    ap.add_argument("--fp32", action="store_true", help="FP32-shifted populations instead of FP64")
    a = ap.parse_args(argv)
    w = workloads.naca_re1000_c128(a.aoa, ns=a.ns, band=a.band, nl=a.nl)
    prec = hlbm.FP32_SHIFTED if a.fp32 else hlbm.FP64
    sim = hlbm.HLBM.from_workload(w, precision=prec, history_len=a.steps + 8, check_every=1000)
    sim.step_logged(a.steps // 2, w.name)
    sim.wall_stats_begin()
    sim.step_logged(a.steps - a.steps // 2, w.name)
    n, cp, cf, cn = sim.wall_stats()
    cd, cl = sim.history()
    sim.close()
    d = hlbm.surface_distributions(w.omesh, cp, cf)
    xs = np.linspace(0.0, 1.0, 21)
    out = {"workload": w.name, "aoa_deg": a.aoa, "steps_averaged": n,
           "precision": "fp32_shifted" if a.fp32 else "fp64",
           "cd": float(np.mean(cd[a.steps // 2:])), "cl": float(np.mean(cl[a.steps // 2:]))}
    for side in ("upper", "lower"):
        x, p, f = d[side]
        out[side] = {"separation_x_over_c": hlbm.separation_point(x, f),
                     "cp_min": float(p.min()), "x_cp_min": float(x[int(np.argmin(p))]),
                     "cp_le": float(p[0]), "cf_max": float(f.max()),
                     "x_stations": [round(float(v), 3) for v in xs],
                     "cp": [round(float(v), 4) for v in np.interp(xs, x, p)],
                     "cf": [round(float(v), 5) for v in np.interp(xs, x, f)]}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
