"""Angle-of-attack sweep of the Re = 1000, c = 128 workload (or, with --family
re5000_c512, of the Re = 5000, c = 512 throughput workload) in FP64 and
FP32-shifted.

For every angle: time-averaged C_D and C_L over the second half of the run,
the Strouhal number of the lift signal, and the FP32-shifted deviations from
FP64 (relative; absolute for C_L where it vanishes by symmetry).

    python -m paper_2006_10487_amd.polar --aoa 0,5 --steps 40000 --ns 512
    python -m paper_2006_10487_amd.polar --family re5000_c512 --aoa 0,4,8,12 --steps 10000

prints one JSON object per angle.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import hlbm, workloads


def run(aoa_deg: float, steps: int, ns: int, precision: int, band: float, nl: int, family: str = "re1000_c128"):
    if family == "re5000_c512":
        w = workloads.naca_re5000_c512(aoa_deg, band=51.2 if band is None else band, nl=128 if nl is None else nl)
    else:
        w = workloads.naca_re1000_c128(aoa_deg, ns=ns, band=workloads.RE1000_C128_DOUT if band is None else band,
                                       nl=64 if nl is None else nl)
    sim = hlbm.HLBM.from_workload(w, precision=precision, history_len=steps + 8, check_every=1000)
    t0 = time.perf_counter()
    sim.step_logged(steps, w.name)
    dt = time.perf_counter() - t0
    cd, cl = sim.history()
    sim.close()
    win = slice(steps // 2, steps)
    return w, dt, float(np.mean(cd[win])), float(np.mean(cl[win])), hlbm.strouhal(cl[win], w.chord, w.u_inf)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--aoa", default="0,5,10,15,20")
    ap.add_argument("--steps", type=int, default=40000)
    ap.add_argument("--ns", type=int, default=512, help="surface points of the O-mesh")
    ap.add_argument("--band", type=float, default=None,
                    help="O-mesh band thickness (lu; default: the family's, 24 at c = 128, 51.2 at c = 512)")
    ap.add_argument("--nl", type=int, default=None, help="O-mesh layers (default: 64 at c = 128, 128 at c = 512)")
    ap.add_argument("--fp64-only", action="store_true", help="skip the FP32-shifted run")
    ap.add_argument("--family", default="re1000_c128", choices=["re1000_c128", "re5000_c512"],
                    help="workload family (re5000_c512: 2048 surface points, --ns unused)")
    a = ap.parse_args(argv)
    for aoa in [float(x) for x in a.aoa.split(",")]:
        out = {"aoa_deg": aoa, "steps": a.steps, "family": a.family,
               "ns": a.ns if a.family == "re1000_c128" else 2048}
        try:
            w, t64, cd64, cl64, st64 = run(aoa, a.steps, a.ns, hlbm.FP64, a.band, a.nl, a.family)
            if a.fp64_only:
                out.update({"workload": w.name, "mesh_nodes": int(w.mesh_xy.shape[0]),
                            "fp64": {"cd": cd64, "cl": cl64, "st": st64, "seconds": round(t64, 3)}})
                print(json.dumps(out), flush=True)
                continue
            _, t32, cd32, cl32, st32 = run(aoa, a.steps, a.ns, hlbm.FP32_SHIFTED, a.band, a.nl, a.family)
        except hlbm.HLBMError as e:
            out["error"] = str(e)
            print(json.dumps(out), flush=True)
            continue
        scale_l = abs(cl64) if abs(cl64) > 1e-6 else 1.0
        out.update({
            "workload": w.name, "mesh_nodes": int(w.mesh_xy.shape[0]),
            "fp64": {"cd": cd64, "cl": cl64, "st": st64, "seconds": round(t64, 3)},
            "fp32_shifted": {"cd": cd32, "cl": cl32, "st": st32, "seconds": round(t32, 3)},
            "cd_rel_err": abs(cd32 - cd64) / abs(cd64),
            "cl_err": abs(cl32 - cl64) / scale_l, "cl_err_kind": "relative" if scale_l != 1.0 else "absolute",
            "st_rel_err": (abs(st32 - st64) / st64) if (math.isfinite(st32) and math.isfinite(st64)) else None,
        })
        print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
