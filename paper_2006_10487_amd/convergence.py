"""Self-convergence study of the mean drag (Sec. 5).

Re = 500, alpha = 0, chords 48, 64, 96, 128, 144, FP64.  Two layouts:
``--levels 2`` (``workloads.naca_re500_conv``: a base grid of spacing 2 and
one box) and ``--levels 4`` (``workloads.naca_re500_four_levels``: the paper's
four structured levels, base spacing 8 and three nested boxes, with the
filtered fine -> coarse transfer that keeps its coarse levels stable at tau
close to 1/2).  Both have geometrically similar grids and boxes, the same wall
element size and FV time step for every chord.  Each run starts from the uniform state and lasts
``passes`` chord-transit times (c / U finest steps each); C_D is averaged over
the last tenth.  The paper measures the drag error against XFOIL; without an
external reference, the limit C_D(inf) and the order p come from a
least-squares fit of C_D(c) = C_D(inf) + K c^-p to the five chords
(Richardson extrapolation), and the errors are stated against that limit.

    python -m paper_2006_10487_amd.convergence --passes 40 [--levels 4]

prints one JSON object per chord and one for the fit.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import hlbm, workloads


def run(chord: int, passes: float, precision: int, levels: int = 2):
    w = workloads.naca_re500_conv(chord) if levels == 2 else workloads.naca_re500_four_levels(chord, f2c_filter=True)
    per = 2 ** w.n_refine
    steps = int(round(passes * chord / w.u_inf / per)) * per
    sim = hlbm.HLBM.from_workload(w, precision=precision, history_len=steps + 8, check_every=4000)
    t0 = time.perf_counter()
    sim.step_logged(steps, w.name)
    dt = time.perf_counter() - t0
    cd, cl = sim.history()
    sim.close()
    k = steps // 10
    last, prev = cd[-k:].mean(), cd[-2 * k:-k].mean()
    return w, steps, dt, float(last), float(abs(last - prev) / abs(last)), float(np.abs(cl[-k:]).max())


def richardson(chords, cd):
    """Least-squares C_D(c) = C_D(inf) + K c^-p: for each p the problem is
    linear in (C_D(inf), K); p minimises the residual (golden-section search)."""
    c = np.asarray(chords, dtype=np.float64)
    y = np.asarray(cd, dtype=np.float64)

    def fit(p):
        A = np.stack([np.ones_like(c), c ** -p], 1)
        sol, *_ = np.linalg.lstsq(A, y, rcond=None)
        return float(np.sum((A @ sol - y) ** 2)), sol

    lo, hi = 0.2, 6.0
    g = 0.5 * (np.sqrt(5.0) - 1.0)
    a, b = hi - g * (hi - lo), lo + g * (hi - lo)
    fa, fb = fit(a)[0], fit(b)[0]
    for _ in range(200):
        if fa < fb:
            hi, b, fb = b, a, fa
            a = hi - g * (hi - lo)
            fa = fit(a)[0]
        else:
            lo, a, fa = a, b, fb
            b = lo + g * (hi - lo)
            fb = fit(b)[0]
    p = 0.5 * (lo + hi)
    res, (cinf, K) = fit(p)
    return float(p), float(cinf), float(K), float(np.sqrt(res / len(c)))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--chords", default=",".join(str(c) for c in workloads.CONV_CHORDS))
    ap.add_argument("--passes", type=float, default=40.0, help="chord-transit times per run")
    ap.add_argument("--fp32", action="store_true", help="FP32-shifted populations instead of FP64")
    ap.add_argument("--levels", type=int, default=2, choices=(2, 4), help="structured levels of the layout")
    a = ap.parse_args(argv)
    prec = hlbm.FP32_SHIFTED if a.fp32 else hlbm.FP64
    chords = [int(x) for x in a.chords.split(",")]
    cds = []
    for c in chords:
        w, steps, dt, cd, drift, clmax = run(c, a.passes, prec, a.levels)
        cds.append(cd)
        print(json.dumps({"chord": c, "workload": w.name, "finest_steps": steps, "n_sub": w.n_sub,
                          "tau_s": w.tau_s, "mesh_nodes": int(w.mesh_xy.shape[0]), "cd": cd,
                          "cd_drift_last_tenth": drift, "cl_abs_max": clmax, "seconds": round(dt, 2)}),
              flush=True)
    if len(chords) >= 3:
        p, cinf, K, rms = richardson(chords, cds)
        print(json.dumps({"fit": "cd = cd_inf + K c^-p", "p": p, "cd_inf": cinf, "K": K, "rms": rms,
                          "err_pct": {str(c): 100.0 * (cd - cinf) / cinf for c, cd in zip(chords, cds)}}),
              flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
