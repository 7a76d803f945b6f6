"""Writes the FP64 oracle's drag and lift history of the Re = 1e4 workload.

The workload is the NACA 0012 at zero incidence, chord 256 lu, a 2048 x 1024
base grid with two nested factor-two boxes, and a 1024 x 128 O-mesh
(`workloads.naca_re1e4_c256`).  The script runs the first STEPS finest steps of
the plain FP64 CPU oracle from the initial state and stores C_D and C_L of
every step (eqs. (10)-(11)).  The GPU tests compare the library's FP64 history
with it and state the FP32-shifted deviation from it.  With these settings the
run turns non-finite at finest step 1482: the velocity first grows at the
upstream edge of the finest box, where the middle level (tau 0.5015) hands its
values to the finest one, the refinement-interface growth that sets in for a
coarse tau close to 1/2.  From there on the stored values are nan.  It calls
only the oracle and the input generator.  With --filtered it runs the same
workload with the fine -> coarse f^neq full-weighted over 3 x 3 fine nodes,
which stays finite, into naca_re1e4_c256_f2c3x3_fp64_history.txt.  Each run
takes about an hour on 8 cores:

    python tests/golden/make_re1e4_history.py [steps] [--filtered]
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O                      # noqa: E402
from paper_2006_10487_amd import workloads as W     # noqa: E402

OUT = os.path.join(HERE, "naca_re1e4_c256_fp64_history.txt")
OUT_FILTERED = os.path.join(HERE, "naca_re1e4_c256_f2c3x3_fp64_history.txt")


def main(steps: int = 2000, chunk: int = 100, filtered: bool = False) -> None:
    w = W.naca_re1e4_c256(f2c_filter=filtered)
    out = OUT_FILTERED if filtered else OUT
    o = O.Oracle.from_workload(w)
    t0 = time.time()
    done = 0
    while done < steps:
        n = min(chunk, steps - done)
        o.step(n)
        done += n
        print(f"{done} steps, {time.time() - t0:.0f} s", flush=True)
    cd, cl = o.history()
    tmp = out + ".tmp"
    with open(tmp, "w") as fh:
        fh.write(f"# workload {w.name}: Re {w.re:g}, aoa {w.aoa_deg:g} deg, chord {w.chord:g} lu, "
                 f"tau_s {w.tau_s!r}, n_sub {o.n_sub}, FP64 CPU oracle\n")
        fh.write("# finest step t (0-based), C_D, C_L after step t\n")
        for t in range(len(cd)):
            fh.write(f"{t} {float(cd[t])!r} {float(cl[t])!r}\n")
    os.replace(tmp, out)


if __name__ == "__main__":
    args = [a for a in sys.argv[1:] if not a.startswith("--")]
    main(int(args[0]) if args else 2000, filtered="--filtered" in sys.argv[1:])
