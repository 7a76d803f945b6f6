"""Writes the grid struct bytes and mesh arrays of several workloads (one .bin file each) into the
directory given as argument, as input of plan_main.cpp (the host-side sanitizer run)."""
import os, sys, ctypes as C, struct
sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
import numpy as np
from paper_2006_10487_amd import hlbm, workloads as W
cases = [
    ("bench_fp32", W.naca_re5000_c512(), hlbm.FP32_SHIFTED, 0),
    ("bench_fp64", W.naca_re5000_c512(), hlbm.FP64, 0),
    ("re1000_fp32_f3", W.naca_re1000_c128(10.0), hlbm.FP32_SHIFTED, 3),
    ("re1000_fp64_f4", W.naca_re1000_c128(10.0), hlbm.FP64, 4),
    ("re100_refined", W.naca_re100_c40_refined(3.0, bumps=W.hh_amplitudes(1)), hlbm.FP64, 2),
    ("re1e4", W.naca_re1e4_c256(), hlbm.FP32_SHIFTED, 0),
    ("four_levels", W.naca_re500_four_levels(48), hlbm.FP64, 0),
]
for name, w, prec, fuse in cases:
    g, m, keep = hlbm.structs_from_workload(w, precision=prec, interp=hlbm.INTERP_QUADRATIC, n_sub=w.n_sub,
                                            wall_bc=True, aoa_rad=w.aoa_rad, check_every=0, history_len=0,
                                            fv_fuse=fuse)
    gb = bytes(C.string_at(C.addressof(g), C.sizeof(g)))
    nn, nt = m.n_nodes, m.n_tris
    xy = np.ctypeslib.as_array(m.xy, shape=(2 * nn,)).astype(np.float64) if nn else np.zeros(0)
    tri = np.ctypeslib.as_array(m.tri, shape=(3 * nt,)).astype(np.int32) if nt else np.zeros(0, np.int32)
    kind = np.ctypeslib.as_array(m.kind, shape=(nn,)).astype(np.uint8) if nn else np.zeros(0, np.uint8)
    with open(os.path.join(sys.argv[1], f'{name}.bin'), 'wb') as f:
        f.write(struct.pack('<iid4dd', len(gb), 0, 0.0, *list(m.inner_ellipse), m.chord))
        f.write(gb)
        f.write(struct.pack('<ii', nn, nt))
        f.write(xy.tobytes()); f.write(tri.tobytes()); f.write(kind.tobytes())
        f.write(struct.pack('<d', w.tau_s))
    print(name, C.sizeof(g), nn, nt)
