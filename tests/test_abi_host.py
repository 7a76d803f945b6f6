"""Host-only checks of the C ABI: the library loads without a GPU, exports every
function declared in include/hlbm.h, and rejects bad problems before any device
work (hlbm_validate / hlbm_workspace_size)."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

from paper_2006_10487_amd import hlbm, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(hlbm.LIB_PATH):
        from paper_2006_10487_amd import build
        build.build()
    return hlbm.lib()


def test_header_symbols_exported(lib):
    text = open(os.path.join(ROOT, "include", "hlbm.h")).read()
    declared = set(re.findall(r"\b(hlbm_[a-z_]+)\s*\(", text))
    assert declared == set(hlbm.EXPORTED)
    for name in declared:
        assert hasattr(lib, name), name


def test_struct_sizes_match_header(lib):
    # hlbm_grid: 15 int32 (60 B, padded to 64), 3 doubles, 9 int32 (36 B, padded to 40)
    assert C.sizeof(hlbm.Grid) == 64 + 3 * 8 + 40
    # hlbm_mesh: 2 int32, 3 pointers, 5 doubles, int32 n_shape (padded to 8), 1 pointer,
    # int32 body_n (padded to 8), 1 pointer
    assert C.sizeof(hlbm.Mesh) == 4 + 4 + 3 * 8 + 8 + 32 + 8 + 8 + 8 + 8


def test_struct_layouts_match_compiled_header(tmp_path):
    """Size and every field offset of the binding's structs against the C compiler's
    reading of include/hlbm.h."""
    structs = {"hlbm_grid": hlbm.Grid, "hlbm_mesh": hlbm.Mesh, "hlbm_info_t": hlbm.Info,
               "hlbm_objective": hlbm.Objective}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "hlbm.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for f in py._fields_:
            lines.append(f'printf("{cname} {f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    import subprocess
    subprocess.check_call(["gcc", "-std=c11", "-I", inc, str(src), "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)], text=True).splitlines():
        cname, field, value = line.split()
        got[(cname, field)] = int(value)
    for cname, py in structs.items():
        assert got[(cname, "sizeof")] == C.sizeof(py), cname
        for f in py._fields_:
            assert got[(cname, f[0])] == getattr(py, f[0]).offset, (cname, f[0])


def _small(**kw):
    w = W.naca_re100_c40()
    return hlbm.structs_from_workload(w, **kw), w


def test_validate_ok_and_workspace(lib):
    (g, m, keep), w = _small()
    assert hlbm.validate(g, m, 0.0, w.tau_s) == 0
    assert hlbm.validate(g, m, w.re, 0.0) == 0
    n = hlbm.workspace_size(g, m, 0.0, w.tau_s)
    # two FP64 buffers of the 241 x 121 grid at least
    assert n > 2 * 9 * 121 * 241 * 8
    (g32, m32, keep32), _ = _small(precision=hlbm.FP32_SHIFTED)
    assert hlbm.workspace_size(g32, m32, 0.0, w.tau_s) < n


def test_validate_errors(lib):
    (g, m, keep), w = _small()
    assert hlbm.validate(g, m, 0.0, 0.5) == -3                 # tau <= 1/2
    assert hlbm.validate(g, m, 0.0, 0.0) == -3                 # neither Re nor tau
    assert hlbm.validate(g, m, 123.0, w.tau_s) == -3           # Re and tau disagree
    # clockwise triangle
    tri = w.mesh_tri.copy()
    tri[5, 1], tri[5, 2] = tri[5, 2], tri[5, 1]
    g2, m2, k2 = hlbm.structs_from_workload(w, mesh_tri=tri)
    assert hlbm.validate(g2, m2, 0.0, w.tau_s) == -2
    assert "counter-clockwise" in hlbm.last_error()
    # inner ellipse reaching past the mesh: structured interpolation node outside the mesh
    g3, m3, k3 = hlbm.structs_from_workload(w, inner_ellipse=(100.0, 60.0, 80.0, 50.0))
    assert hlbm.validate(g3, m3, 0.0, w.tau_s) == -2
    # mesh interpolation node whose 3x3 donors fall inside the inactive region
    g4, m4, k4 = hlbm.structs_from_workload(w, inner_ellipse=(100.0, 60.0, 71.0, 51.0))
    assert hlbm.validate(g4, m4, 0.0, w.tau_s) == -2
    # odd box size / box outside its parent
    g5, m5, k5 = hlbm.make_structs(64, 32, [(4, 4, 31, 20)], periodic=True)
    assert hlbm.validate(g5, m5, 0.0, 0.6) == -2
    g6, m6, k6 = hlbm.make_structs(64, 32, [(40, 4, 60, 20)], periodic=True)
    assert hlbm.validate(g6, m6, 0.0, 0.6) == -2
    g7, m7, k7 = hlbm.make_structs(64, 32, [(8, 4, 40, 20)], periodic=True)
    assert hlbm.validate(g7, m7, 0.0, 0.6) == 0


def test_validate_bad_enums(lib):
    (g, m, keep), w = _small(precision=7)
    assert hlbm.validate(g, m, 0.0, w.tau_s) == -1


def test_f2c_filter_option(lib):
    """The four-level layout with the filtered fine -> coarse transfer validates for
    every chord of the convergence family; values other than 0 and 1 are rejected."""
    for c in W.CONV_CHORDS:
        w = W.naca_re500_four_levels(c, f2c_filter=True)
        assert w.n_refine == 3 and w.f2c_filter
        g, m, keep = hlbm.structs_from_workload(w)
        assert g.f2c_filter == 1 and hlbm.validate(g, m, 0.0, w.tau_s) == 0, (c, hlbm.last_error())
    g.f2c_filter = 2
    assert hlbm.validate(g, m, 0.0, w.tau_s) == -1 and "f2c_filter" in hlbm.last_error()


def test_workloads_validate(lib):
    """Every preset passes host validation (stencils, boxes, inner ellipse)."""
    for name in ("naca_re100_c40", "naca_re1000_c128", "naca_re1e4_c256", "naca_re1000_c128_bumps"):
        w = W.PRESETS[name]()
        g, m, keep = hlbm.structs_from_workload(w)
        assert hlbm.validate(g, m, 0.0, w.tau_s) == 0, (name, hlbm.last_error())
    # the four-level convergence family: every chord, one FV time step
    for c in W.CONV_CHORDS:
        w = W.naca_re500_conv(c)
        assert w.n_refine == W.FAMILY_BOXES and w.n_sub == W.CONV_N_SUB
        assert 2 ** w.n_refine * w.re / w.chord <= 21.0      # coarse-level cell Reynolds number
        g, m, keep = hlbm.structs_from_workload(w)
        assert hlbm.validate(g, m, 0.0, w.tau_s) == 0, (c, hlbm.last_error())
        assert abs(w.tau_s - (0.5 + 3 * 0.05 * c / 500.0)) < 1e-12
        assert W.CONV_N_SUB >= 1.0 / (w.tau_s - 0.5)
    w = W.naca_re500_four_levels(48)
    g, m, keep = hlbm.structs_from_workload(w)
    assert w.n_refine == 3 and hlbm.validate(g, m, 0.0, w.tau_s) == 0


def test_equivalent_lbm_workload(lib):
    """The eq. (14) comparison grid: one more box of half spacing over the finest box, no mesh,
    the same Reynolds number (chord doubled in the new finest units), the profile's wall
    points doubled as the body polygon."""
    for name in ("naca_re1000_c128", "naca_re5000_c512"):
        w = W.PRESETS[name]()
        e = W.equivalent_lbm(w)
        assert e.n_refine == w.n_refine + 1 and e.mesh_xy is None and e.chord == 2 * w.chord
        assert np.array_equal(e.body_xy, 2.0 * w.omesh.xy[w.omesh.surface_index])
        assert W.equivalent_lbm(w, body=False).body_xy is None
        px, py = w.patches[-1][2], w.patches[-1][3]
        assert e.patches[-1] == (8, 8, 2 * (px - 16), 2 * (py - 16))
        assert abs((e.tau_s - 0.5) - 2 * (w.tau_s - 0.5)) < 1e-12
        g, m, keep = hlbm.structs_from_workload(e)
        assert hlbm.validate(g, m, 0.0, e.tau_s) == 0, hlbm.last_error()


def test_richardson_fit_recovers_order():
    from paper_2006_10487_amd.convergence import richardson
    c = np.array([48, 64, 96, 128, 144], dtype=float)
    for p0, cinf0, k0 in ((2.0, 0.18, 40.0), (1.3, 0.05, -3.0)):
        p, cinf, K, rms = richardson(c, cinf0 + k0 * c ** -p0)
        assert abs(p - p0) < 1e-5 and abs(cinf - cinf0) < 1e-8 and rms < 1e-10


def test_strouhal_of_sinusoid():
    """Strouhal estimator on a synthetic lift signal of known period."""
    period = 1234.5
    t = np.arange(40000)
    cl = 0.3 + 0.2 * np.sin(2 * np.pi * t / period + 0.4)
    st = hlbm.strouhal(cl, chord=128.0, u_inf=0.05)
    assert abs(st - 128.0 / (0.05 * period)) < 1e-6 * st
    assert math.isnan(hlbm.strouhal(np.full(100, 0.1), 128.0, 0.05))


def test_body_option_validation(lib):
    """A body resolved by bounce-back: accepted without a mesh, rejected with one,
    near the edge of the finest level, or covering no node (host checks only)."""
    import dataclasses
    e = W.equivalent_lbm(W.naca_re100_c40_refined(0.0))
    g, m, keep = hlbm.structs_from_workload(e)
    assert hlbm.validate(g, m, 0.0, e.tau_s) == 0
    w = W.naca_re100_c40_refined(0.0)
    g, m, keep = hlbm.structs_from_workload(w, body_xy=2.0 * w.omesh.xy[w.omesh.surface_index])
    assert hlbm.validate(g, m, 0.0, w.tau_s) == -1
    ox = e.patches[0][0] * 4 + e.patches[1][0] * 2   # finest-level origin (finest lu)
    shifted = dataclasses.replace(e, body_xy=e.body_xy + np.array([ox + 3.0 - e.body_xy[:, 0].min(), 0.0]))
    g, m, keep = hlbm.structs_from_workload(shifted)
    assert hlbm.validate(g, m, 0.0, e.tau_s) == -2
    tiny = dataclasses.replace(e, body_xy=np.array([[300.2, 100.2], [300.6, 100.2], [300.4, 100.6]]))
    g, m, keep = hlbm.structs_from_workload(tiny)
    assert hlbm.validate(g, m, 0.0, e.tau_s) == -2


def _bench_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "bench_mod", os.path.join(os.path.dirname(__file__), os.pardir, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_traffic_record_applies_only_to_its_kernels_and_launch_shape(tmp_path):
    """The counter traffic is reported only while the forward kernels hash to the
    recorded value and, for the FV launch, the sub-steps per launch match."""
    import hashlib
    import json
    B = _bench_module()
    src = open(os.path.join(os.path.dirname(B.__file__), "paper_2006_10487_amd", "csrc", "kernels.hip")).read()
    sha = hashlib.sha256(src[:src.index(B.ADJOINT_MARKER)].encode()).hexdigest()
    rec = {"forward_kernels_sha256": sha, "fv_substep": {"traffic_bytes": 1234.4, "fv_fuse": 4},
           "collide_l0": {"traffic_bytes": 99.6}}
    f = tmp_path / "traffic.md"
    f.write_text("# summary\n\n```json\n" + json.dumps(rec) + "\n```\n")
    B.TRAFFIC_SUMMARY = str(f)
    assert B.measured_traffic("fv_substep", 4) == 1234
    assert B.measured_traffic("fv_substep", 3) is None
    assert B.measured_traffic("collide_l0") == 100
    rec["forward_kernels_sha256"] = "0" * 64
    f.write_text("```json\n" + json.dumps(rec) + "\n```\n")
    assert B.measured_traffic("fv_substep", 4) is None and B.measured_traffic("collide_l0") is None
    B.TRAFFIC_SUMMARY = str(tmp_path / "missing.md")
    assert B.measured_traffic("collide_l0") is None


def test_committed_traffic_record_matches_the_committed_kernels():
    """profiles/ holds the counter summary of the kernels in this tree (four FV
    sub-steps per launch on the bench mesh): after a forward-kernel change the
    counters must be taken again, or bench.py reports null traffic."""
    B = _bench_module()
    assert isinstance(B.measured_traffic("fv_substep", 4), int)
    assert isinstance(B.measured_traffic("collide_l0"), int)
