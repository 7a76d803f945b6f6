"""Mean wall coefficients C_p, C_f, C_n (eqs. (12)-(13)) on the GPU against the oracle.

FP64: element-wise within 1e-11 relative (to the largest magnitude of each
coefficient) after windows that start mid-run, on the single-level case, the
one-box refined case and the Re = 1000 geometry (512 wall nodes, several
blocks).  FP32-shifted: the same means within 1e-4.  Also the
call-order rules and the profiler class.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2006_10487_amd import hlbm, workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-11


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    hlbm.lib()


def run_pair(w, before, steps, precision=hlbm.FP64):
    sim = hlbm.HLBM.from_workload(w, precision=precision)
    ref = O.Oracle.from_workload(w)
    sim.step(before)
    ref.step(before)
    sim.wall_stats_begin()
    ref.wall_stats_begin()
    sim.step(steps)
    ref.step(steps)
    return sim, sim.wall_stats(), ref.wall_stats()


def errors(g, r):
    out = {}
    for name, a, b in zip(("cp", "cf", "cn"), g[1:], r[1:]):
        assert a.shape == b.shape
        out[name] = float(np.abs(a - b).max() / np.abs(b).max())
    print("wall stats parity:", out, flush=True)
    return out


@pytest.mark.parametrize("case", ["re100_c40_a6", "re100_c40_refined_a3", "re1000_c128_a10"])
def test_wall_stats_fp64_match_oracle(case):
    if case == "re100_c40_a6":
        w, before, steps = W.naca_re100_c40(6.0), 40, 120
    elif case == "re100_c40_refined_a3":
        w, before, steps = W.naca_re100_c40_refined(3.0), 20, 40
    else:
        w, before, steps = W.naca_re1000_c128(10.0), 4, 6
    sim, g, r = run_pair(w, before, steps)
    assert g[0] == r[0] == steps
    assert g[1].size == w.omesh.ns
    e = errors(g, r)
    assert max(e.values()) < TOL


def test_wall_stats_fp32_shifted():
    w = W.naca_re100_c40(6.0)
    sim, g, r = run_pair(w, 300, 300, precision=hlbm.FP32_SHIFTED)
    e = errors(g, r)
    # FP32 storage of the populations (measured ~4e-6 on each coefficient)
    assert max(e.values()) < 1e-4


def test_wall_stats_call_order_and_profile():
    w = W.naca_re100_c40(3.0)
    sim = hlbm.HLBM.from_workload(w)
    with pytest.raises(hlbm.HLBMError) as ei:
        sim.wall_stats()
    assert ei.value.code == -6
    sim.wall_stats_begin()
    with pytest.raises(hlbm.HLBMError):
        sim.wall_stats()                      # no step yet
    sim.profile(True)
    sim.step(5)
    prof = sim.profile_read()
    assert prof["wall_stats"][1] == 5 and prof["wall_force"][1] == 5
    assert sim.wall_stats()[0] == 5
    # a new begin clears the sums
    sim.wall_stats_begin()
    sim.step(3)
    assert sim.wall_stats()[0] == 3
    # importing a state ends the accumulation
    sim.set_state(hlbm.PART_MESH, sim.get_state(hlbm.PART_MESH))
    with pytest.raises(hlbm.HLBMError):
        sim.wall_stats()
    # so does an objective run
    sim.wall_stats_begin()
    sim.step(2)
    sim.run_objective(t_end=20, t0=10, t1=20, ckpt_every=10, store_substeps=False)
    with pytest.raises(hlbm.HLBMError):
        sim.wall_stats()
