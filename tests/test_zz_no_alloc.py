"""hlbm_create_noalloc (static per-device workspace, no allocation) against
hlbm_create with a caller workspace: the same kernels on the same inputs, so
every state and force is expected bit for bit equal.  Two calls in a row, the
second with a smaller problem (a different geometry and precision over the
array the first one used), and a problem too large for the array."""
import numpy as np
import pytest

from paper_2006_10487_amd import hlbm, workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    hlbm.lib()


def _state(sim):
    parts = list(range(sim.info.n_levels)) + [hlbm.PART_MESH]
    return [sim.get_state(p) for p in parts]


def _run(w, precision, steps, noalloc):
    sim = hlbm.HLBM.from_workload(w, precision=precision, noalloc=noalloc)
    assert (sim.workspace is None) == noalloc
    sim.step(steps)
    out = (np.asarray(sim.history(0, steps)), _state(sim))
    sim.close()
    return out


@pytest.mark.parametrize("case", ["re100_fp64", "re100_refined_fp32"])
def test_noalloc_equals_create(case):
    w, precision = {"re100_fp64": (W.naca_re100_c40(3.0), hlbm.FP64),
                    "re100_refined_fp32": (W.naca_re100_c40_refined(3.0), hlbm.FP32_SHIFTED)}[case]
    g, m, keep = hlbm.structs_from_workload(w, precision=precision)
    need = hlbm.workspace_size(g, m, 0.0, w.tau_s)
    assert need <= 64 << 20
    print(f"{case}: workspace {need} bytes", flush=True)
    h_ref, s_ref = _run(w, precision, 40, noalloc=False)
    h_na, s_na = _run(w, precision, 40, noalloc=True)
    assert np.array_equal(h_ref, h_na)
    for a, b in zip(s_ref, s_na):
        assert np.array_equal(a, b)


def test_noalloc_two_calls_second_smaller():
    """Two contexts in a row on the static array: the larger FP64 problem, then a
    smaller FP32 one that reuses the array the first left behind."""
    w1, w2 = W.naca_re100_c40(3.0), W.naca_re100_c40_refined(3.0)
    sizes = []
    for w, precision in ((w1, hlbm.FP64), (w2, hlbm.FP32_SHIFTED)):
        g, m, keep = hlbm.structs_from_workload(w, precision=precision)
        sizes.append(hlbm.workspace_size(g, m, 0.0, w.tau_s))
        h_na, s_na = _run(w, precision, 20, noalloc=True)
        h_ref, s_ref = _run(w, precision, 20, noalloc=False)
        assert np.array_equal(h_ref, h_na)
        for a, b in zip(s_ref, s_na):
            assert np.array_equal(a, b)
    assert sizes[1] < sizes[0]


def test_noalloc_rejects_a_problem_beyond_the_array():
    w = W.naca_re1000_c128()
    g, m, keep = hlbm.structs_from_workload(w, precision=hlbm.FP64)
    assert hlbm.workspace_size(g, m, 0.0, w.tau_s) > 64 << 20
    with pytest.raises(hlbm.HLBMError) as ei:
        hlbm.HLBM(g, m, tau=w.tau_s, keep=keep, noalloc=True)
    assert ei.value.code == -7
    assert "static workspace" in str(ei.value)
