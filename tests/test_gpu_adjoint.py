"""Discrete adjoint of the HLBM step (FP64, single structured level) on the GPU.

Checked against central finite differences of the GPU forward and of the CPU
oracle forward (the oracle's gradient), the mirror symmetry dC_D/dalpha = 0 at
zero incidence, independence of the checkpoint interval, and the
torch.autograd.Function wrapper.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2006_10487_amd import hlbm, workloads as W

pytestmark = pytest.mark.gpu

SPEC = dict(t_end=160, t0=80, t1=160, ckpt_every=40, w_cd=1.0, w_cl=0.0)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    hlbm.lib()


def gpu_J(w, aoa, tau, n_sub, spec=SPEC):
    sim = hlbm.HLBM.from_workload(w, aoa_rad=aoa, tau=tau, n_sub=n_sub)
    J = sim.run_objective(**spec)
    return J, sim


def oracle_J(w, aoa, tau, n_sub, spec=SPEC):
    o = O.Oracle.from_workload(w, aoa_rad=aoa, tau_s=tau, n_sub=n_sub)
    o.step(spec["t_end"])
    cd, cl = o.history()
    s = slice(spec["t0"], spec["t1"])
    return float(np.mean(spec["w_cd"] * cd[s] + spec["w_cl"] * cl[s]))


def test_adjoint_matches_finite_differences():
    w = W.naca_re100_c40(3.0)
    a0, t0 = w.aoa_rad, w.tau_s
    n_sub = 17
    J, sim = gpu_J(w, a0, t0, n_sub)
    g = sim.adjoint(1.0)
    ha, ht = 1e-6, 1e-7
    fd_a = (gpu_J(w, a0 + ha, t0, n_sub)[0] - gpu_J(w, a0 - ha, t0, n_sub)[0]) / (2 * ha)
    fd_t = (gpu_J(w, a0, t0 + ht, n_sub)[0] - gpu_J(w, a0, t0 - ht, n_sub)[0]) / (2 * ht)
    ofd_a = (oracle_J(w, a0 + ha, t0, n_sub) - oracle_J(w, a0 - ha, t0, n_sub)) / (2 * ha)
    ofd_t = (oracle_J(w, a0, t0 + ht, n_sub) - oracle_J(w, a0, t0 - ht, n_sub)) / (2 * ht)
    print(f"J {J:.12f}  adjoint {g}  gpu FD [{fd_a:.10g}, {fd_t:.10g}]  oracle FD [{ofd_a:.10g}, {ofd_t:.10g}]",
          flush=True)
    assert abs(g[0] - fd_a) < 1e-6 * max(1.0, abs(fd_a))
    assert abs(g[1] - fd_t) < 1e-5 * max(1.0, abs(fd_t))
    assert abs(g[0] - ofd_a) < 1e-5 * max(1.0, abs(ofd_a))
    assert abs(g[1] - ofd_t) < 1e-4 * max(1.0, abs(ofd_t))


def test_adjoint_lift_objective_and_symmetry():
    """alpha = 0: dC_D/dalpha vanishes by mirror symmetry; the lift slope does not."""
    w = W.naca_re100_c40(0.0)
    spec = dict(SPEC, w_cd=1.0, w_cl=0.0)
    _, sim = gpu_J(w, 0.0, w.tau_s, 17, spec)
    gd = sim.adjoint()
    spec_l = dict(SPEC, w_cd=0.0, w_cl=1.0)
    _, sim = gpu_J(w, 0.0, w.tau_s, 17, spec_l)
    gl = sim.adjoint()
    h = 1e-6
    fd_l = (gpu_J(w, h, w.tau_s, 17, spec_l)[0] - gpu_J(w, -h, w.tau_s, 17, spec_l)[0]) / (2 * h)
    print("drag grad", gd, "lift grad", gl, "lift FD", fd_l, flush=True)
    assert abs(gd[0]) < 1e-9
    assert abs(gl[0] - fd_l) < 1e-6 * max(1.0, abs(fd_l))
    assert abs(gl[0]) > 1e-3


def test_adjoint_checkpoint_interval_independent():
    w = W.naca_re100_c40(3.0)
    g = []
    for k in (20, 160):
        _, sim = gpu_J(w, w.aoa_rad, w.tau_s, 17, dict(SPEC, ckpt_every=k))
        g.append(sim.adjoint())
    assert np.array_equal(g[0], g[1])


def test_autograd_function():
    import torch
    w = W.naca_re100_c40(3.0)
    F = hlbm.objective_function()
    aoa = torch.tensor(w.aoa_rad, dtype=torch.float64, requires_grad=True)
    tau = torch.tensor(w.tau_s, dtype=torch.float64, requires_grad=True)
    J = F.apply(aoa, tau, w, SPEC)
    J.backward()
    _, sim = gpu_J(w, w.aoa_rad, w.tau_s, 17)
    g = sim.adjoint()
    assert abs(aoa.grad.item() - g[0]) < 1e-12 * max(1, abs(g[0]))
    assert abs(tau.grad.item() - g[1]) < 1e-12 * max(1, abs(g[1]))
