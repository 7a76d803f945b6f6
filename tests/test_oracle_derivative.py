"""Pins of the oracle's reference gradient (complex-step build of the oracle).

The complex-step build computes, in its imaginary parts, exact directional
derivatives of the same arithmetic the FP64 build runs.  These tests tie it to
things outside itself:
  * its real part is the FP64 oracle, bit for bit;
  * its derivatives agree with central finite differences of the FP64 oracle
    (angle of attack, tau, mesh shape) to the finite-difference error;
  * mirror symmetry: at zero incidence on a mirror-symmetric mesh the drag is
    even in alpha, so dC_D/dalpha vanishes, while the lift slope does not;
  * the bump tangent of the mesh generator equals its finite differences.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2006_10487_amd import workloads as W

SPEC = dict(t_end=120, t0=60, t1=120, w_cd=1.0, w_cl=0.0)
N_SUB = 17


def plain_J(w, spec=SPEC, aoa=None, tau=None, xy=None):
    if xy is not None:
        w = W.Workload(**{**w.__dict__, "mesh_xy": xy})
    o = O.Oracle.from_workload(w, aoa_rad=aoa, tau_s=tau, n_sub=N_SUB)
    o.step(spec["t_end"])
    cd, cl = o.history()
    s = slice(spec["t0"], spec["t1"])
    return float(np.mean(spec["w_cd"] * cd[s] + spec["w_cl"] * cl[s]))


def test_real_part_is_the_fp64_oracle():
    w = W.naca_re100_c40(3.0, bumps=W.hh_amplitudes(1))
    rng = np.random.default_rng(5)
    J, _ = O.objective_derivative(w, SPEC, d_aoa=0.7, d_tau=-0.3, d_xy=rng.standard_normal(w.mesh_xy.shape),
                                  n_sub=N_SUB)
    assert J == plain_J(w)


@pytest.mark.parametrize("what", ["aoa", "tau"])
def test_derivative_matches_finite_differences(what):
    w = W.naca_re100_c40(3.0)
    a0, t0 = w.aoa_rad, w.tau_s
    if what == "aoa":
        _, d = O.objective_derivative(w, SPEC, d_aoa=1.0, n_sub=N_SUB)
        h = 1e-6
        fd = (plain_J(w, aoa=a0 + h, tau=t0) - plain_J(w, aoa=a0 - h, tau=t0)) / (2 * h)
    else:
        _, d = O.objective_derivative(w, SPEC, d_tau=1.0, n_sub=N_SUB)
        h = 1e-7
        fd = (plain_J(w, aoa=a0, tau=t0 + h) - plain_J(w, aoa=a0, tau=t0 - h)) / (2 * h)
    print(what, d, fd)
    assert abs(d - fd) < 2e-6 * max(1.0, abs(fd))
    assert abs(d) > 1e-3


def test_shape_derivative_matches_finite_differences():
    """Along the tangent of two Hicks-Henne bumps (upper surface near x/c = 0.3, 0.6)."""
    amps = W.hh_amplitudes(0)
    w = W.naca_re100_c40(3.0, bumps=amps)
    tan = w.omesh.bump_tangent(W.HH_PEAKS)
    v = tan[2] - 0.5 * tan[5]
    _, d = O.objective_derivative(w, SPEC, d_xy=v, n_sub=N_SUB)
    h = 1e-5
    da = np.zeros(8)
    da[2], da[5] = 1.0, -0.5
    Jp = plain_J(W.naca_re100_c40(3.0, bumps=amps + h * da))
    Jm = plain_J(W.naca_re100_c40(3.0, bumps=amps - h * da))
    fd = (Jp - Jm) / (2 * h)
    print("shape", d, fd)
    assert abs(d - fd) < 1e-5 * max(1.0, abs(fd))
    assert abs(d) > 1e-2


def test_zero_incidence_symmetry():
    w = W.naca_re100_c40(0.0)
    _, dd = O.objective_derivative(w, SPEC, d_aoa=1.0, n_sub=N_SUB)
    _, dl = O.objective_derivative(w, dict(SPEC, w_cd=0.0, w_cl=1.0), d_aoa=1.0, n_sub=N_SUB)
    print("dCd/da", dd, "dCl/da", dl)
    assert abs(dd) < 1e-10
    assert dl > 0.05


def test_bump_tangent_matches_generator():
    amps = W.hh_amplitudes(3)
    om = W.naca_re100_c40(0.0, bumps=amps).omesh
    tan = om.bump_tangent(W.HH_PEAKS)
    for m in (0, 4, 7):
        e = np.zeros(8)
        e[m] = 1e-3
        xp = W.naca_re100_c40(0.0, bumps=amps + e).mesh_xy
        xm = W.naca_re100_c40(0.0, bumps=amps - e).mesh_xy
        fd = (xp - xm) / 2e-3
        assert np.abs(fd - tan[m]).max() < 1e-9
    # wall nodes move, the outer (interpolation) ring does not
    assert np.abs(tan[:, :om.ns, 1]).max() > 1.0
    assert np.abs(tan[:, om.nl * om.ns:, :]).max() == 0.0


@pytest.mark.parametrize("f2c_filter", [False, True])
def test_refined_derivative_matches_finite_differences(f2c_filter):
    """One refinement box: the derivative crosses the coarse <-> fine transfers
    (fine -> coarse pointwise, and with the f^neq full-weighted over 3 x 3 fine
    nodes, where the real part must still be the FP64 oracle bit for bit)."""
    import dataclasses
    w = dataclasses.replace(W.naca_re100_c40_refined(3.0), f2c_filter=f2c_filter)
    J, d = O.objective_derivative(w, SPEC, d_tau=1.0, n_sub=N_SUB)
    assert J == plain_J(w)
    h = 1e-7
    fd = (plain_J(w, tau=w.tau_s + h) - plain_J(w, tau=w.tau_s - h)) / (2 * h)
    print("refined tau", d, fd)
    assert abs(d - fd) < 2e-6 * max(1.0, abs(fd))
