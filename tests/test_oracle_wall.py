"""Pins of the oracle's wall coefficients, eqs. (12)-(13), and the host-side
post-processing of them (surface distributions, separation point).

  * closed form: a state built from a prescribed density and a shear flow
    parallel to the wall (first-order Chapman-Enskog non-equilibrium part of
    the continuous BGK equation, viscosity c_s^2 tau_u) gives
    C_p = (rho - rho0) c_s^2 / q and C_f = mu du_t/dn / q against the exact
    (analytic) NACA 0012 normals, with a free-stream velocity added so that the
    rho u u part of the momentum flux is exercised;
  * the time means reproduce the mean drag and lift: the wall force is the
    trapezoidal sum of the wall-node momentum flux, so
    sum_P |V_P| (-C_p n + C_f t + C_n n) is the mean force coefficient;
  * mirror symmetry: alpha and -alpha give mirrored C_p, C_n and opposite
    C_f on mirrored nodes;
  * the separation point of synthetic C_f curves.
"""
import math

import numpy as np
import pytest

from flowfields import CX, CY
from oracle import oracle as O
from paper_2006_10487_amd import hlbm, workloads as W

CS2 = 1.0 / 3.0
WQ = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def analytic_normals(om):
    """Unit normals into the fluid of the exact NACA 0012 surface at the surface points."""
    xi = om.surface_xi
    with np.errstate(divide="ignore", invalid="ignore"):
        s = 0.6 * (0.2969 * 0.5 / np.sqrt(xi) - 0.1260 - 2 * 0.3516 * xi + 3 * 0.2843 * xi**2
                   - 4 * 0.1036 * xi**3)
    n = np.where(om.surface_upper[:, None], np.stack([-s, np.ones_like(s)], 1),
                 np.stack([-s, -np.ones_like(s)], 1))
    n[om.ns // 2] = (-1.0, 1e-300)
    return n / np.linalg.norm(n, axis=1)[:, None]


def test_wall_coefficients_closed_form():
    w = W.naca_re100_c40(0.0)
    om, ns = w.omesh, w.omesh.ns
    o = O.Oracle.from_workload(w)
    tau_u = o.tau_u
    n = analytic_normals(om)
    t = np.stack([n[:, 1], -n[:, 0]], 1)            # fluid on the left of t
    rng = np.random.default_rng(3)
    rho = 1.0 + 0.02 * rng.standard_normal(ns)
    dudn = 1e-3 * (1.0 + rng.random(ns))             # du_t / dn > 0
    u0 = (0.03, -0.02)
    f = o.get_mesh()
    for j in range(ns):
        # grad u = dudn * n (x) t (the t-component grows along n)
        G = dudn[j] * np.outer(n[j], t[j])
        Qg = np.array([(CX[i] * CX[i] - CS2) * G[0, 0] + CX[i] * CY[i] * (G[0, 1] + G[1, 0])
                       + (CY[i] * CY[i] - CS2) * G[1, 1] for i in range(9)])
        fneq = -tau_u * WQ * rho[j] * Qg / CS2
        f[:, j] = O.equilibrium(rho[j], *u0) + fneq
    o.set_mesh(f)
    cp, cf, cn = o.wall_coefficients()
    q = 0.5 * w.rho0 * w.u_inf**2
    mu = rho * CS2 * tau_u
    assert np.abs(cp - (rho - w.rho0) * CS2 / q).max() < 1e-12 * np.abs(cp).max()
    smooth = (om.surface_xi > 0.05) & (om.surface_xi < 0.95)
    exact = mu * dudn / q
    print("C_f rel err", np.abs(cf[smooth] / exact[smooth] - 1).max())
    assert np.abs(cf[smooth] / exact[smooth] - 1).max() < 1e-4
    assert np.abs(cn[smooth]).max() < 1e-2 * exact[smooth].min()
    # the leading-edge node lies on the symmetry line: its normal is exact
    le = ns // 2
    assert abs(cf[le] / exact[le] - 1) < 1e-12


def test_wall_means_reproduce_the_mean_force():
    """Mean force from the wall-node momentum flux = mean of the C_D, C_L history."""
    a = math.radians(4.0)
    w = W.naca_re100_c40(4.0)
    o = O.Oracle.from_workload(w, aoa_rad=a)
    o.step(40)
    nw = o.wall_stats_begin()
    assert nw == w.omesh.ns
    o.step(60)
    steps, cp, cf, cn = o.wall_stats()
    assert steps == 60
    cd, cl = o.history()
    xy = w.mesh_xy[:nw]
    # V_P: half the sum of the length-normals pointing into the body of the two
    # wall edges at P; surface points run TE -> upper -> LE -> lower, with the
    # body on their left
    d = np.roll(xy, -1, 0) - np.roll(xy, 1, 0)
    V = 0.5 * np.stack([-d[:, 1], d[:, 0]], 1)
    assert V[5, 1] < 0 and V[nw - 5, 1] > 0
    a_P = np.linalg.norm(V, axis=1)
    n = -V / a_P[:, None]
    t = np.stack([n[:, 1], -n[:, 0]], 1)
    F = ((-cp + cn)[:, None] * n + cf[:, None] * t) * a_P[:, None]
    fx, fy = F.sum(0) / w.chord
    cd_w = fx * math.cos(a) + fy * math.sin(a)
    cl_w = -fx * math.sin(a) + fy * math.cos(a)
    print("mean C_D", cd[40:].mean(), cd_w, "mean C_L", cl[40:].mean(), cl_w)
    assert abs(cd_w - cd[40:].mean()) < 1e-11
    assert abs(cl_w - cl[40:].mean()) < 1e-11
    # the pressure part dominates, the shear part is not negligible at Re = 100
    Fp = (-cp[:, None] * n * a_P[:, None]).sum(0) / w.chord
    assert 0.05 < abs(cd_w - (Fp[0] * math.cos(a) + Fp[1] * math.sin(a))) < abs(cd_w)


def test_wall_means_mirror_symmetry():
    w = W.naca_re100_c40(0.0)
    ns = w.omesh.ns
    out = []
    for sgn in (1, -1):
        o = O.Oracle.from_workload(w, aoa_rad=sgn * math.radians(5.0))
        o.wall_stats_begin()
        o.step(80)
        out.append(o.wall_stats())
    (_, cp1, cf1, cn1), (_, cp2, cf2, cn2) = out
    mirror = (ns - np.arange(ns)) % ns
    assert np.abs(cp1 - cp2[mirror]).max() < 1e-12 * np.abs(cp1).max()
    assert np.abs(cf1 + cf2[mirror]).max() < 1e-12 * np.abs(cf1).max()
    assert np.abs(cn1 - cn2[mirror]).max() < 1e-12 * np.abs(cn1).max()
    assert np.abs(cp1 - cp1[mirror]).max() > 1e-3     # not symmetric by itself at 5 degrees


def test_wall_stats_window_is_the_step_mean():
    """The running mean equals the mean of the per-step coefficients."""
    w = W.naca_re100_c40(2.0)
    o = O.Oracle.from_workload(w)
    o.wall_stats_begin()
    per = []
    for _ in range(6):
        o.step(1)
        per.append(o.wall_coefficients())
    steps, cp, cf, cn = o.wall_stats()
    assert steps == 6
    assert np.allclose(cp, np.mean([p[0] for p in per], 0), rtol=0, atol=1e-14)
    assert np.allclose(cf, np.mean([p[1] for p in per], 0), rtol=0, atol=1e-14)


def test_surface_distributions_and_separation_point():
    w = W.naca_re100_c40(0.0)
    om, ns = w.omesh, w.omesh.ns
    cp = np.arange(ns, dtype=float)
    cf = np.where(om.surface_upper, 1.0, -1.0)
    d = hlbm.surface_distributions(om, cp, cf)
    xu, cpu, cfu = d["upper"]
    xl, cpl, cfl = d["lower"]
    assert xu[0] == 0.0 and xu[-1] == 1.0 and np.all(np.diff(xu) > 0)
    assert xl[0] == 0.0 and xl[-1] == 1.0 and np.all(np.diff(xl) > 0)
    assert np.all(cfu == 1.0) and np.all(cfl[1:-1] == 1.0)
    assert cpu[0] == ns // 2 and cpl[-1] == 0
    # separation: first + to - crossing, linear interpolation
    x = np.linspace(0, 1, 11)
    assert hlbm.separation_point(x, 0.41 - x) == pytest.approx(0.41, abs=1e-12)
    assert hlbm.separation_point(x, np.cos(2 * np.pi * x)) == pytest.approx(0.25, abs=0.02)
    assert hlbm.separation_point(x, -x) is None                # never positive
    assert hlbm.separation_point(x, 1 + x) is None             # attached everywhere
    # reattached bubble: the first separation is reported
    cfb = np.array([1, 0.5, -0.2, -0.1, 0.3, 0.2, -0.4, -0.5, -0.1, 0.1, 0.2])
    assert hlbm.separation_point(x, cfb) == pytest.approx(0.1 + 0.1 * 0.5 / 0.7, abs=1e-12)
