"""Closed-form flow fields and small helpers shared by the tests.

Only elementary moments of the populations are computed here (density and
momentum as plain sums); no scheme arithmetic.
"""
import math

import numpy as np

CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])


def macro(f):
    """(rho, ux, uy) of populations with the lattice index first."""
    rho = f.sum(0)
    safe = np.where(rho != 0, rho, 1.0)
    ux = np.tensordot(CX, f, axes=(0, 0)) / safe
    uy = np.tensordot(CY, f, axes=(0, 0)) / safe
    return rho, ux, uy


def taylor_green(x, y, length, u0, nu, t, rho0=1.0):
    """Decaying Taylor-Green vortex of wavelength `length` (closed form)."""
    k = 2.0 * math.pi / length
    d = math.exp(-2.0 * nu * k * k * t)
    ux = -u0 * np.cos(k * x) * np.sin(k * y) * d
    uy = u0 * np.sin(k * x) * np.cos(k * y) * d
    p = -0.25 * rho0 * u0 * u0 * (np.cos(2 * k * x) + np.cos(2 * k * y)) * d * d
    rho = rho0 + 3.0 * p
    return rho, ux, uy


def feq_field(eq, rho, ux, uy):
    """Population array [9, *shape] from a pointwise equilibrium function."""
    shape = np.shape(rho)
    out = np.zeros((9,) + shape)
    it = np.nditer(np.asarray(rho), flags=["multi_index"])
    for _ in it:
        idx = it.multi_index
        out[(slice(None),) + idx] = eq(float(rho[idx]), float(ux[idx]), float(uy[idx]))
    return out


def amplitude(ux, uy, sx, sy):
    """Least-squares amplitude of (ux, uy) along the mode shape (sx, sy)."""
    return float((ux * sx + uy * sy).sum() / (sx * sx + sy * sy).sum())
