"""Seeded, synthetic inputs for the hybrid lattice Boltzmann (HLBM) solver.

This module builds the *inputs* of the method: the NACA 0012 profile, the
body-fitted triangular O-mesh around it, the structured grid with its nested
refinement boxes, and small test geometries (periodic triangulated squares,
rectangular mesh patches).  It holds none of the method's arithmetic: no
equilibrium, no collision, no finite-volume coefficients, no interpolation
weights.  Both the HIP library and the CPU oracle consume what it returns.

Geometry, in the paper's terms:
  * NACA 0012, symmetric, 12 % thickness (Sec. 4, problem setup).
  * Body-fitted unstructured triangular mesh confined around the body whose
    outer boundary is an ellipse; a second, inner fictitious ellipse closes the
    overlap band in which the interpolation nodes sit (Sec. 4).
  * Uniform Cartesian grid with nested factor-two refinement boxes; the
    innermost box has unit spacing and overlaps the mesh (Sec. 4).
Coordinates are in lattice units of the finest structured level.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

KIND_INTERIOR = 0
KIND_WALL = 1
KIND_INTERP = 2


# ---------------------------------------------------------------------------
# NACA 0012 profile and O-mesh
# ---------------------------------------------------------------------------

def naca0012_half_thickness(xi: np.ndarray) -> np.ndarray:
    """Half thickness over chord of the NACA 0012 section (closed trailing edge)."""
    xi = np.clip(xi, 0.0, 1.0)
    return 0.6 * (0.2969 * np.sqrt(xi) - 0.1260 * xi - 0.3516 * xi**2
                  + 0.2843 * xi**3 - 0.1036 * xi**4)


def hicks_henne(xi: np.ndarray, peaks, amps, exponent: float = 3.0) -> np.ndarray:
    """Sum of Hicks-Henne bumps a_m sin^e(pi xi^(ln 0.5 / ln x_m)) (chord units)."""
    xi = np.clip(np.asarray(xi, dtype=np.float64), 0.0, 1.0)
    out = np.zeros_like(xi)
    for xm, am in zip(peaks, amps):
        p = math.log(0.5) / math.log(xm)
        out += am * np.sin(np.pi * xi**p) ** exponent
    return out


def _growth_for_first_height(h1: float, dist: float, nl: int) -> float:
    """Geometric growth r with (r-1)/(r^nl-1)*dist == h1 (bisection)."""
    if h1 * nl >= dist:
        raise ValueError("first height too large for uniform-or-growing layers")
    lo, hi = 1.0 + 1e-12, 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        h = (mid - 1.0) / (mid**nl - 1.0) * dist
        if h > h1:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


@dataclasses.dataclass
class OMesh:
    xy: np.ndarray          # [n_nodes, 2] float64
    tri: np.ndarray         # [n_tris, 3] int32, counter-clockwise
    kind: np.ndarray        # [n_nodes] uint8: 0 interior, 1 wall, 2 interpolation
    ns: int
    nl: int
    growth: float
    centre: Tuple[float, float]
    outer_axes: Tuple[float, float]
    outer_layer_thickness: float
    surface_index: np.ndarray   # [ns] node index of the wall node j
    chord: float = 0.0
    surface_xi: Optional[np.ndarray] = None   # [ns] x/c of surface point j
    surface_upper: Optional[np.ndarray] = None  # [ns] bool: point j carries the bumps
    eta: Optional[np.ndarray] = None          # [nl + 1] layer fractions, 0 at the wall, 1 outside

    def bump_tangent(self, peaks) -> np.ndarray:
        """d(node coordinates)/d(bump amplitudes), shape [len(peaks), n_nodes, 2].

        The bumps displace the upper-surface points in y by c * sum_m a_m b_m(x/c)
        (leading and trailing edge points excluded) and layer l carries the
        displacement of its surface point scaled by 1 - eta_l, so the mesh is
        linear in the amplitudes and this is exact."""
        ns, nl = self.ns, self.nl
        out = np.zeros((len(peaks), (nl + 1) * ns, 2))
        for m, xm in enumerate(peaks):
            amps = np.zeros(len(peaks))
            amps[m] = 1.0
            dy = self.chord * np.where(self.surface_upper, hicks_henne(self.surface_xi, peaks, amps), 0.0)
            dy[0] = 0.0
            dy[ns // 2] = 0.0
            out[m, :, 1] = ((1.0 - self.eta)[:, None] * dy[None, :]).ravel()
        return out

    @property
    def n_nodes(self) -> int:
        return int(self.xy.shape[0])

    @property
    def n_tris(self) -> int:
        return int(self.tri.shape[0])


def _surface_parameter(ns: int, spacing: str, bump=None) -> np.ndarray:
    """Curve parameter theta_j of the ns surface points (j = 0 at the trailing edge).

    The profile is x = x_LE + c (1 + cos theta) / 2, upper surface for theta <= pi.
    "cosine": theta_j = 2 pi j / ns.  "arclength": theta_j chosen so that the
    surface points are equally spaced along the profile, which bounds the
    smallest wall element (cosine spacing shrinks the trailing-edge element to
    ~c pi^2/ns^2 and with it the stable explicit finite-volume time step).
    """
    if spacing == "cosine":
        return 2.0 * np.pi * np.arange(ns) / ns
    if spacing != "arclength":
        raise ValueError(spacing)
    m = 200001
    tt = np.linspace(0.0, np.pi, m)
    xi = 0.5 * (1.0 + np.cos(tt))
    yy = naca0012_half_thickness(xi)
    if bump is not None:
        yy = yy + bump(xi)
    seg = np.hypot(np.diff(xi), np.diff(yy))
    s = np.concatenate([[0.0], np.cumsum(seg)])
    half = ns // 2
    target = s[-1] * np.arange(half + 1) / half
    th_up = np.interp(target, s, tt)
    th_up[0], th_up[-1] = 0.0, np.pi
    th = np.empty(ns)
    th[:half + 1] = th_up
    th[half + 1:] = 2.0 * np.pi - th_up[1:half][::-1]
    return th


def _ellipse_parameter(ns: int, a: float, b: float) -> np.ndarray:
    """Angles of ns points equally spaced in arc length on the ellipse
    (a cos t, b sin t), point 0 at t = 0, point ns/2 at t = pi, mirror symmetric."""
    m = 200001
    tt = np.linspace(0.0, np.pi, m)
    seg = np.hypot(np.diff(a * np.cos(tt)), np.diff(b * np.sin(tt)))
    s = np.concatenate([[0.0], np.cumsum(seg)])
    half = ns // 2
    t_up = np.interp(s[-1] * np.arange(half + 1) / half, s, tt)
    t_up[0], t_up[-1] = 0.0, np.pi
    t = np.empty(ns)
    t[:half + 1] = t_up
    t[half + 1:] = 2.0 * np.pi - t_up[1:half][::-1]
    return t


def naca0012_omesh(chord: float, le: Tuple[float, float], ns: int, nl: int,
                   d_out: float, growth: Optional[float] = None,
                   h1: Optional[float] = None,
                   bump_amps=None, bump_peaks=None, spacing: str = "arclength",
                   split: str = "halves", outer: str = "theta") -> OMesh:
    """O-mesh of ns surface points times nl layers around the NACA 0012.

    Surface point j (j = 0 at the trailing edge, counter-clockwise) sits at
    curve parameter theta_j, x = x_LE + c (1 + cos theta) / 2, upper surface
    for theta <= pi (see _surface_parameter for the spacing).  The outer
    boundary is the ellipse centred at mid-chord with semi-axes
    (c/2 + d_out, d_out); layer l interpolates between the surface point and
    the ellipse point of the same theta with geometric spacing.  Quads are
    split so that the mesh is mirror symmetric about the chord line: split =
    "halves" uses one diagonal on the upper half and the mirrored one on the
    lower half; "checker" alternates the diagonal from quad to quad.  outer =
    "theta" joins surface point j to the ellipse point of the same theta;
    "arclength" to the j-th of ns points equally spaced along the ellipse.
    """
    if ns % 2:
        raise ValueError("ns must be even")
    x_le, y_le = le
    th = _surface_parameter(ns, spacing)
    xi = 0.5 * (1.0 + np.cos(th))
    yt = naca0012_half_thickness(xi)
    upper = th <= np.pi + 1e-12
    ys = np.where(upper, yt, -yt)
    if bump_amps is not None:
        bump = hicks_henne(xi, bump_peaks, bump_amps)
        ys = ys + np.where(upper, bump, 0.0)
    sx = x_le + chord * xi
    sy = y_le + chord * ys
    # exact zero thickness at the leading and trailing edge points
    sy[0] = y_le
    sy[ns // 2] = y_le
    xc, yc = x_le + 0.5 * chord, y_le
    a_out, b_out = 0.5 * chord + d_out, d_out
    th_out = th if outer == "theta" else _ellipse_parameter(ns, a_out, b_out)
    ox = xc + a_out * np.cos(th_out)
    oy = yc + b_out * np.sin(th_out)
    if growth is None:
        if h1 is None:
            raise ValueError("need growth or h1")
        growth = _growth_for_first_height(h1, d_out, nl)
    r = growth
    if abs(r - 1.0) < 1e-14:
        eta = np.arange(nl + 1) / nl
    else:
        eta = (r ** np.arange(nl + 1) - 1.0) / (r**nl - 1.0)
    # node (j, l) -> l * ns + j
    X = sx[None, :] + eta[:, None] * (ox - sx)[None, :]
    Y = sy[None, :] + eta[:, None] * (oy - sy)[None, :]
    if bump_amps is None:
        # exact mirror images about the chord line: node ns - j mirrors node j
        half = ns // 2
        X[:, half + 1:] = X[:, 1:half][:, ::-1]
        Y[:, half + 1:] = 2.0 * y_le - Y[:, 1:half][:, ::-1]
        Y[:, 0] = y_le
        Y[:, half] = y_le
    xy = np.stack([X.ravel(), Y.ravel()], axis=1)
    kind = np.zeros((nl + 1) * ns, dtype=np.uint8)
    kind[:ns] = KIND_WALL
    kind[nl * ns:] = KIND_INTERP
    tris = []
    for l in range(nl):
        for j in range(ns):
            jp = (j + 1) % ns
            a, b = l * ns + j, l * ns + jp
            c, d = (l + 1) * ns + jp, (l + 1) * ns + j
            use_ac = (j < ns // 2) if split == "halves" else ((j + l) % 2 == 0)
            if use_ac:          # diagonal (j,l)-(j+1,l+1) = a-c
                t1, t2 = (a, c, b), (a, d, c)
            else:               # diagonal (j+1,l)-(j,l+1) = b-d
                t1, t2 = (a, d, b), (b, d, c)
            tris.append(t1)
            tris.append(t2)
    tri = np.asarray(tris, dtype=np.int32)
    tri = _orient_ccw(xy, tri)
    t_outer = float(np.max(np.hypot(X[nl] - X[nl - 1], Y[nl] - Y[nl - 1])))
    return OMesh(xy=xy, tri=tri, kind=kind, ns=ns, nl=nl, growth=float(r),
                 centre=(xc, yc), outer_axes=(a_out, b_out),
                 outer_layer_thickness=t_outer,
                 surface_index=np.arange(ns, dtype=np.int64), chord=float(chord),
                 surface_xi=xi, surface_upper=upper, eta=eta)


def _orient_ccw(xy: np.ndarray, tri: np.ndarray) -> np.ndarray:
    p, q, r = xy[tri[:, 0]], xy[tri[:, 1]], xy[tri[:, 2]]
    cross = (q[:, 0] - p[:, 0]) * (r[:, 1] - p[:, 1]) - (q[:, 1] - p[:, 1]) * (r[:, 0] - p[:, 0])
    out = tri.copy()
    flip = cross < 0
    out[flip, 1], out[flip, 2] = tri[flip, 2], tri[flip, 1]
    return out


# ---------------------------------------------------------------------------
# Test geometries
# ---------------------------------------------------------------------------

def periodic_square_mesh(n: int, length: float, diagonal: str = "alternate"):
    """Regular triangulation of a periodic square of side `length`, n x n nodes.

    Node (i, j) -> j * n + i at ((i + 0.5) h, (j + 0.5) h).  Each grid square is
    split into two triangles; connectivity wraps around both directions.
    Returns (xy, tri, kind) with every node interior.
    """
    h = length / n
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    xy = np.stack([(ii.ravel() + 0.5) * h, (jj.ravel() + 0.5) * h], axis=1)
    tris = []
    for j in range(n):
        for i in range(n):
            a = j * n + i
            b = j * n + (i + 1) % n
            c = ((j + 1) % n) * n + (i + 1) % n
            d = ((j + 1) % n) * n + i
            alt = (diagonal == "alternate" and (i + j) % 2 == 1)
            if alt:
                tris += [(a, b, d), (b, c, d)]
            else:
                tris += [(a, b, c), (a, c, d)]
    tri = np.asarray(tris, dtype=np.int32)
    kind = np.zeros(n * n, dtype=np.uint8)
    return xy, tri, kind


def periodic_channel_mesh(nx: int, ny: int, length: float, height: float,
                          diagonal: str = "alternate"):
    """Triangulated strip [0, length) x [0, height], periodic in x, with wall rows.

    nx nodes per row (x = (i + 0.5) length / nx, wrapping around in x) and
    ny + 1 rows (y = j height / ny).  The rows j = 0 and j = ny are wall nodes;
    every other node is interior.  Each cell is split into two triangles along
    alternating diagonals ("alternate") or always along the same one ("same").
    Returns (xy, tri, kind).
    """
    hx, hy = length / nx, height / ny
    ii, jj = np.meshgrid(np.arange(nx), np.arange(ny + 1), indexing="xy")
    xy = np.stack([(ii.ravel() + 0.5) * hx, jj.ravel() * hy], axis=1)
    tris = []
    for j in range(ny):
        for i in range(nx):
            a = j * nx + i
            b = j * nx + (i + 1) % nx
            c = (j + 1) * nx + (i + 1) % nx
            d = (j + 1) * nx + i
            if diagonal == "alternate" and (i + j) % 2 == 1:
                tris += [(a, b, d), (b, c, d)]
            else:
                tris += [(a, b, c), (a, c, d)]
    tri = np.asarray(tris, dtype=np.int32)
    kind = np.zeros((ny + 1, nx), dtype=np.uint8)
    kind[0, :] = kind[-1, :] = KIND_WALL
    return xy, tri, kind.ravel()


def rect_patch_mesh(x0: float, y0: float, nx: int, ny: int, h: float,
                    jitter: float = 0.0, seed: int = 0):
    """Triangulated rectangle [x0, x0+nx h] x [y0, y0+ny h] of (nx+1)(ny+1) nodes.

    Interior nodes are displaced by a seeded uniform jitter of at most
    `jitter * h` per coordinate; boundary nodes are the interpolation ring.
    Returns (xy, tri, kind) (no wall nodes).
    """
    rng = np.random.default_rng(seed)
    ii, jj = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), indexing="xy")
    x = x0 + ii.astype(np.float64) * h
    y = y0 + jj.astype(np.float64) * h
    kind = np.zeros((ny + 1, nx + 1), dtype=np.uint8)
    kind[0, :] = kind[-1, :] = KIND_INTERP
    kind[:, 0] = kind[:, -1] = KIND_INTERP
    inner = kind == KIND_INTERIOR
    if jitter > 0:
        x = x + np.where(inner, rng.uniform(-jitter, jitter, x.shape) * h, 0.0)
        y = y + np.where(inner, rng.uniform(-jitter, jitter, y.shape) * h, 0.0)
    xy = np.stack([x.ravel(), y.ravel()], axis=1)
    tris = []
    for j in range(ny):
        for i in range(nx):
            a = j * (nx + 1) + i
            b = a + 1
            d = a + (nx + 1)
            c = d + 1
            if (i + j) % 2 == 0:
                tris += [(a, b, c), (a, c, d)]
            else:
                tris += [(a, b, d), (b, c, d)]
    tri = _orient_ccw(xy, np.asarray(tris, dtype=np.int32))
    return xy, tri, kind.ravel()


# ---------------------------------------------------------------------------
# Workload presets
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    """One HLBM problem: structured grid, refinement boxes, mesh and flow."""
    name: str
    nx_cells: int            # base-level cells along x
    ny_cells: int            # base-level cells along y
    patches: List[Tuple[int, int, int, int]]  # (i0, j0, nx, ny): origin in parent nodes, size in own cells
    u_inf: float
    aoa_deg: float
    re: float
    chord: float
    mesh_xy: Optional[np.ndarray]
    mesh_tri: Optional[np.ndarray]
    mesh_kind: Optional[np.ndarray]
    inner_ellipse: Tuple[float, float, float, float]   # (xc, yc, a, b), finest lu
    steps: int
    rho0: float = 1.0
    periodic: bool = False
    n_sub: int = 0
    omesh: Optional[OMesh] = None
    notes: str = ""
    f2c_filter: bool = False   # fine -> coarse f^neq full-weighted over 3 x 3 fine nodes
    # solid body on the finest level resolved by bounce-back (a standard LBM, no mesh):
    # polygon vertices (x, y) in finest lu, counter-clockwise
    body_xy: Optional[np.ndarray] = None

    @property
    def n_refine(self) -> int:
        return len(self.patches)

    @property
    def base_spacing(self) -> int:
        return 2 ** self.n_refine

    @property
    def tau_s(self) -> float:
        """Finest-level relaxation time from Re on chord and free-stream speed."""
        nu = self.u_inf * self.chord / self.re
        return 0.5 + 3.0 * nu

    @property
    def aoa_rad(self) -> float:
        return math.radians(self.aoa_deg)

    def level_nodes(self) -> List[Tuple[int, int]]:
        """(nx_nodes, ny_nodes) for every level, coarse to fine."""
        out = [(self.nx_cells + (0 if self.periodic else 1),
                self.ny_cells + (0 if self.periodic else 1))]
        for (_, _, px, py) in self.patches:
            out.append((px + 1, py + 1))
        return out

    def structured_node_count(self) -> int:
        return int(sum(a * b for a, b in self.level_nodes()))


def _place_patches(x_mid: float, y_mid: float, sizes, n_levels: int, base_spacing: int):
    """Centre nested boxes on (x_mid, y_mid), origins aligned to parent nodes."""
    patches = []
    parent_origin = (0.0, 0.0)
    parent_sp = base_spacing
    for (pnx, pny) in sizes:
        own_sp = parent_sp // 2
        wx, wy = pnx * own_sp, pny * own_sp
        i0 = int(math.floor((x_mid - 0.5 * wx - parent_origin[0]) / parent_sp + 0.5))
        j0 = int(math.floor((y_mid - 0.5 * wy - parent_origin[1]) / parent_sp + 0.5))
        patches.append((i0, j0, pnx, pny))
        parent_origin = (parent_origin[0] + i0 * parent_sp, parent_origin[1] + j0 * parent_sp)
        parent_sp = own_sp
    return patches


def _inner_ellipse(om: OMesh) -> Tuple[float, float, float, float]:
    """Inner fictitious ellipse: outer ellipse shrunk by w = max(4, 2 t_outer + 2)."""
    w = max(4.0, 2.0 * om.outer_layer_thickness + 2.0)
    a, b = om.outer_axes
    return (om.centre[0], om.centre[1], a - w, b - w)


def _naca_workload(name, nx, ny, patch_sizes, chord, re, u, aoa, ns, nl, d_out,
                   growth=None, h1=None, steps=1000, bumps=None, notes="", split="halves", outer="theta",
                   spacing="arclength"):
    n_ref = len(patch_sizes)
    sp = 2 ** n_ref
    W, H = nx * sp, ny * sp
    le = (float(round(W / 3.0)), 0.5 * H)
    peaks = [0.1 * (m + 1) for m in range(8)]
    om = naca0012_omesh(chord, le, ns, nl, d_out, growth=growth, h1=h1,
                        bump_amps=bumps, bump_peaks=peaks if bumps is not None else None, split=split,
                        outer=outer, spacing=spacing)
    patches = _place_patches(le[0] + 0.5 * chord, le[1], patch_sizes, n_ref, sp)
    return Workload(name=name, nx_cells=nx, ny_cells=ny, patches=patches, u_inf=u,
                    aoa_deg=aoa, re=re, chord=chord, mesh_xy=om.xy, mesh_tri=om.tri,
                    mesh_kind=om.kind, inner_ellipse=_inner_ellipse(om), steps=steps,
                    omesh=om, notes=notes)


HH_PEAKS = [0.1 * (m + 1) for m in range(8)]


def hh_amplitudes(seed: int = 0) -> np.ndarray:
    """Seeded Hicks-Henne amplitudes, uniform in [-0.002, 0.002] (chord units)."""
    return np.random.default_rng(seed).uniform(-0.002, 0.002, 8)


def naca_re100_c40(aoa_deg: float = 0.0, bumps=None, spacing: str = "arclength") -> Workload:
    """Small FP64 case: 240x120 grid, c = 40, Re = 100, 128x16 O-mesh
    (optionally with Hicks-Henne bumps of the given amplitudes at HH_PEAKS).
    spacing="cosine" places the surface points as the configuration text
    states (the smallest wall element then shrinks to ~c pi^2 / ns^2 at the
    trailing edge; the default is equal arc length)."""
    name = "naca0012_re100_c40_240x120" + ("_bumps" if bumps is not None else "") + \
        ("_cosine" if spacing == "cosine" else "")
    return _naca_workload(name, 240, 120, [], 40.0, 100.0, 0.05, aoa_deg, 128, 16, 52.0, growth=1.15,
                          steps=2000, bumps=None if bumps is None else np.asarray(bumps, dtype=np.float64),
                          spacing=spacing)


def naca_re100_c40_refined(aoa_deg: float = 0.0, bumps=None) -> Workload:
    """Small refined case: the c = 40 airfoil on a 120x60 base grid (spacing 2)
    with one 128x64 box (unit spacing) around a 128x16 O-mesh reaching 20 lu
    out from the profile."""
    return _naca_workload("naca0012_re100_c40_120x60_r1" + ("_bumps" if bumps is not None else ""), 120, 60,
                          [(128, 64)], 40.0, 100.0, 0.05, aoa_deg, 128, 16, 20.0, growth=1.15, steps=2000,
                          bumps=None if bumps is None else np.asarray(bumps, dtype=np.float64))


# Thickness of the O-mesh band.  The finite-volume streaming of eq. (3) is a
# central scheme; where the shed wake crosses the mesh it diverges at these
# relaxation times (Re = 1000, c = 128, tau_u = 0.0192: a band reaching 92 lu
# = 0.72 c out diverged after 7,000-31,000 steps for 512-2048 surface points;
# measured), while a thin band that hands the wake to the Cartesian grid runs
# 40,000 steps (24 lu = 0.19 c; 512 and 1024 surface points agree on C_D
# within 0.5%).  The paper's own Re = 1000 meshes are thin bands too (~2.2e4
# nodes, ~0.8 lu at the wall).
RE1000_C128_DOUT, RE1000_C128_H1 = 24.0, 0.25


def naca_re1000_c128(aoa_deg: float = 0.0, ns: int = 512, band: float = RE1000_C128_DOUT,
                     nl: int = 64) -> Workload:
    """Re = 1000, c = 128: 1024x512 base cells (spacing 2), one 384x192 box, ns x nl mesh
    in a band `band` lu thick (default 24, 64 layers; first layer 0.25 lu)."""
    tag = ("" if ns == 512 else f"_m{ns}") + ("" if (band, nl) == (RE1000_C128_DOUT, 64) else f"_b{band:g}x{nl}")
    return _naca_workload("naca0012_re1000_c128_1024x512_r1" + tag, 1024, 512,
                          [(384, 192)], 128.0, 1000.0, 0.05, aoa_deg, ns, nl, band,
                          h1=RE1000_C128_H1, steps=40000)


def naca_re1e4_c256(f2c_filter: bool = False) -> Workload:
    """Re = 1e4, c = 256: 2048x1024 base cells (spacing 4), two nested boxes, 1024x128 mesh.
    Its coarse levels run at tau = 0.5008 and 0.5015; with the pointwise fine -> coarse
    transfer the run blows up at the upstream edge of the finest box after ~1,500 steps,
    with the filtered one (f2c_filter) it runs on."""
    w = _naca_workload("naca0012_re1e4_c256_2048x1024_r2" + ("_f2c3x3" if f2c_filter else ""), 2048, 1024,
                       [(768, 384), (768, 384)], 256.0, 1.0e4, 0.04, 0.0, 1024, 128,
                       188.0, h1=0.512, steps=100000)
    return dataclasses.replace(w, f2c_filter=bool(f2c_filter))


def naca_re1000_c128_bumps(bumps=None) -> Workload:
    """Shape-gradient case: the Re = 1000, c = 128 geometry at 5 deg with Hicks-Henne bumps
    (default: the seeded amplitudes hh_amplitudes(0))."""
    amps = hh_amplitudes(0) if bumps is None else np.asarray(bumps, dtype=np.float64)
    return _naca_workload("naca0012_re1000_c128_aoa5_bumps", 1024, 512, [(384, 192)], 128.0,
                          1000.0, 0.05, 5.0, 512, 64, RE1000_C128_DOUT, h1=RE1000_C128_H1, steps=25000,
                          bumps=amps)


def naca_re5000_c512(aoa_deg: float = 8.0, band: float = 51.2, nl: int = 128) -> Workload:
    """Throughput case: 8192x4096 base cells (spacing 2), 2048x1024 box, 2048x128 mesh in
    a band 0.1c = 51.2 lu thick with a 0.25 lu first layer (outer cells ~0.6 lu), at 8 deg
    unless aoa_deg says otherwise.  A band reaching 508 lu out (outer cells 13 lu across)
    carried a spurious lift oscillation with a period of ~100 steps."""
    name = "naca0012_re5000_c512_8192x4096_r1" + ("" if aoa_deg == 8.0 else f"_aoa{aoa_deg:g}") + \
        ("" if (band, nl) == (51.2, 128) else f"_band{band:g}_nl{nl}")
    return _naca_workload(name, 8192, 4096, [(2048, 1024)],
                          512.0, 5000.0, 0.05, aoa_deg, 2048, nl, band, h1=0.25, steps=10000)


CONV_CHORDS = (48, 64, 96, 128, 144)
CONV_N_SUB = 70     # ceil(1 / tau_u) of the smallest chord: one FV time step for every chord

# Levels of the Re 500 and Re-sweep families.  With acoustic scaling level l
# has tau_l - 1/2 = (tau_s - 1/2) / 2^(L-l), so its cell Reynolds number is
# U dx_l / nu_l = 2^(L-l) Re / c (in chords).  At 83 (Re 500, c = 48, four
# levels, coarse tau 0.5018 and 0.5036) the upstream coarse-to-fine interface
# diverged after 4,000-8,000 steps (measured).  The growth needs both
# non-equilibrium rescalings of the refinement interface and sets in for a
# coarse tau below about 0.506 (seeded-noise runs of the oracle, far field
# only); two levels keep every coarse tau above that, with cell Reynolds
# numbers at or below 21 in the convergence family and 4-39 in the sweep.
FAMILY_BOXES = 1


def naca_re500_four_levels(chord: int = 48, f2c_filter: bool = False) -> Workload:
    """Four structured levels (base spacing 8 over 30c x 15c, three nested boxes
    of 2.5c x 1.25c cells each) around a 4c x c/2 O-mesh, Re = 500: the paper's
    level layout.  Its coarse levels run close to tau = 1/2 (0.5018 and 0.5036
    at c = 48): long runs need the filtered fine -> coarse transfer
    (f2c_filter); with the pointwise one it serves short parity runs."""
    c = int(chord)
    if c % 8:
        raise ValueError("chord must be a multiple of 8")
    box = (5 * c // 2, 5 * c // 4)
    w = _naca_workload(f"naca0012_re500_c{c}_four_levels" + ("_f2c3x3" if f2c_filter else ""), 15 * c // 4,
                       15 * c // 8, [box, box, box], float(c), 500.0, 0.05, 0.0, 4 * c, c // 2, c / 4.0, h1=0.25,
                       steps=1000)
    return dataclasses.replace(w, n_sub=CONV_N_SUB, f2c_filter=bool(f2c_filter))


def naca_re500_conv(chord: int = 48) -> Workload:
    """Self-convergence family (Sec. 5): Re = 500, alpha = 0, a base grid of
    spacing 2 spanning 30c x 15c and one box of unit spacing (2.5c x 1.25c)
    centred on mid-chord, so every chord gives the same geometry in chord
    units.  The O-mesh has the same wall element size for every chord (4c
    surface points, ~0.5 lu apart; first layer 0.25 lu; a band c/4 thick in c/2
    layers), and the finite-volume time step is the same for all (n = 70)."""
    c = int(chord)
    if c % 16:
        raise ValueError("chord must be a multiple of 16")
    sp = 2 ** FAMILY_BOXES
    w = _naca_workload(f"naca0012_re500_c{c}_conv", 30 * c // sp, 15 * c // sp, [(5 * c // 2, 5 * c // 4)],
                       float(c), 500.0, 0.05, 0.0, 4 * c, c // 2, c / 4.0, h1=0.25, steps=600 * c)
    return dataclasses.replace(w, n_sub=CONV_N_SUB)


def naca_re_sweep(re: float = 2000.0, ns: int = 1280, d_out: float = 0.19, nl: int = 64,
                  h1: float = 0.8, f2c_filter: bool = False) -> Workload:
    """Reynolds sweep at zero incidence (Sec. 6.2): c = 512, U = 0.05, a base grid
    of spacing 2 spanning 16c x 8c with one box of unit spacing (2c x c) and a thin
    O-mesh band (outer ellipse d_out c beyond the chord line and the edges; by
    default 1280 surface points ~0.8 lu apart, first layer 0.8 lu, 64 layers).
    The base level runs at tau = 0.5 + 38.4 / Re (0.5038 at Re 1e4)."""
    c = 512
    default = (ns, d_out, nl, h1) == (1280, 0.19, 64, 0.8)
    tag = ("" if default else f"_m{ns}_d{d_out:g}_l{nl}_h{h1:g}") + ("_f2c3x3" if f2c_filter else "")
    w = _naca_workload(f"naca0012_re{int(re)}_c512_sweep{tag}", 8 * c, 4 * c, [(2 * c, c)], float(c),
                       float(re), 0.05, 0.0, ns, nl, d_out * c, h1=h1, steps=200 * c)
    return dataclasses.replace(w, f2c_filter=bool(f2c_filter))


def equivalent_lbm(w: Workload, margin: int = 8, body: bool = True) -> Workload:
    """The standard LBM against which eq. (14) prices the hybrid scheme: w's
    structured grid with one more box of half the finest spacing over w's finest
    box (inset by `margin` cells of that box on every side) and no mesh, the
    profile resolved on that box by bounce-back (its wall points as a polygon;
    body=False leaves it out).  Its finest spacing is half a lattice unit of w,
    the wall spacing of the workloads' meshes.  Lengths are in the new finest
    units, so coordinates and the chord double and Re, U (hence tau) hold."""
    if w.patches:
        px, py = w.patches[-1][2], w.patches[-1][3]
    else:
        px, py = w.nx_cells, w.ny_cells
    box = (margin, margin, 2 * (px - 2 * margin), 2 * (py - 2 * margin))
    poly = None
    if body and w.omesh is not None:
        poly = 2.0 * w.omesh.xy[w.omesh.surface_index]
    return dataclasses.replace(
        w, name=w.name + ("_equivalent_lbm" if body else "_equivalent_lbm_nobody"), patches=list(w.patches) + [box],
        chord=2.0 * w.chord, mesh_xy=None, mesh_tri=None, mesh_kind=None, inner_ellipse=(0.0, 0.0, 0.0, 0.0),
        omesh=None, n_sub=0, body_xy=poly)


PRESETS = {
    "naca_re100_c40": naca_re100_c40,
    "naca_re100_c40_refined": naca_re100_c40_refined,
    "naca_re1000_c128": naca_re1000_c128,
    "naca_re1e4_c256": naca_re1e4_c256,
    "naca_re1000_c128_bumps": naca_re1000_c128_bumps,
    "naca_re5000_c512": naca_re5000_c512,
    "naca_re500_conv": naca_re500_conv,
    "naca_re500_four_levels": naca_re500_four_levels,
    "naca_re_sweep": naca_re_sweep,
}
