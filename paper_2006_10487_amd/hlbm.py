"""Python binding of the HLBM C ABI (``include/hlbm.h``).

Argument marshalling only: every step of the method runs in the HIP library
``libhlbm.so``.  PyTorch provides the device workspace and the stream.  The
binding fails loudly when the library is missing; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhlbm.so")

HLBM_OK = 0
ERRORS = {-1: "HLBM_E_ARG", -2: "HLBM_E_GEOMETRY", -3: "HLBM_E_PARAM", -4: "HLBM_E_DEVICE",
          -5: "HLBM_E_NONFINITE", -6: "HLBM_E_STATE", -7: "HLBM_E_WORKSPACE"}
FP64, FP32_SHIFTED = 0, 1
INTERP_QUADRATIC, INTERP_LINEAR = 0, 1
BC_FARFIELD, BC_PERIODIC = 0, 1
PART_MESH = 100

EXPORTED = ["hlbm_validate", "hlbm_workspace_size", "hlbm_create", "hlbm_step", "hlbm_forces",
            "hlbm_force_history", "hlbm_get_state", "hlbm_set_state", "hlbm_info", "hlbm_last_error",
            "hlbm_destroy", "hlbm_profile", "hlbm_profile_read", "hlbm_kernel_bench",
            "hlbm_objective_workspace_size", "hlbm_run_objective", "hlbm_adjoint",
            "hlbm_wall_stats_begin", "hlbm_wall_stats", "hlbm_create_noalloc"]
KERNEL_CLASSES = ["collide_l0", "collide_l1", "collide_l2", "collide_l3", "coarse_to_fine",
                  "fine_to_coarse", "mesh_to_struct", "struct_to_mesh", "fv_substep", "wall_force",
                  "wall_stats"]


class HLBMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Grid(C.Structure):
    _fields_ = [
        ("nx_cells", C.c_int32), ("ny_cells", C.c_int32), ("n_refine", C.c_int32),
        ("patch_i0", C.c_int32 * 3), ("patch_j0", C.c_int32 * 3),
        ("patch_nx", C.c_int32 * 3), ("patch_ny", C.c_int32 * 3),
        ("u_inf", C.c_double), ("aoa_rad", C.c_double), ("rho0", C.c_double),
        ("precision", C.c_int32), ("interp", C.c_int32), ("n_sub", C.c_int32), ("bc", C.c_int32),
        ("wall_bc", C.c_int32), ("check_every", C.c_int32), ("history_len", C.c_int32),
        ("fv_fuse", C.c_int32), ("f2c_filter", C.c_int32),
    ]


class Mesh(C.Structure):
    _fields_ = [
        ("n_nodes", C.c_int32), ("n_tris", C.c_int32),
        ("xy", C.POINTER(C.c_double)), ("tri", C.POINTER(C.c_int32)), ("kind", C.POINTER(C.c_uint8)),
        ("chord", C.c_double), ("inner_ellipse", C.c_double * 4),
        ("n_shape", C.c_int32), ("dxy_dshape", C.POINTER(C.c_double)),
        ("body_n", C.c_int32), ("body_xy", C.POINTER(C.c_double)),
    ]


class Objective(C.Structure):
    _fields_ = [("t_end", C.c_int64), ("t0", C.c_int64), ("t1", C.c_int64), ("ckpt_every", C.c_int64),
                ("w_cd", C.c_double), ("w_cl", C.c_double), ("mesh_grad", C.c_int32),
                ("store_substeps", C.c_int32)]


class Info(C.Structure):
    _fields_ = [
        ("n_levels", C.c_int32), ("n_sub", C.c_int32),
        ("nx", C.c_int32 * 4), ("ny", C.c_int32 * 4), ("pitch", C.c_int32 * 4),
        ("tau", C.c_double * 4), ("tau_u", C.c_double), ("active_nodes", C.c_int64 * 4),
        ("n_mesh_nodes", C.c_int32), ("n_wall_nodes", C.c_int32), ("n_interp_mesh", C.c_int32),
        ("n_interp_struct", C.c_int32), ("n_fallback", C.c_int32), ("n_wall_edges", C.c_int32),
        ("nnz", C.c_int32), ("bytes_per_finest_step", C.c_int64), ("k1_bytes", C.c_int64 * 4),
        ("fv_bytes", C.c_int64), ("t", C.c_int64), ("workspace_bytes", C.c_size_t),
        ("fv_fuse", C.c_int32), ("fv_tiles", C.c_int32), ("fv_tile_nodes", C.c_int32),
        ("fv_threads", C.c_int32), ("fv_layout_bytes", C.c_int64),
        ("n_solid", C.c_int32), ("n_bounce", C.c_int32),
    ]


_lib = None


def lib():
    """Load libhlbm.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.hlbm_validate.argtypes = [C.POINTER(Grid), C.POINTER(Mesh), C.c_double, C.c_double]
        L.hlbm_workspace_size.argtypes = [C.POINTER(Grid), C.POINTER(Mesh), C.c_double, C.c_double,
                                          C.POINTER(C.c_size_t)]
        L.hlbm_create.argtypes = [C.POINTER(Grid), C.POINTER(Mesh), C.c_double, C.c_double, P,
                                  C.c_size_t, P, C.POINTER(P)]
        L.hlbm_create_noalloc.argtypes = [C.POINTER(Grid), C.POINTER(Mesh), C.c_double, C.c_double, P,
                                          C.POINTER(P)]
        L.hlbm_step.argtypes = [P, C.c_int64]
        L.hlbm_forces.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.hlbm_force_history.argtypes = [P, C.c_int64, C.c_int64, P, P]
        L.hlbm_get_state.argtypes = [P, C.c_int32, P, C.c_size_t]
        L.hlbm_set_state.argtypes = [P, C.c_int32, P, C.c_size_t]
        L.hlbm_info.argtypes = [P, C.POINTER(Info)]
        L.hlbm_last_error.argtypes = [P]
        L.hlbm_last_error.restype = C.c_char_p
        L.hlbm_destroy.argtypes = [P]
        L.hlbm_destroy.restype = None
        L.hlbm_profile.argtypes = [P, C.c_int]
        L.hlbm_profile_read.argtypes = [P, P, P]
        L.hlbm_kernel_bench.argtypes = [P, C.c_int, C.c_int, C.POINTER(C.c_double)]
        L.hlbm_objective_workspace_size.argtypes = [P, C.POINTER(Objective), C.POINTER(C.c_size_t)]
        L.hlbm_run_objective.argtypes = [P, C.POINTER(Objective), P, C.c_size_t, C.POINTER(C.c_double)]
        L.hlbm_adjoint.argtypes = [P, C.c_double, P, P]
        L.hlbm_wall_stats_begin.argtypes = [P]
        L.hlbm_wall_stats.argtypes = [P, C.POINTER(C.c_int64), P, P, P]
        _lib = L
    return _lib


def _np_ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def make_structs(nx_cells, ny_cells, patches=(), *, u_inf=0.05, aoa_rad=0.0, rho0=1.0,
                 precision=FP64, interp=INTERP_QUADRATIC, n_sub=0, periodic=False, wall_bc=True,
                 check_every=0, history_len=0, fv_fuse=0, mesh_xy=None, mesh_tri=None, mesh_kind=None,
                 chord=1.0, inner_ellipse=None, dxy_dshape=None, f2c_filter=False, body_xy=None):
    """ctypes Grid and Mesh (plus the arrays they point into, kept alive).

    dxy_dshape: optional [n_shape, n_nodes, 2] derivatives of the node
    coordinates with respect to shape parameters; the adjoint then returns
    dJ/d(parameter) for each of them.  body_xy: optional [n, 2] polygon of a
    solid body resolved on the finest level by bounce-back (no mesh)."""
    g = Grid()
    g.nx_cells, g.ny_cells, g.n_refine = nx_cells, ny_cells, len(patches)
    for k, (i0, j0, px, py) in enumerate(patches):
        g.patch_i0[k], g.patch_j0[k], g.patch_nx[k], g.patch_ny[k] = i0, j0, px, py
    g.u_inf, g.aoa_rad, g.rho0 = u_inf, aoa_rad, rho0
    g.precision, g.interp, g.n_sub = precision, interp, n_sub
    g.bc = BC_PERIODIC if periodic else BC_FARFIELD
    g.wall_bc, g.check_every, g.history_len = int(wall_bc), check_every, history_len
    g.fv_fuse = int(fv_fuse)
    g.f2c_filter = int(f2c_filter)
    m = Mesh()
    keep = []
    if mesh_xy is not None:
        xy = np.ascontiguousarray(mesh_xy, dtype=np.float64).reshape(-1, 2)
        tri = np.ascontiguousarray(mesh_tri, dtype=np.int32).reshape(-1, 3)
        kind = np.ascontiguousarray(mesh_kind, dtype=np.uint8)
        keep += [xy, tri, kind]
        m.n_nodes, m.n_tris = xy.shape[0], tri.shape[0]
        m.xy = xy.ctypes.data_as(C.POINTER(C.c_double))
        m.tri = tri.ctypes.data_as(C.POINTER(C.c_int32))
        m.kind = kind.ctypes.data_as(C.POINTER(C.c_uint8))
        if dxy_dshape is not None:
            d = np.ascontiguousarray(dxy_dshape, dtype=np.float64).reshape(-1, xy.shape[0], 2)
            keep.append(d)
            m.n_shape = d.shape[0]
            m.dxy_dshape = d.ctypes.data_as(C.POINTER(C.c_double))
    if body_xy is not None:
        bxy = np.ascontiguousarray(body_xy, dtype=np.float64).reshape(-1, 2)
        keep.append(bxy)
        m.body_n = bxy.shape[0]
        m.body_xy = bxy.ctypes.data_as(C.POINTER(C.c_double))
    m.chord = chord
    ein = inner_ellipse if inner_ellipse is not None else (0.0, 0.0, 0.0, 0.0)
    for k in range(4):
        m.inner_ellipse[k] = float(ein[k])
    return g, m, keep


def structs_from_workload(w, **over):
    kw = dict(u_inf=w.u_inf, aoa_rad=w.aoa_rad, rho0=w.rho0, periodic=w.periodic, n_sub=w.n_sub,
              mesh_xy=w.mesh_xy, mesh_tri=w.mesh_tri, mesh_kind=w.mesh_kind, chord=w.chord,
              inner_ellipse=w.inner_ellipse, f2c_filter=w.f2c_filter, body_xy=w.body_xy)
    kw.update(over)
    return make_structs(w.nx_cells, w.ny_cells, w.patches, **kw)


def validate(grid: Grid, mesh: Mesh, re: float = 0.0, tau: float = 0.0) -> int:
    return lib().hlbm_validate(C.byref(grid), C.byref(mesh), re, tau)


def last_error(ctx=None) -> str:
    return (lib().hlbm_last_error(ctx) or b"").decode()


def workspace_size(grid: Grid, mesh: Mesh, re: float = 0.0, tau: float = 0.0) -> int:
    n = C.c_size_t(0)
    rc = lib().hlbm_workspace_size(C.byref(grid), C.byref(mesh), re, tau, C.byref(n))
    if rc:
        raise HLBMError(rc, last_error())
    return n.value


class HLBM:
    """One HLBM problem on the current CUDA/HIP device.

    ``HLBM(grid, mesh, tau=...)`` with ctypes structs, or ``HLBM.from_workload(w)``.
    """

    def __init__(self, grid: Grid, mesh: Mesh, *, re: float = 0.0, tau: float = 0.0,
                 keep=(), stream=None, noalloc: bool = False):
        """noalloc: the library's static per-device workspace (hlbm_create_noalloc)
        instead of a torch buffer; one such context per device at a time."""
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("HLBM needs a GPU (torch.cuda is not available)")
        self._keep = list(keep)
        self.grid, self.mesh = grid, mesh
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        ctx = C.c_void_p()
        if noalloc:
            self.workspace = None
            rc = lib().hlbm_create_noalloc(C.byref(grid), C.byref(mesh), re, tau,
                                           C.c_void_p(self.stream.cuda_stream), C.byref(ctx))
        else:
            nbytes = workspace_size(grid, mesh, re, tau)
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            rc = lib().hlbm_create(C.byref(grid), C.byref(mesh), re, tau,
                                   C.c_void_p(self.workspace.data_ptr()), nbytes,
                                   C.c_void_p(self.stream.cuda_stream), C.byref(ctx))
        if rc:
            raise HLBMError(rc, last_error())
        self._ctx = ctx
        self.info = self.get_info()
        self.n_nodes = int(mesh.n_nodes)
        self.n_wall = 0
        if self.n_nodes > 0:
            kinds = np.ctypeslib.as_array(mesh.kind, shape=(self.n_nodes,))
            self.n_wall = int(np.count_nonzero(kinds == 1))

    @classmethod
    def from_workload(cls, w, *, precision=FP64, interp=INTERP_QUADRATIC, n_sub=0, wall_bc=True,
                      aoa_rad=None, tau=None, check_every=0, history_len=0, fv_fuse=0, stream=None,
                      dxy_dshape=None, noalloc=False):
        g, m, keep = structs_from_workload(
            w, precision=precision, interp=interp, n_sub=n_sub or w.n_sub, wall_bc=wall_bc,
            aoa_rad=w.aoa_rad if aoa_rad is None else aoa_rad, check_every=check_every,
            history_len=history_len, fv_fuse=fv_fuse, dxy_dshape=dxy_dshape)
        return cls(g, m, tau=w.tau_s if tau is None else tau, keep=keep, stream=stream, noalloc=noalloc)

    def _check(self, rc):
        if rc:
            raise HLBMError(rc, last_error(self._ctx))

    def close(self):
        if getattr(self, "_ctx", None):
            lib().hlbm_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_info(self) -> Info:
        info = Info()
        self._check(lib().hlbm_info(self._ctx, C.byref(info)))
        return info

    @property
    def t(self) -> int:
        return int(self.get_info().t)

    def step(self, n: int):
        self._check(lib().hlbm_step(self._ctx, int(n)))

    def step_logged(self, n: int, label: str = "", chunk: int = 20000):
        """step(n) in chunks of about `chunk` finest steps, each followed by a
        synchronisation and a progress line on stderr (for long runs)."""
        import sys
        per = 2 ** max(0, int(self.info.n_levels) - 1)
        chunk = max(per, chunk - chunk % per)
        done = 0
        while done < n:
            k = min(chunk, n - done)
            self.step(k)
            self.synchronize()
            done += k
            print(f"[{label}] {done}/{n} steps", file=sys.stderr, flush=True)

    def forces(self):
        cd, cl = C.c_double(), C.c_double()
        self._check(lib().hlbm_forces(self._ctx, C.byref(cd), C.byref(cl)))
        return cd.value, cl.value

    def history(self, t0: Optional[int] = None, t1: Optional[int] = None):
        t = self.t
        t1 = t if t1 is None else t1
        t0 = max(0, t1 - (self.grid.history_len or 65536)) if t0 is None else t0
        cd = np.zeros(max(t1 - t0, 1))
        cl = np.zeros(max(t1 - t0, 1))
        self._check(lib().hlbm_force_history(self._ctx, t0, t1, _np_ptr(cd), _np_ptr(cl)))
        return cd[:t1 - t0], cl[:t1 - t0]

    def level_shape(self, l: int):
        return (int(self.info.ny[l]), int(self.info.nx[l]))

    def get_state(self, part: int) -> np.ndarray:
        if part == PART_MESH:
            out = np.zeros((9, int(self.info.n_mesh_nodes)))
        else:
            out = np.zeros((9,) + self.level_shape(part))
        self._check(lib().hlbm_get_state(self._ctx, part, _np_ptr(out), out.size))
        return out

    def set_state(self, part: int, f: np.ndarray):
        f = np.ascontiguousarray(f, dtype=np.float64)
        self._check(lib().hlbm_set_state(self._ctx, part, _np_ptr(f), f.size))

    def profile(self, enable: bool = True):
        self._check(lib().hlbm_profile(self._ctx, int(enable)))

    def profile_read(self):
        """{kernel class: (total ms, launches)} since the last read."""
        ms = np.zeros(len(KERNEL_CLASSES))
        n = np.zeros(len(KERNEL_CLASSES), np.int64)
        self._check(lib().hlbm_profile_read(self._ctx, _np_ptr(ms), _np_ptr(n)))
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(KERNEL_CLASSES)}

    def kernel_bench(self, kclass: str, n: int) -> float:
        """Mean ms per launch of n back-to-back launches of one kernel class.

        Benchmark only: the state afterwards is not a solution of the scheme."""
        ms = C.c_double()
        self._check(lib().hlbm_kernel_bench(self._ctx, KERNEL_CLASSES.index(kclass), int(n), C.byref(ms)))
        return ms.value

    def _prepare_objective(self, t_end, t0, t1, ckpt_every, w_cd, w_cl, mesh_grad, store_substeps):
        """Objective struct and a workspace that holds it (allocated or grown here)."""
        import torch
        o = Objective(int(t_end), int(t0), int(t1), int(ckpt_every), float(w_cd), float(w_cl), int(bool(mesh_grad)), 0)
        n = C.c_size_t(0)
        if store_substeps is None or store_substeps:
            o.store_substeps = 1
            self._check(lib().hlbm_objective_workspace_size(self._ctx, C.byref(o), C.byref(n)))
            if store_substeps is None:
                free, _ = torch.cuda.mem_get_info()
                have = 0 if getattr(self, "obj_ws", None) is None else self.obj_ws.numel()
                o.store_substeps = int(n.value <= 0.5 * (free + have))
        self._check(lib().hlbm_objective_workspace_size(self._ctx, C.byref(o), C.byref(n)))
        if getattr(self, "obj_ws", None) is None or self.obj_ws.numel() < n.value:
            self.obj_ws = None   # release the smaller workspace first
            self.obj_ws = torch.empty(n.value, dtype=torch.uint8, device="cuda")
        return o

    def reserve_objective(self, t_end: int, t0: int, t1: int, ckpt_every: int = 100, w_cd: float = 1.0,
                          w_cl: float = 0.0, mesh_grad: bool = False, store_substeps=None):
        """Allocate the objective workspace of run_objective(same arguments) without running it."""
        self._prepare_objective(t_end, t0, t1, ckpt_every, w_cd, w_cl, mesh_grad, store_substeps)

    def run_objective(self, t_end: int, t0: int, t1: int, ckpt_every: int = 100, w_cd: float = 1.0,
                      w_cl: float = 0.0, mesh_grad: bool = False, store_substeps=None) -> float:
        """Run from the initial state and return the windowed mean of w_cd C_D + w_cl C_L.

        mesh_grad: the following adjoint also returns d J / d(mesh coordinates)
        and the shape-parameter gradient.
        store_substeps: keep the FV sub-step states of a segment instead of
        recomputing them (None: when the workspace stays under half the free
        device memory)."""
        o = self._prepare_objective(t_end, t0, t1, ckpt_every, w_cd, w_cl, mesh_grad, store_substeps)
        self._objective = o
        J = C.c_double()
        self._check(lib().hlbm_run_objective(self._ctx, C.byref(o), C.c_void_p(self.obj_ws.data_ptr()),
                                             self.obj_ws.numel(), C.byref(J)))
        return J.value

    def adjoint(self, j_bar: float = 1.0) -> np.ndarray:
        """[dJ/d aoa_rad, dJ/d tau, dJ/d a_0, ..] of the last run_objective (discrete
        adjoint), one entry per shape parameter of the mesh (NaN unless the
        objective asked for mesh_grad).

        When that objective asked for mesh_grad, d J / d(mesh coordinates) of
        the caller's nodes is left in ``self.grad_xy`` ([n_nodes, 2]).  The
        context is back at the end of the objective run afterwards."""
        g = np.zeros(2 + int(self.mesh.n_shape))
        gxy = np.zeros((self.n_nodes, 2)) if self._objective.mesh_grad else None
        self.grad_xy = None
        self._check(lib().hlbm_adjoint(self._ctx, float(j_bar), _np_ptr(g),
                                       None if gxy is None else _np_ptr(gxy)))
        self.grad_xy = gxy
        return g

    def wall_stats_begin(self):
        """Start time means of the wall coefficients C_p, C_f, C_n (eqs. (12)-(13))
        over the finest steps that follow."""
        self._check(lib().hlbm_wall_stats_begin(self._ctx))

    def wall_stats(self):
        """(steps, C_p, C_f, C_n) means since wall_stats_begin(), one entry per
        wall node in increasing node index.  C_f and C_n are the shear and normal
        viscous stress on the wall tangent t with the fluid on its left and the
        normal n into the fluid."""
        n = max(self.n_wall, 1)
        cp, cf, cn = np.zeros(n), np.zeros(n), np.zeros(n)
        steps = C.c_int64(0)
        self._check(lib().hlbm_wall_stats(self._ctx, C.byref(steps), _np_ptr(cp), _np_ptr(cf), _np_ptr(cn)))
        k = self.n_wall
        return int(steps.value), cp[:k], cf[:k], cn[:k]

    def synchronize(self):
        self.stream.synchronize()


def surface_distributions(omesh, cp: np.ndarray, cf: np.ndarray) -> dict:
    """Wall coefficients of an O-mesh along the chord, per surface.

    cp, cf: one value per surface point (wall nodes in node order, as
    HLBM.wall_stats returns them).  Returns {"upper": (x/c, C_p, C_f),
    "lower": (...)}, each ordered from the leading to the trailing edge, with
    C_f signed positive for shear towards the trailing edge (attached flow) on
    both surfaces: the wall tangent with the fluid on its left runs downstream
    on the upper surface and upstream on the lower one."""
    ns = omesh.ns
    le = ns // 2
    up = np.arange(le, -1, -1)                                # LE -> TE over the upper surface
    lo = np.concatenate([np.arange(le, ns), [0]])             # LE -> TE over the lower surface
    xi = omesh.surface_xi
    return {"upper": (xi[up], cp[up], cf[up]), "lower": (xi[lo], cp[lo], -cf[lo])}


def separation_point(xc: np.ndarray, cf: np.ndarray) -> Optional[float]:
    """First zero of C_f with negative slope along x/c (Sec. 6: separation is where
    the skin friction vanishes and turns negative), by linear interpolation
    between the two bracketing points; None if C_f never changes from positive
    to non-positive."""
    for k in range(len(xc) - 1):
        if cf[k] > 0.0 >= cf[k + 1]:
            return float(xc[k] + cf[k] * (xc[k + 1] - xc[k]) / (cf[k] - cf[k + 1]))
    return None


def strouhal(cl: np.ndarray, chord: float, u_inf: float, steady_tol: float = 1e-6) -> float:
    """Strouhal number c / (U T) of a lift history sampled every finest step.

    T is the mean spacing of the upward crossings of C_L - mean(C_L), located
    by linear interpolation.  Returns NaN for a steady signal (peak-to-peak
    below steady_tol) or fewer than two crossings.
    """
    cl = np.asarray(cl, dtype=np.float64)
    if cl.size < 3 or np.ptp(cl) < steady_tol:
        return math.nan
    x = cl - cl.mean()
    idx = np.nonzero((x[:-1] < 0) & (x[1:] >= 0))[0]
    if idx.size < 2:
        return math.nan
    tc = idx + (-x[idx]) / (x[idx + 1] - x[idx])
    period = (tc[-1] - tc[0]) / (idx.size - 1)
    return chord / (u_inf * period)


def objective_function():
    """torch.autograd.Function J(aoa_rad, tau, bumps) of the HLBM drag/lift objective.

    Usage: ``J = objective_function().apply(aoa, tau, bumps, build, spec)`` with
    ``aoa`` and ``tau`` 0-d float64 CPU tensors, ``bumps`` a float64 CPU tensor of
    Hicks-Henne amplitudes (or None for a fixed shape), ``build`` a callable
    mapping the amplitudes (numpy array or None) to a workload whose ``omesh``
    provides ``bump_tangent``, and ``spec`` a dict with t_end, t0, t1,
    ckpt_every, w_cd, w_cl.  forward runs the GPU objective on a mesh that
    carries the generator's bump tangent as its shape derivatives; backward
    runs the discrete adjoint of the same run, which returns the gradient with
    respect to the angle, tau and every amplitude.
    """
    import torch

    class HLBMObjective(torch.autograd.Function):
        @staticmethod
        def forward(ctx, aoa, tau, bumps, build, spec):
            from . import workloads
            amps = None if bumps is None else bumps.detach().cpu().numpy().astype(np.float64)
            w = build(amps)
            want_shape = bumps is not None and ctx.needs_input_grad[2]
            tan = None
            if want_shape:
                peaks = getattr(build, "peaks", None)
                tan = w.omesh.bump_tangent(workloads.HH_PEAKS if peaks is None else peaks)
            sim = HLBM.from_workload(w, aoa_rad=float(aoa), tau=float(tau), precision=FP64,
                                     history_len=max(65536, int(spec["t_end"])), dxy_dshape=tan)
            J = sim.run_objective(**spec, mesh_grad=want_shape)
            ctx.sim, ctx.want_shape = sim, want_shape
            return torch.tensor(J, dtype=torch.float64)

        @staticmethod
        def backward(ctx, g):
            grad = ctx.sim.adjoint(float(g))
            gb = torch.tensor(grad[2:], dtype=torch.float64) if ctx.want_shape else None
            ctx.sim.close()
            return (torch.tensor(grad[0], dtype=torch.float64), torch.tensor(grad[1], dtype=torch.float64),
                    gb, None, None)

    return HLBMObjective
