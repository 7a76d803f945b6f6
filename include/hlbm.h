/*
 * hlbm.h -- C ABI of the hybrid lattice Boltzmann (HLBM) step on one MI355X.
 *
 * Method: G. Di Ilio et al., "Fluid flow around NACA 0012 airfoil at low
 * Reynolds numbers with hybrid lattice Boltzmann method" (arXiv 2006.10487).
 * One call of hlbm_step advances, per finest time step:
 *   - the D2Q9 BGK collide-stream of eq. (1)-(2) on a uniform Cartesian grid
 *     with nested factor-two refinement boxes and time subcycling (Sec. 4);
 *   - the cell-vertex finite-volume update of eq. (3) on a body-fitted
 *     triangular mesh, n sub-steps per structured step (Sec. 6.3);
 *   - the two-way coupling of eqs. (4)-(7) at interpolation nodes, with the
 *     quadratic interpolations of eqs. (8)-(9) (Sec. 3);
 *   - the drag and lift of eqs. (10)-(11) from the wall momentum flux.
 *
 * Conventions.
 *   - Coordinates and times are lattice units of the finest structured level
 *     (spacing 1, time step 1).  Level 0 is the coarsest (base) grid; level
 *     n_refine is the finest.  Level l has spacing 2^(n_refine - l).
 *   - D2Q9 population order: (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1)
 *     (-1,-1) (1,-1).
 *   - Host arrays passed in are borrowed for the duration of the call.  The
 *     device workspace is owned by the caller, must stay allocated until
 *     hlbm_destroy, and is carved by the library; the library never allocates
 *     device memory and enqueues all work on the caller's HIP stream.
 *   - Every function returns HLBM_OK (0) or a negative error code; the text
 *     of the last error of a context is given by hlbm_last_error.
 *   - One host thread per context.  hlbm_step is asynchronous; calls that
 *     return host data synchronise the stream.
 */
#ifndef HLBM_H
#define HLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    HLBM_OK = 0,
    HLBM_E_ARG = -1,        /* null pointer, out-of-range argument, bad part or count     */
    HLBM_E_GEOMETRY = -2,   /* mesh not counter-clockwise, degenerate control volume,
                               box outside its parent, stencil donor not active, ...      */
    HLBM_E_PARAM = -3,      /* tau <= 1/2 on some level, Re and tau inconsistent          */
    HLBM_E_DEVICE = -4,     /* a HIP call failed                                          */
    HLBM_E_NONFINITE = -5,  /* non-finite force detected; context poisoned                */
    HLBM_E_STATE = -6,      /* call not allowed in this state (e.g. poisoned context)     */
    HLBM_E_WORKSPACE = -7   /* workspace too small or misaligned                          */
};

enum { HLBM_FP64 = 0, HLBM_FP32_SHIFTED = 1 };
enum { HLBM_INTERP_QUADRATIC = 0, HLBM_INTERP_LINEAR = 1 };
enum { HLBM_BC_FARFIELD = 0, HLBM_BC_PERIODIC = 1 };
enum { HLBM_PART_MESH = 100 };   /* hlbm_get_state / hlbm_set_state: mesh populations */

typedef struct hlbm_ctx hlbm_ctx;

/* Structured grid and run options. */
typedef struct {
    int32_t nx_cells, ny_cells;   /* base-level cells (nodes = cells + 1; periodic: nodes = cells) */
    int32_t n_refine;             /* nested refinement boxes, 0..3                                  */
    int32_t patch_i0[3], patch_j0[3]; /* box origin, in nodes of its parent level                  */
    int32_t patch_nx[3], patch_ny[3]; /* box size in its own cells (even)                          */
    double u_inf;                 /* free-stream speed (finest lattice units)                       */
    double aoa_rad;               /* angle of attack: the free stream is U (cos a, sin a)           */
    double rho0;                  /* reference density (1)                                          */
    int32_t precision;            /* HLBM_FP64 or HLBM_FP32_SHIFTED                                 */
    int32_t interp;               /* HLBM_INTERP_QUADRATIC (eqs 8-9) or HLBM_INTERP_LINEAR          */
    int32_t n_sub;                /* FV sub-steps per finest step; 0 = max(10, ceil(1 / tau_u))      */
    int32_t bc;                   /* HLBM_BC_FARFIELD or HLBM_BC_PERIODIC (base level)              */
    int32_t wall_bc;              /* 1 = no-slip at mesh wall nodes, 0 = off (free-stream checks)    */
    int32_t check_every;          /* non-finite check interval in finest steps, 0 = off             */
    int32_t history_len;          /* force history ring length, 0 = 65536                            */
    int32_t fv_fuse;              /* FV sub-steps per launch, 1..4 (falls back to the largest count
                                     whose tile of mesh nodes and halo fit in 64 KB of LDS with at
                                     most 512 updated nodes per tile, else 1); 0 = 2 on meshes with at most
                                     8 neighbour slots per node, else 1.  Results do not depend on
                                     it (same arithmetic, same order)                                */
    int32_t f2c_filter;           /* fine -> coarse transfer (Sec. 4): 0 = the rescaled f^neq of the
                                     coincident fine node; 1 = that f^neq full-weighted over the
                                     3 x 3 fine nodes around it (weights (2-|di|)(2-|dj|)/16), which
                                     keeps the interface stable with tau close to 1/2 on the coarse
                                     levels (boxes of at least 8 x 8 cells)                          */
} hlbm_grid;

/* Body-fitted triangular mesh (Sec. 2 and 4). */
typedef struct {
    int32_t n_nodes, n_tris;      /* 0 nodes = no mesh (structured grid only)                       */
    const double *xy;             /* [2 * n_nodes] node coordinates                                 */
    const int32_t *tri;           /* [3 * n_tris] counter-clockwise vertex triples                  */
    const uint8_t *kind;          /* [n_nodes] 0 interior, 1 wall (no-slip), 2 interpolation node   */
    double chord;                 /* reference length of eqs. (10)-(11)                             */
    double inner_ellipse[4];      /* xc, yc, a, b of the inner fictitious ellipse; structured nodes
                                     strictly inside are inactive (a <= 0: none)                     */
    int32_t n_shape;              /* shape parameters a_m of the discrete adjoint (0: none)         */
    const double *dxy_dshape;     /* [n_shape][n_nodes][2] d(node x, y)/d a_m in the caller's node
                                     order (borrowed, copied at create), or NULL when n_shape = 0   */
    int32_t body_n;               /* without a mesh (n_nodes = 0, no inner ellipse): vertices of a
                                     solid body resolved on the finest structured level, the standard
                                     LBM that eq. (14) compares the hybrid scheme with; 0 = none.
                                     Nodes strictly inside the polygon (crossing number, an edge
                                     counted when exactly one of its end points has y' <= y) are
                                     solid, one run of them per row, at least 6 nodes from the edges
                                     of the finest level.  A population that would stream out of a
                                     solid node is the fluid node's own post-collision population of
                                     the opposite direction (halfway bounce-back); C_D and C_L come
                                     from the momentum those populations exchange with the body,
                                     2 c_i f~_i per link, over rho0 U^2 chord / 2                    */
    const double *body_xy;        /* [2 * body_n] polygon vertices (x, y) in finest-level coordinates
                                     (borrowed, copied at create), or NULL when body_n = 0           */
} hlbm_mesh;

typedef struct {
    int32_t n_levels;             /* n_refine + 1 (0 without a grid)                                */
    int32_t n_sub;                /* FV sub-steps per finest step                                   */
    int32_t nx[4], ny[4], pitch[4];   /* nodes and row pitch (elements) per level                  */
    double tau[4];                /* relaxation time per level (level units)                        */
    double tau_u;                 /* FV relaxation time = tau_finest - 1/2 (finest units)           */
    int64_t active_nodes[4];      /* collide-stream nodes per level                                 */
    int32_t n_mesh_nodes, n_wall_nodes, n_interp_mesh, n_interp_struct, n_fallback;
    int32_t n_wall_edges, nnz;
    int64_t bytes_per_finest_step;    /* algorithmic bytes, all kernels                             */
    int64_t k1_bytes[4];          /* algorithmic bytes of one collide-stream launch per level:
                                     9 populations read and 9 written per active node               */
    int64_t fv_bytes;             /* algorithmic bytes of one FV sub-step: per mesh node the 9
                                     populations read and written, its own C_PP and G_PP, and
                                     one row pointer; per neighbour entry its column index and
                                     (G_x, G_y, C) -- what eq. (3) must move, whatever the layout    */
    int64_t t;                    /* finest steps done                                              */
    size_t workspace_bytes;
    int32_t fv_fuse;              /* FV sub-steps per launch (the HLBM_K_FV class of hlbm_profile_read
                                     and hlbm_kernel_bench covers that many)                         */
    int32_t fv_tiles;             /* workgroups of one fused FV launch (tiles), 0 when fv_fuse = 1  */
    int32_t fv_tile_nodes;        /* nominal mesh nodes per tile                                    */
    int32_t fv_threads;           /* threads per fused-launch workgroup                             */
    int64_t fv_layout_bytes;      /* bytes one unfused FV sub-step of this layout reads and writes:
                                     node records with their stored moments (rho, u) in and out,
                                     every slot of the padded neighbour table                       */
    int32_t n_solid;              /* solid nodes of a body resolved by bounce-back (0: none)         */
    int32_t n_bounce;             /* fluid nodes next to it (at least one bounce-back link)          */
} hlbm_info_t;

/* Checks the problem on the host only (no GPU).  Re > 0 gives
 * tau = 1/2 + 3 U chord / Re (nu = c_s^2 (tau - 1/2), Sec. 2); tau > 1/2 is used
 * as is, and then Re must be <= 0 or consistent to 1e-12.  Returns HLBM_OK or
 * HLBM_E_ARG / HLBM_E_GEOMETRY / HLBM_E_PARAM. */
int hlbm_validate(const hlbm_grid *grid, const hlbm_mesh *mesh, double Re, double tau);

/* Device workspace bytes needed by hlbm_create (host only, no GPU). */
int hlbm_workspace_size(const hlbm_grid *grid, const hlbm_mesh *mesh, double Re, double tau,
                        size_t *ws_bytes);

/* Builds the context for the problem of Sec. 4: host preprocessing
 * (median-dual control volumes and the S, C coefficients of eq. (3), the
 * stencils of eqs. (8)-(9), node order), copies the tables into d_workspace
 * (device pointer, 256-byte aligned, ws_bytes >= hlbm_workspace_size; the
 * caller keeps ownership) and sets the initial state f^eq(rho0, u_inf) of
 * eq. (2) (f^eq(rho0, 0) at wall nodes).  Re and tau as in hlbm_validate.
 * hip_stream is a hipStream_t (NULL = default stream); all device work of the
 * context goes on it.  Errors: those of hlbm_validate, HLBM_E_WORKSPACE,
 * HLBM_E_DEVICE.  On failure *out is NULL and nothing is left allocated. */
int hlbm_create(const hlbm_grid *grid, const hlbm_mesh *mesh, double Re, double tau,
                void *d_workspace, size_t ws_bytes, void *hip_stream, hlbm_ctx **out);

/* Size of the static workspace of hlbm_create_noalloc (bytes). */
#define HLBM_NOALLOC_MAX_BYTES ((size_t)64 << 20)

/* hlbm_create for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * workspace is a static device array of HLBM_NOALLOC_MAX_BYTES that the
 * library holds on each device it runs on until the process ends, instead of
 * a caller buffer.  No hipMalloc, hipFree or other allocating routine is
 * called.  Problems whose hlbm_workspace_size exceeds the array get
 * HLBM_E_WORKSPACE (host-side check, before any device work); the Re = 100
 * workloads of the tests (about 35-39 MiB) fit.  Every context created this
 * way on one device uses that device's array: creating another one overwrites
 * the earlier context's state (destroy it first), and work on two such
 * contexts of one device races.  The array keeps the contents of the last
 * call; create writes every part of it that the context reads before reading
 * it.  Otherwise as hlbm_create; hlbm_destroy frees only host memory. */
int hlbm_create_noalloc(const hlbm_grid *grid, const hlbm_mesh *mesh, double Re, double tau, void *hip_stream,
                        hlbm_ctx **out);

/* Advances n_finest_steps finest steps (a multiple of 2^n_refine): per finest
 * step the coupling of eq. (4), the collide-stream of eqs. (1)-(2) on every
 * level with the subcycling and box transfers of Sec. 4, eq. (9), the n
 * finite-volume sub-steps of eqs. (3) and (5)-(7), and the force of
 * eqs. (10)-(11) into the history.  Async (enqueued on the context's stream).
 * Errors: HLBM_E_ARG (count), HLBM_E_STATE (poisoned context),
 * HLBM_E_NONFINITE (a non-finite force at a check_every boundary; the context
 * is poisoned). */
int hlbm_step(hlbm_ctx *ctx, int64_t n_finest_steps);

/* Drag and lift coefficients of the last finest step (eqs. (10)-(11)).  Syncs. */
int hlbm_forces(hlbm_ctx *ctx, double *cd, double *cl);

/* Coefficients of finest steps [t0, t1) (within the last history_len steps).  Syncs. */
int hlbm_force_history(hlbm_ctx *ctx, int64_t t0, int64_t t1, double *cd, double *cl);

/* Canonical state in FP64: the populations f_i of eq. (1) (structured) and of
 * eq. (3) (mesh) after the last finest step.  part = level l: pre-collision
 * populations [9][ny][nx] of level l (host array, row-major, x fastest), zero
 * at nodes that are not collide-stream nodes; part = HLBM_PART_MESH: mesh
 * populations [9][n_nodes] in the caller's node order.  count = number of
 * doubles (HLBM_E_ARG if it does not match).  FP32-shifted contexts return
 * w_i rho0 + the stored value.  Syncs. */
int hlbm_get_state(hlbm_ctx *ctx, int32_t part, double *host, size_t count);

/* Replaces a part of the state of eqs. (1) and (3) (same layout and count
 * rule as hlbm_get_state; on a level, values at non-collide-stream nodes are
 * ignored; copied from the borrowed host array).  Set every level and the
 * mesh before stepping on: the next step rebuilds the derived values (box
 * transfers of Sec. 4, eq. (9) at t) from them.  Ends wall statistics.
 * Syncs. */
int hlbm_set_state(hlbm_ctx *ctx, int32_t part, const double *host, size_t count);

int hlbm_info(hlbm_ctx *ctx, hlbm_info_t *out);

/* Objective for the discrete adjoint: a run of t_end finest steps from the
 * initial state; J = mean over history entries h in [t0, t1) of
 * w_cd C_D(h) + w_cl C_L(h) (eqs. (10)-(11)).  The forward stores the state
 * every ckpt_every steps in the objective workspace (revolve-style
 * checkpointing); the reverse sweep recomputes each segment from its
 * checkpoint.  mesh_grad != 0 asks the adjoint for d J / d(mesh node
 * coordinates) as well (shape gradient; needs more workspace).  Gradients do
 * not depend on ckpt_every or store_substeps. */
typedef struct {
    int64_t t_end, t0, t1, ckpt_every;
    double w_cd, w_cl;
    int32_t mesh_grad;
    int32_t store_substeps;   /* != 0: keep every FV sub-step state of a segment
                                 (ckpt_every * n_sub mesh states more workspace)
                                 instead of recomputing them in the reverse sweep */
} hlbm_objective;

/* Device bytes of the objective workspace (checkpoints, one recomputed
 * segment, the adjoint fields and transposed tables).  Supported: FP64
 * contexts with a walled mesh and any number of refinement boxes; other
 * contexts get HLBM_E_ARG. */
int hlbm_objective_workspace_size(hlbm_ctx *ctx, const hlbm_objective *obj, size_t *bytes);

/* Restarts the run from the initial state, advances obj->t_end finest steps,
 * storing checkpoints in d_ckpt (device, 256-byte aligned, caller-owned), and
 * returns J.  Syncs. */
int hlbm_run_objective(hlbm_ctx *ctx, const hlbm_objective *obj, void *d_ckpt, size_t ckpt_bytes, double *J);

/* Discrete adjoint of the last hlbm_run_objective, reverse mode over the
 * forward kernels (eqs. (1)-(11) as implemented), FP64 accumulation,
 * deterministic.  grad (host, 2 + n_shape doubles):
 *   grad[0]      = J_bar dJ/d aoa_rad,
 *   grad[1]      = J_bar dJ/d tau (finest-level relaxation time; the number of
 *                  FV sub-steps is held fixed),
 *   grad[2 + m]  = J_bar dJ/d a_m = J_bar sum over nodes of dJ/d(x, y) .
 *                  dxy_dshape[m] (the mesh's shape parameters), when the
 *                  objective's mesh_grad is set; NaN (not computed) otherwise.
 * The mesh-coordinate gradient runs through the finite-volume coefficients of
 * eq. (3), the wall normals of eqs. (10)-(11) and the interpolation weights of
 * eqs. (8)-(9), with node kinds, connectivity, stencil donors and the inactive
 * structured region held fixed.  grad_xy (host, 2 * n_nodes doubles, caller's
 * node order, (x, y) pairs) optionally receives J_bar dJ/d(mesh coordinates)
 * itself when mesh_grad is set (NULL: not wanted); it must be NULL otherwise
 * (HLBM_E_ARG).  Afterwards the context holds the state at t_end of the
 * objective run again (as after hlbm_run_objective), so stepping, forces and
 * state export continue from there; a second adjoint needs a new objective
 * run (HLBM_E_STATE).  Syncs. */
int hlbm_adjoint(hlbm_ctx *ctx, double J_bar, double *grad, double *grad_xy);

/* Mean wall coefficients, eqs. (12)-(13).  After hlbm_wall_stats_begin, every
 * finest step taken by hlbm_step adds its post-step values at each wall node
 * (kind 1) to FP64 running sums on the device:
 *   C_p = (rho - rho0) c_s^2 / q   (pressure p = rho c_s^2, q = rho0 u_inf^2 / 2),
 *   C_f = t . sigma . n / q        (wall shear stress),
 *   C_n = n . sigma . n / q        (normal viscous stress),
 * with sigma = -(sum_i c_i c_i f_i - rho c_s^2 I - rho u u), the viscous
 * stress of the continuous BGK equation that the finite-volume scheme
 * integrates (viscosity c_s^2 tau_u), n the unit normal into the fluid
 * (opposite to the sum of the node's two half wall-edge normals) and
 * t = (n_y, -n_x) the wall tangent with the fluid on its left.  Clears the sums
 * (async).  hlbm_run_objective and hlbm_set_state end the accumulation. */
int hlbm_wall_stats_begin(hlbm_ctx *ctx);

/* Time means since hlbm_wall_stats_begin: *n_steps = number of finest steps
 * averaged; cp, cf (and cn unless NULL) receive one value per wall node, in
 * increasing caller node index (host arrays of n_wall doubles, n_wall = number
 * of kind-1 nodes).  HLBM_E_STATE when no accumulation is in effect or no step
 * was taken.  Syncs. */
int hlbm_wall_stats(hlbm_ctx *ctx, int64_t *n_steps, double *cp, double *cf, double *cn);

/* Kernel classes timed by hlbm_profile_read. */
enum {
    HLBM_K_COLLIDE_L0 = 0,      /* collide-stream of level 0 (+1, +2, +3 for finer levels) */
    HLBM_K_COARSE_TO_FINE = 4,
    HLBM_K_FINE_TO_COARSE = 5,
    HLBM_K_MESH_TO_STRUCT = 6,  /* eq. (4) */
    HLBM_K_STRUCT_TO_MESH = 7,  /* eq. (9) */
    HLBM_K_FV = 8,              /* finite-volume sub-steps, eqs. (3), (5): one launch = fv_fuse of them */
    HLBM_K_FORCE = 9,           /* eqs. (10)-(11) */
    HLBM_K_WALL_STATS = 10,     /* eqs. (12)-(13), while hlbm_wall_stats_begin is in effect */
    HLBM_K_COUNT = 11
};

/* Instrumentation: with enable != 0, every kernel launched by hlbm_step is
 * bracketed by a pair of HIP events recorded on the context's stream.  Events
 * are created by the library on first use (no device memory is allocated). */
int hlbm_profile(hlbm_ctx *ctx, int enable);

/* Synchronises the stream and returns, per kernel class, the summed
 * event-measured time in ms and the launch count since the last read
 * (arrays of HLBM_K_COUNT entries); then resets the counters. */
int hlbm_profile_read(hlbm_ctx *ctx, double *ms, int64_t *launches);

/* Instrumentation: launches n times back to back the kernel of class kclass
 * (HLBM_K_COLLIDE_L0 + l, or HLBM_K_FV: one launch of hlbm_info_t.fv_fuse
 * sub-steps) on the context's buffers and returns
 * the mean time per launch from one pair of HIP events around the batch.
 * The launches advance that part of the state on its own, so afterwards the
 * state is not a solution of the coupled scheme: benchmark use only (restore
 * with hlbm_set_state or create a new context).  Syncs. */
int hlbm_kernel_bench(hlbm_ctx *ctx, int kclass, int n, double *avg_ms);

/* Text of the last error of ctx (or of the last failed create when ctx is NULL). */
const char *hlbm_last_error(const hlbm_ctx *ctx);

/* Releases the host side of the context (the workspace stays the caller's). */
void hlbm_destroy(hlbm_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* HLBM_H */
