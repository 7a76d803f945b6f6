/*
 * hlbm_oracle.c -- plain FP64 CPU oracle of the hybrid lattice Boltzmann step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the HIP library; it is written for a reader
 * who checks it against the paper, not for speed (plain loops, no blocking,
 * no fusion, -ffp-contract=off; OpenMP only splits independent node loops).
 *
 * Paper: G. Di Ilio et al., "Fluid flow around NACA 0012 airfoil at low
 * Reynolds numbers with hybrid lattice Boltzmann method" (arXiv 2006.10487).
 *
 * What it computes, per finest time step t -> t+1 (Delta t_s = 1 on the
 * finest level):
 *   1. structured BGK collision + streaming on every level, eq. (1)-(2),
 *      with nested factor-two boxes and time subcycling (Sec. 4);
 *   2. structured interpolation nodes from the mesh, eq. (4) with the
 *      six-node quadratic interpolation of eq. (8);
 *   3. n finite-volume sub-steps of eq. (3) on the triangular mesh; the mesh
 *      interpolation nodes follow eq. (5) with the star values of eqs. (6)-(7)
 *      and the nine-node interpolation of eq. (9);
 *   4. drag and lift from the wall momentum flux, eqs. (10)-(11).
 *
 * Readings of points the paper leaves open (each is a constant of the run):
 *   - lattice: D2Q9, order (0,0),(1,0),(0,1),(-1,0),(0,-1),(1,1),(-1,1),
 *     (-1,-1),(1,-1); weights 4/9, 1/9, 1/36; c_s^2 = 1/3.
 *   - tau_u = tau_s - 1/2 (the viscosities of Sec. 2 agree); Delta t_u = 1/n.
 *   - S and C of eq. (3): median-dual control volumes with piecewise linear
 *     f; S_ik = c_i . G_Pk, C_Pk = (1/A_P) integral of the hat function of k
 *     over the control volume of P; lumped time derivative.
 *   - mesh boundary control volumes are closed by half boundary edges.
 *   - refinement (Sec. 4, Filippova-Haenel): acoustic scaling
 *     tau_c - 1/2 = 2 (tau_f - 1/2); non-equilibrium rescaled by tau_f/(2 tau_c)
 *     coarse -> fine and by 2 tau_c / tau_f fine -> coarse; linear in space at
 *     odd fine nodes and linear in time.
 *   - far field: non-equilibrium extrapolation at inlet (u given, rho from the
 *     neighbour) and outlet (rho given, u from the neighbour); all nine
 *     populations copied from the inner neighbour at top and bottom.
 *   - no-slip on the mesh: half control volume update, then u -> 0 keeping
 *     rho and the non-equilibrium part.
 *   - the standard LBM that resolves the body, against which eq. (14) prices
 *     the hybrid scheme (no mesh, the body a polygon on the finest level):
 *     nodes strictly inside the polygon (crossing-number test, an edge counted
 *     when exactly one of its end points lies on or below the node's row) are
 *     solid; a population that would stream out of a solid node is the
 *     fluid node's own post-collision population of the opposite direction
 *     (halfway bounce-back, wall midway between the two nodes), and the force
 *     on the body is the momentum those populations bring back, 2 c f~ per
 *     link (momentum exchange).
 *   - exchange order inside a finest step: eq. (4) from the mesh at t, the
 *     finest level to t+1, eq. (9) at t+1, then the n sub-steps with the
 *     structured values blended linearly in time.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* Arithmetic type.  The plain build computes in FP64 (real == double).  The
 * complex-step build (-DOR_COMPLEX_STEP) makes every quantity that depends on
 * the angle of attack, tau, the free stream or the mesh coordinates complex:
 * with an input perturbed by i h v (h ~ 1e-30), the imaginary part of any
 * output divided by h is its exact directional derivative along v, free of
 * the cancellation of finite differences (complex-step differentiation,
 * Squire and Trapp 1998; Martins, Sturdza and Alonso 2003).  Branches,
 * pivot choices and point location look at real parts only, so the real part
 * repeats the FP64 build operation for operation.  ABS_A is the analytic
 * absolute value the method needs (sign taken from the real part). */
#ifdef OR_COMPLEX_STEP
#include <complex.h>
#include <tgmath.h>
typedef double complex real;
#define RE(x) creal(x)
#else
typedef double real;
#define RE(x) (x)
#endif
#define ABS_A(x) (RE(x) < 0.0 ? -(x) : (x))

#define Q 9

/* D2Q9 velocities and weights. */
static const int CX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double W[Q] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
/* index of -c_i */
static const int OPPOSITE[Q] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

/* Deliberate-mistake multipliers for mutation tests of the pins (all 1 in a
 * normal run): [0] eq. (4) non-equilibrium factor, [1] eq. (5)-(6) factor,
 * [2] coarse -> fine rescaling, [3] fine -> coarse rescaling, [4] the
 * non-equilibrium part kept by the no-slip reset of wall nodes, [5] the reset
 * itself (0 skips it), [6] the time fraction theta = m/n at which the
 * structured values are blended into the finite-volume sub-steps, [7] the
 * bounce-back at a solid body (0: the population of the same direction comes
 * back instead of the opposite one), [8] the returning half of the momentum
 * exchanged per bounce-back link (0: only the outgoing population counts). */
#define N_PLANT 9
static double plant[N_PLANT] = {1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0};

void or_plant(int32_t which, double value)
{
    if (which >= 0 && which < N_PLANT) plant[which] = value;
}

/* node classes of a structured level */
enum { CL_ACTIVE = 0, CL_INACTIVE = 1, CL_INTERP = 2, CL_PERIM = 3, CL_RING = 4, CL_COVERED = 5, CL_SOLID = 6 };
enum { KIND_INTERIOR = 0, KIND_WALL = 1, KIND_INTERP = 2 };

typedef struct {
    /* structured grid (finest lattice units) */
    int32_t nx_cells, ny_cells;       /* base level cells; 0 = no structured grid   */
    int32_t n_refine;                 /* nested boxes, 0..3                          */
    int32_t patch_i0[3], patch_j0[3]; /* box origin in parent nodes                  */
    int32_t patch_nx[3], patch_ny[3]; /* box size in its own cells                   */
    int32_t periodic;                 /* base level periodic (no far-field BCs)      */
    int32_t wall_bc;                  /* 1: no-slip reset at wall nodes              */
    int32_t n_sub;                    /* FV sub-steps per finest step; 0 = default   */
    int32_t interp;                   /* 0 quadratic (eqs 8-9), 1 linear             */
    real u_inf, aoa, rho0, tau_s;   /* free stream, finest-level tau               */
    double chord;
    double ein[4];                    /* inner ellipse xc, yc, a, b (a <= 0: none)   */
    double mesh_period[2];            /* periodic mesh (0 = not periodic)            */
    /* mesh */
    int32_t n_nodes, n_tris;
    const real *xy;                 /* [2*n_nodes]                                 */
    const int32_t *tri;               /* [3*n_tris] counter-clockwise                */
    const uint8_t *kind;              /* [n_nodes]                                   */
    /* channel variant of the base-level boundaries (closed-form checks only):
     * no-slip top and bottom by non-equilibrium extrapolation, parabolic inlet */
    int32_t channel;
    /* fine -> coarse restriction: 0 = f^neq of the coincident fine node,
     * 1 = f^neq full-weighted over the 3 x 3 fine nodes around it */
    int32_t f2c_filter;
    /* solid body resolved on the finest level by bounce-back (no mesh):
     * polygon vertices (x, y) in finest-level units, body_n = 0: none */
    int32_t body_n;
    const double *body_xy;
} or_cfg;

typedef struct {
    int nx, ny;          /* nodes */
    int sp;              /* spacing in finest units */
    double ox, oy;       /* origin (finest units) */
    real tau;
    int i0, j0;          /* origin in parent nodes (levels > 0) */
    uint8_t *cls;
    real *f;           /* pre-collision [Q][ny][nx] */
    real *post;        /* post-collision */
    real *save;        /* pre-collision at the start of the current step */
} olevel;

typedef struct {
    or_cfg cfg;
    int L;                 /* number of refinement boxes; levels 0..L */
    olevel lev[4];
    /* mesh */
    int nn, nt;
    real *xy;
    int32_t *tri;
    uint8_t *kind;
    int *rowptr, *col;     /* CSR, neighbours sorted, self included */
    real *gx, *gy, *cc;  /* G_Pk and C_Pk */
    real *area;          /* A_P */
    int n_wall_edges;
    int *wedge;            /* [2*n] directed P->Q, fluid on the left */
    real *fu, *fu_new;   /* mesh populations [Q][nn] */
    /* interpolation node lists */
    int n_sint;            /* structured interpolation nodes (finest level) */
    int *sint_ij;          /* [2*n] */
    int *sint_don;         /* [8*n] mesh donors (-1 unused) */
    real *sint_w;        /* [8*n] */
    int n_fallback;
    int n_uint;            /* mesh interpolation nodes */
    int *uint_node;        /* [n] mesh node index */
    int *uint_slot;        /* [nn] slot or -1 */
    int *uint_don;         /* [9*n] finest-level node (i + nx*j) */
    real *uint_w;        /* [9*n] */
    int n_sub;
    real tau_u;
    int64_t t;             /* finest steps done */
    int64_t hist_cap;
    real *cd, *cl;
    /* running sums of the wall coefficients, eqs. (12)-(13), per wall node */
    int ws_on, n_wn;
    int64_t ws_n;
    real *ws_sum, *ws_tmp; /* [3][n_wn] each */
    char err[256];
} oracle_t;

/* ------------------------------------------------------------------ */
/* D2Q9 basics: moments and the second-order equilibrium, eq. (2)       */
/* ------------------------------------------------------------------ */

static void moments(const real *f, real *rho, real *ux, real *uy)
{
    real r = 0.0, mx = 0.0, my = 0.0;
    for (int i = 0; i < Q; ++i) {
        r += f[i];
        mx += f[i] * CX[i];
        my += f[i] * CY[i];
    }
    *rho = r;
    *ux = mx / r;
    *uy = my / r;
}

/* f_i^eq = w_i rho (1 + c.u / c_s^2 + (c.u)^2 / (2 c_s^4) - u^2 / (2 c_s^2)), c_s^2 = 1/3 */
static void equilibrium(real rho, real ux, real uy, real *feq)
{
    const double cs2 = 1.0 / 3.0;
    real uu = ux * ux + uy * uy;
    for (int i = 0; i < Q; ++i) {
        real cu = CX[i] * ux + CY[i] * uy;
        feq[i] = W[i] * rho * (1.0 + cu / cs2 + (cu * cu) / (2.0 * cs2 * cs2) - uu / (2.0 * cs2));
    }
}

void or_equilibrium(real rho, real ux, real uy, real *feq) { equilibrium(rho, ux, uy, feq); }

void or_lattice(int32_t *cx, int32_t *cy, real *w)
{
    for (int i = 0; i < Q; ++i) { cx[i] = CX[i]; cy[i] = CY[i]; w[i] = W[i]; }
}

/* BGK collision of eq. (1): f~ = f - (f - f^eq) / tau (Delta t_s = 1 in level units) */
static void bgk(const real *f, real tau, real *out)
{
    real rho, ux, uy, feq[Q];
    moments(f, &rho, &ux, &uy);
    equilibrium(rho, ux, uy, feq);
    for (int i = 0; i < Q; ++i) out[i] = f[i] - (f[i] - feq[i]) / tau;
}

void or_bgk(const real *f, real tau, real *out) { bgk(f, tau, out); }

/* (rho, u, f^neq) of one population vector */
static void macro_neq(const real *f, real *rho, real *ux, real *uy, real *neq)
{
    real feq[Q];
    moments(f, rho, ux, uy);
    equilibrium(*rho, *ux, *uy, feq);
    for (int i = 0; i < Q; ++i) neq[i] = f[i] - feq[i];
}

/* ------------------------------------------------------------------ */
/* structured levels                                                     */
/* ------------------------------------------------------------------ */

#define LIDX(lv, q, i, j) (((size_t)(q) * (size_t)(lv)->ny + (size_t)(j)) * (size_t)(lv)->nx + (size_t)(i))

static void get_node(const olevel *lv, const real *a, int i, int j, real *f)
{
    for (int q = 0; q < Q; ++q) f[q] = a[LIDX(lv, q, i, j)];
}

static void put_node(const olevel *lv, real *a, int i, int j, const real *f)
{
    for (int q = 0; q < Q; ++q) a[LIDX(lv, q, i, j)] = f[q];
}

static int inside_ellipse(const double *e, double x, double y)
{
    double dx = (x - e[0]) / e[2], dy = (y - e[1]) / e[3];
    return dx * dx + dy * dy < 1.0;
}

/* Crossing number of the ray from (x, y) towards +x with the polygon's edges;
 * an edge counts when exactly one of its end points has y' <= y.  Odd: inside. */
static int inside_polygon(int n, const double *xy, double x, double y)
{
    int crossings = 0;
    for (int e = 0; e < n; ++e) {
        const double *a = xy + 2 * e, *b = xy + 2 * ((e + 1) % n);
        int a_below = a[1] <= y, b_below = b[1] <= y;
        if (a_below == b_below) continue;
        double x_cross = a[0] + (y - a[1]) * (b[0] - a[0]) / (b[1] - a[1]);
        if (x < x_cross) crossings++;
    }
    return crossings % 2;
}

/* Node classes (Sec. 4): boxes covered by a finer box keep their boundary
 * nodes; the first ring inside receives the restricted fine values; the finest
 * level has an inactive region inside the inner ellipse whose nodes with an
 * active neighbour are the structured interpolation nodes. */
static void classify(oracle_t *o)
{
    for (int l = 0; l <= o->L; ++l) {
        olevel *lv = &o->lev[l];
        for (int j = 0; j < lv->ny; ++j)
            for (int i = 0; i < lv->nx; ++i) {
                uint8_t c = CL_ACTIVE;
                if (l > 0 && (i == 0 || j == 0 || i == lv->nx - 1 || j == lv->ny - 1)) c = CL_PERIM;
                if (l < o->L) {
                    int ci0 = o->lev[l + 1].i0, cj0 = o->lev[l + 1].j0;
                    int ci1 = ci0 + (o->lev[l + 1].nx - 1) / 2, cj1 = cj0 + (o->lev[l + 1].ny - 1) / 2;
                    if (i > ci0 && i < ci1 && j > cj0 && j < cj1) {
                        if (i == ci0 + 1 || i == ci1 - 1 || j == cj0 + 1 || j == cj1 - 1) c = CL_RING;
                        else c = CL_COVERED;
                    }
                }
                if (l == o->L && o->cfg.ein[2] > 0.0 && c == CL_ACTIVE) {
                    double x = lv->ox + i * lv->sp, y = lv->oy + j * lv->sp;
                    if (inside_ellipse(o->cfg.ein, x, y)) c = CL_INACTIVE;
                }
                if (l == o->L && o->cfg.body_n > 0 && c == CL_ACTIVE) {
                    double x = lv->ox + i * lv->sp, y = lv->oy + j * lv->sp;
                    if (inside_polygon(o->cfg.body_n, o->cfg.body_xy, x, y)) c = CL_SOLID;
                }
                lv->cls[(size_t)j * lv->nx + i] = c;
            }
        if (l == o->L) {
            for (int j = 1; j < lv->ny - 1; ++j)
                for (int i = 1; i < lv->nx - 1; ++i) {
                    if (lv->cls[(size_t)j * lv->nx + i] != CL_INACTIVE) continue;
                    for (int q = 1; q < Q; ++q) {
                        int a = i + CX[q], b = j + CY[q];
                        if (lv->cls[(size_t)b * lv->nx + a] == CL_ACTIVE) {
                            lv->cls[(size_t)j * lv->nx + i] = CL_INTERP;
                            break;
                        }
                    }
                }
        }
    }
}

/* ------------------------------------------------------------------ */
/* finite-volume geometry on the median dual (eq. (3), reading above)   */
/* ------------------------------------------------------------------ */

typedef struct { int k; real gx, gy, c; } nbr_t;

static void nb_add(nbr_t *row, int *len, int k, real gx, real gy, real c)
{
    for (int a = 0; a < *len; ++a)
        if (row[a].k == k) { row[a].gx += gx; row[a].gy += gy; row[a].c += c; return; }
    row[*len].k = k; row[*len].gx = gx; row[*len].gy = gy; row[*len].c = c;
    (*len)++;
}

static int cmp_nbr(const void *a, const void *b)
{
    return ((const nbr_t *)a)->k - ((const nbr_t *)b)->k;
}

static real wrap(real d, double period)
{
    if (period <= 0.0) return d;
    return d - period * floor(RE(d) / period + 0.5);
}

#define MAXNB 32

/* triangles incident to each node, in increasing triangle index */
static void node_triangles(int nn, int nt, const int32_t *tri, int **ptr_o, int **lst_o)
{
    int *ptr = (int *)calloc((size_t)nn + 1, sizeof(int));
    int *lst = (int *)malloc(sizeof(int) * 3 * (size_t)(nt > 0 ? nt : 1));
    for (int t = 0; t < 3 * nt; ++t) ptr[tri[t] + 1]++;
    for (int p = 0; p < nn; ++p) ptr[p + 1] += ptr[p];
    int *fill = (int *)calloc((size_t)nn, sizeof(int));
    for (int t = 0; t < nt; ++t)
        for (int r = 0; r < 3; ++r) { int p = tri[3 * t + r]; lst[ptr[p] + fill[p]++] = t; }
    free(fill);
    *ptr_o = ptr; *lst_o = lst;
}

/* Builds CSR rows (neighbours sorted by index, self included) of
 *   G_Pk = -(1/A_P) sum_segments N_seg psi_k(mid_seg),
 *   C_Pk =  (1/A_P) integral over CV_P of psi_k,
 * with N_seg the outward normal times length of each control-volume segment,
 * and the list of wall edges.  Returns 0 or a negative error. */
static int fv_geometry(int nn, int nt, const real *xy, const int32_t *tri, const uint8_t *kind,
                       const double *period, int **rowptr_o, int **col_o, real **gx_o,
                       real **gy_o, real **cc_o, real **area_o, int *n_wall_o, int **wedge_o,
                       char *err)
{
    nbr_t *rows = (nbr_t *)calloc((size_t)nn * MAXNB, sizeof(nbr_t));
    int *len = (int *)calloc((size_t)nn, sizeof(int));
    real *area = (real *)calloc((size_t)nn, sizeof(real));
    if (!rows || !len || !area) { snprintf(err, 256, "oom"); return -1; }
    for (int t = 0; t < nt; ++t) {
        int v[3] = {tri[3 * t], tri[3 * t + 1], tri[3 * t + 2]};
        for (int r = 0; r < 3; ++r) {
            int P = v[r], A = v[(r + 1) % 3], B = v[(r + 2) % 3];
            /* positions relative to P (minimum image on a periodic mesh) */
            real ax = wrap(xy[2 * A] - xy[2 * P], period[0]), ay = wrap(xy[2 * A + 1] - xy[2 * P + 1], period[1]);
            real bx = wrap(xy[2 * B] - xy[2 * P], period[0]), by = wrap(xy[2 * B + 1] - xy[2 * P + 1], period[1]);
            real at = 0.5 * (ax * by - ay * bx);
            if (!(RE(at) > 0.0)) { snprintf(err, 256, "triangle %d not counter-clockwise or degenerate", t); free(rows); free(len); free(area); return -2; }
            real mpa_x = 0.5 * ax, mpa_y = 0.5 * ay;
            real mpb_x = 0.5 * bx, mpb_y = 0.5 * by;
            real g_x = (ax + bx) / 3.0, g_y = (ay + by) / 3.0;
            /* segment M_PA -> G, outward normal = clockwise rotation of the segment */
            real s1x = g_x - mpa_x, s1y = g_y - mpa_y;
            real n1x = s1y, n1y = -s1x;
            /* segment G -> M_PB */
            real s2x = mpb_x - g_x, s2y = mpb_y - g_y;
            real n2x = s2y, n2y = -s2x;
            /* hat-function values at the segment midpoints: (P, A, B) */
            const double m1[3] = {5.0 / 12.0, 5.0 / 12.0, 1.0 / 6.0};
            const double m2[3] = {5.0 / 12.0, 1.0 / 6.0, 5.0 / 12.0};
            int ids[3] = {P, A, B};
            /* exact integrals of the hat functions over the quadrilateral P-M_PA-G-M_PB */
            const double ci[3] = {11.0 / 54.0, 7.0 / 108.0, 7.0 / 108.0};
            for (int s = 0; s < 3; ++s) {
                real gx = -(n1x * m1[s] + n2x * m2[s]);
                real gy = -(n1y * m1[s] + n2y * m2[s]);
                if (len[P] >= MAXNB) { snprintf(err, 256, "node %d degree too large", P); return -2; }
                nb_add(rows + (size_t)P * MAXNB, &len[P], ids[s], gx, gy, ci[s] * at);
            }
            area[P] += at / 3.0;
        }
    }
    /* boundary edges: a directed edge of a counter-clockwise triangle whose
     * reverse appears in no triangle; the fluid lies on its left. */
    int *n2t_ptr, *n2t;
    node_triangles(nn, nt, tri, &n2t_ptr, &n2t);
    int n_be = 0, cap = 1024;
    int *be = (int *)malloc(sizeof(int) * 2 * cap);
    for (int t = 0; t < nt; ++t) {
        for (int r = 0; r < 3; ++r) {
            int P = tri[3 * t + r], Qn = tri[3 * t + (r + 1) % 3];
            int found = 0;
            for (int a = n2t_ptr[P]; a < n2t_ptr[P + 1] && !found; ++a) {
                int u = n2t[a];
                if (u == t) continue;
                for (int s = 0; s < 3; ++s)
                    if (tri[3 * u + s] == Qn && tri[3 * u + (s + 1) % 3] == P) { found = 1; break; }
            }
            if (!found) {
                if (n_be == cap) { cap *= 2; be = (int *)realloc(be, sizeof(int) * 2 * cap); }
                be[2 * n_be] = P; be[2 * n_be + 1] = Qn; n_be++;
            }
        }
    }
    free(n2t_ptr); free(n2t);
    /* half boundary edges close the control volumes: P -> M_PQ for P with
     * weights (3/4, 1/4), M_PQ -> Q for Q with weights (1/4, 3/4). */
    int n_wall = 0;
    int *wedge = (int *)malloc(sizeof(int) * 2 * (n_be > 0 ? n_be : 1));
    for (int e = 0; e < n_be; ++e) {
        int P = be[2 * e], Qn = be[2 * e + 1];
        real dx = wrap(xy[2 * Qn] - xy[2 * P], period[0]), dy = wrap(xy[2 * Qn + 1] - xy[2 * P + 1], period[1]);
        real nx = 0.5 * dy, ny = -0.5 * dx;   /* each half edge: half length */
        nb_add(rows + (size_t)P * MAXNB, &len[P], P, -0.75 * nx, -0.75 * ny, 0.0);
        nb_add(rows + (size_t)P * MAXNB, &len[P], Qn, -0.25 * nx, -0.25 * ny, 0.0);
        nb_add(rows + (size_t)Qn * MAXNB, &len[Qn], Qn, -0.75 * nx, -0.75 * ny, 0.0);
        nb_add(rows + (size_t)Qn * MAXNB, &len[Qn], P, -0.25 * nx, -0.25 * ny, 0.0);
        if (kind && kind[P] == KIND_WALL && kind[Qn] == KIND_WALL) {
            wedge[2 * n_wall] = P; wedge[2 * n_wall + 1] = Qn; n_wall++;
        }
    }
    free(be);
    int *rowptr = (int *)malloc(sizeof(int) * (nn + 1));
    rowptr[0] = 0;
    for (int p = 0; p < nn; ++p) rowptr[p + 1] = rowptr[p] + len[p];
    int nnz = rowptr[nn];
    int *col = (int *)malloc(sizeof(int) * nnz);
    real *gx = (real *)malloc(sizeof(real) * nnz), *gy = (real *)malloc(sizeof(real) * nnz);
    real *cc = (real *)malloc(sizeof(real) * nnz);
    for (int p = 0; p < nn; ++p) {
        nbr_t *row = rows + (size_t)p * MAXNB;
        qsort(row, len[p], sizeof(nbr_t), cmp_nbr);
        if (!(RE(area[p]) > 0.0)) { snprintf(err, 256, "node %d has no control volume", p); return -2; }
        for (int a = 0; a < len[p]; ++a) {
            int z = rowptr[p] + a;
            col[z] = row[a].k;
            gx[z] = row[a].gx / area[p];
            gy[z] = row[a].gy / area[p];
            cc[z] = row[a].c / area[p];
        }
    }
    free(rows); free(len);
    *rowptr_o = rowptr; *col_o = col; *gx_o = gx; *gy_o = gy; *cc_o = cc; *area_o = area;
    *n_wall_o = n_wall; *wedge_o = wedge;
    return 0;
}

/* Stand-alone geometry export for tests: caller passes arrays of size >= nnz_max. */
int or_fv_geometry(int32_t nn, int32_t nt, const real *xy, const int32_t *tri, const uint8_t *kind,
                   double period_x, double period_y, int32_t nnz_max, int32_t *rowptr_out,
                   int32_t *col_out, real *gx_out, real *gy_out, real *c_out, real *area_out,
                   int32_t *n_wall_out, int32_t *wedge_out, int32_t wedge_max)
{
    char err[256];
    double period[2] = {period_x, period_y};
    int *rowptr, *col, *wedge, n_wall;
    real *gx, *gy, *cc, *area;
    int rc = fv_geometry(nn, nt, xy, tri, kind, period, &rowptr, &col, &gx, &gy, &cc, &area, &n_wall, &wedge, err);
    if (rc) return rc;
    int nnz = rowptr[nn];
    if (nnz > nnz_max || n_wall > wedge_max) rc = -1;
    else {
        for (int p = 0; p <= nn; ++p) rowptr_out[p] = rowptr[p];
        for (int z = 0; z < nnz; ++z) { col_out[z] = col[z]; gx_out[z] = gx[z]; gy_out[z] = gy[z]; c_out[z] = cc[z]; }
        for (int p = 0; p < nn; ++p) area_out[p] = area[p];
        for (int e = 0; e < 2 * n_wall; ++e) wedge_out[e] = wedge[e];
        *n_wall_out = n_wall;
    }
    free(rowptr); free(col); free(gx); free(gy); free(cc); free(area); free(wedge);
    return rc;
}

/* ------------------------------------------------------------------ */
/* interpolation stencils, eqs. (8) and (9)                              */
/* ------------------------------------------------------------------ */

/* barycentric coordinates of (x, y) in triangle t */
static void barycentric(const real *xy, const int32_t *tri, int t, double x, double y, real *lam)
{
    int a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
    real x1 = xy[2 * a], y1 = xy[2 * a + 1], x2 = xy[2 * b], y2 = xy[2 * b + 1], x3 = xy[2 * c], y3 = xy[2 * c + 1];
    real det = (x2 - x1) * (y3 - y1) - (x3 - x1) * (y2 - y1);
    lam[1] = ((x - x1) * (y3 - y1) - (x3 - x1) * (y - y1)) / det;
    lam[2] = ((x2 - x1) * (y - y1) - (x - x1) * (y2 - y1)) / det;
    lam[0] = 1.0 - lam[1] - lam[2];
}

/* Uniform bucket grid over the mesh; every triangle is listed (in increasing
 * index) in each bucket its bounding box overlaps. */
typedef struct {
    double x0, y0, h;
    int nbx, nby;
    int *ptr, *lst;
    int *n2t_ptr, *n2t;   /* triangles around each node */
} search_t;

static void search_build(int nn, int nt, const real *xy, const int32_t *tri, search_t *S)
{
    double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
    for (int p = 0; p < nn; ++p) {
        xmin = fmin(xmin, RE(xy[2 * p])); xmax = fmax(xmax, RE(xy[2 * p]));
        ymin = fmin(ymin, RE(xy[2 * p + 1])); ymax = fmax(ymax, RE(xy[2 * p + 1]));
    }
    double h = sqrt((xmax - xmin) * (ymax - ymin) / (nt > 0 ? nt : 1)) * 2.0;
    if (!(h > 0)) h = 1.0;
    S->x0 = xmin - 1e-6; S->y0 = ymin - 1e-6; S->h = h;
    S->nbx = (int)((xmax - S->x0) / h) + 1; S->nby = (int)((ymax - S->y0) / h) + 1;
    int nb = S->nbx * S->nby;
    int *cnt = (int *)calloc((size_t)nb + 1, sizeof(int));
    for (int pass = 0; pass < 2; ++pass) {
        for (int t = 0; t < nt; ++t) {
            int a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
            double bx0 = fmin(RE(xy[2 * a]), fmin(RE(xy[2 * b]), RE(xy[2 * c]))) - 1e-9, bx1 = fmax(RE(xy[2 * a]), fmax(RE(xy[2 * b]), RE(xy[2 * c]))) + 1e-9;
            double by0 = fmin(RE(xy[2 * a + 1]), fmin(RE(xy[2 * b + 1]), RE(xy[2 * c + 1]))) - 1e-9, by1 = fmax(RE(xy[2 * a + 1]), fmax(RE(xy[2 * b + 1]), RE(xy[2 * c + 1]))) + 1e-9;
            int i0 = (int)floor((bx0 - S->x0) / h), i1 = (int)floor((bx1 - S->x0) / h);
            int j0 = (int)floor((by0 - S->y0) / h), j1 = (int)floor((by1 - S->y0) / h);
            if (i0 < 0) i0 = 0;
            if (j0 < 0) j0 = 0;
            if (i1 >= S->nbx) i1 = S->nbx - 1;
            if (j1 >= S->nby) j1 = S->nby - 1;
            for (int j = j0; j <= j1; ++j)
                for (int i = i0; i <= i1; ++i) {
                    int bk = j * S->nbx + i;
                    if (pass == 0) cnt[bk + 1]++;
                    else S->lst[S->ptr[bk] + cnt[bk]++] = t;
                }
        }
        if (pass == 0) {
            for (int bk = 0; bk < nb; ++bk) cnt[bk + 1] += cnt[bk];
            S->ptr = cnt;
            S->lst = (int *)malloc(sizeof(int) * (size_t)(cnt[nb] > 0 ? cnt[nb] : 1));
            cnt = (int *)calloc((size_t)nb + 1, sizeof(int));
        }
    }
    free(cnt);
    node_triangles(nn, nt, tri, &S->n2t_ptr, &S->n2t);
}

static void search_free(search_t *S)
{
    free(S->ptr); free(S->lst); free(S->n2t_ptr); free(S->n2t);
}

/* Point location: every triangle whose barycentric coordinates at (x, y) are
 * all >= -1e-12 (one inside a triangle, two on an edge, more at a vertex), in
 * increasing index.  Returns the count (at most cap). */
static int locate_all(const search_t *S, const real *xy, const int32_t *tri, double x, double y,
                      int *ts, real *lams, int cap)
{
    int i = (int)floor((x - S->x0) / S->h), j = (int)floor((y - S->y0) / S->h);
    if (i < 0 || j < 0 || i >= S->nbx || j >= S->nby) return 0;
    int bk = j * S->nbx + i, n = 0;
    for (int a = S->ptr[bk]; a < S->ptr[bk + 1] && n < cap; ++a) {
        int t = S->lst[a];
        real lam[3];
        barycentric(xy, tri, t, x, y, lam);
        if (RE(lam[0]) >= -1e-12 && RE(lam[1]) >= -1e-12 && RE(lam[2]) >= -1e-12) {
            ts[n] = t;
            lams[3 * n] = lam[0]; lams[3 * n + 1] = lam[1]; lams[3 * n + 2] = lam[2];
            n++;
        }
    }
    return n;
}

/* third vertex of the triangle other than t that shares edge (a, b); -1 if none */
static int opposite_vertex(const search_t *S, const int32_t *tri, int t, int a, int b)
{
    for (int z = S->n2t_ptr[a]; z < S->n2t_ptr[a + 1]; ++z) {
        int u = S->n2t[z];
        if (u == t) continue;
        int has_b = 0, other = -1;
        for (int s = 0; s < 3; ++s) {
            int v = tri[3 * u + s];
            if (v == b) has_b = 1;
            else if (v != a) other = v;
        }
        if (has_b) return other;
    }
    return -1;
}

/* Solve the n x n system M w = rhs by Gaussian elimination with partial
 * pivoting.  Returns 0, or -1 when a pivot falls below tol * max|M|. */
static int solve_dense(int n, real *M, real *rhs, double tol)
{
    double mx = 0.0;
    for (int a = 0; a < n * n; ++a) mx = fmax(mx, fabs(RE(M[a])));
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int r = k + 1; r < n; ++r) if (fabs(RE(M[r * n + k])) > fabs(RE(M[p * n + k]))) p = r;
        if (fabs(RE(M[p * n + k])) < tol * mx) return -1;
        if (p != k) {
            for (int c = 0; c < n; ++c) { real tmp = M[k * n + c]; M[k * n + c] = M[p * n + c]; M[p * n + c] = tmp; }
            real tmp = rhs[k]; rhs[k] = rhs[p]; rhs[p] = tmp;
        }
        for (int r = k + 1; r < n; ++r) {
            real fct = M[r * n + k] / M[k * n + k];
            for (int c = k; c < n; ++c) M[r * n + c] -= fct * M[k * n + c];
            rhs[r] -= fct * rhs[k];
        }
    }
    for (int k = n - 1; k >= 0; --k) {
        real s = rhs[k];
        for (int c = k + 1; c < n; ++c) s -= M[k * n + c] * rhs[c];
        rhs[k] = s / M[k * n + k];
    }
    return 0;
}

/* Six-node quadratic interpolation of eq. (8) for one triangle t: its three
 * vertices and the opposite vertices of its three edge neighbours.  The
 * weights reproduce 1, x, y, x^2, xy, y^2 exactly at (x, y).  Falls back to the
 * barycentric weights (linear) when a neighbour is missing or the system is
 * singular, or when linear interpolation is asked for.  Returns 6 or 3. */
static int stencil_tri(const search_t *S, const real *xy, const int32_t *tri, int t, const real *lam,
                       double x, double y, int linear, int *don, real *w, int *fallback)
{
    int v0 = tri[3 * t], v1 = tri[3 * t + 1], v2 = tri[3 * t + 2];
    if (!linear) {
        int o01 = opposite_vertex(S, tri, t, v0, v1);
        int o12 = opposite_vertex(S, tri, t, v1, v2);
        int o20 = opposite_vertex(S, tri, t, v2, v0);
        if (o01 >= 0 && o12 >= 0 && o20 >= 0) {
            int nodes[6] = {v0, v1, v2, o01, o12, o20};
            real ax = xy[2 * v1] - xy[2 * v0], ay = xy[2 * v1 + 1] - xy[2 * v0 + 1];
            real bx = xy[2 * v2] - xy[2 * v0], by = xy[2 * v2 + 1] - xy[2 * v0 + 1];
            real h = sqrt(ABS_A(ax * by - ay * bx));   /* sqrt(2 * area) */
            real M[36], rhs[6] = {1, 0, 0, 0, 0, 0};
            for (int k = 0; k < 6; ++k) {
                real xi = (xy[2 * nodes[k]] - x) / h, eta = (xy[2 * nodes[k] + 1] - y) / h;
                M[0 * 6 + k] = 1.0;
                M[1 * 6 + k] = xi;
                M[2 * 6 + k] = eta;
                M[3 * 6 + k] = xi * xi;
                M[4 * 6 + k] = xi * eta;
                M[5 * 6 + k] = eta * eta;
            }
            if (solve_dense(6, M, rhs, 1e-10) == 0) {
                for (int k = 0; k < 6; ++k) { don[k] = nodes[k]; w[k] = rhs[k]; }
                return 6;
            }
        }
        *fallback = 1;
    }
    don[0] = v0; don[1] = v1; don[2] = v2;
    w[0] = lam[0]; w[1] = lam[1]; w[2] = lam[2];
    return 3;
}

#define SDON 8   /* donors of a structured interpolation node */

/* Interpolation weights at (x, y) from the mesh.  A point on a mesh node takes
 * that node; a point inside one triangle takes its stencil; a point on an edge
 * shared by two triangles takes the mean of the two stencils (any of them
 * reproduces quadratics, and the mean keeps mirror-symmetric meshes
 * symmetric).  Returns the donor count (<= SDON) or -1 outside the mesh. */
static int stencil_mesh(const search_t *S, const real *xy, const int32_t *tri, double x, double y,
                        int linear, int *don, real *w, int *fallback)
{
    int ts[8];
    real lams[24];
    int nt = locate_all(S, xy, tri, x, y, ts, lams, 8);
    *fallback = 0;
    if (nt == 0) return -1;
    for (int r = 0; r < 3; ++r)
        if (RE(lams[r]) >= 1.0 - 1e-12) { don[0] = tri[3 * ts[0] + r]; w[0] = 1.0; return 1; }
    if (nt > 2) return -1;
    int n = 0;
    for (int a = 0; a < nt; ++a) {
        int d[6];
        real wt[6];
        int nd = stencil_tri(S, xy, tri, ts[a], lams + 3 * a, x, y, linear, d, wt, fallback);
        for (int k = 0; k < nd; ++k) {
            int found = -1;
            for (int b = 0; b < n; ++b) if (don[b] == d[k]) { found = b; break; }
            if (found < 0) { don[n] = d[k]; w[n] = 0.0; found = n++; }
            w[found] += wt[k] / nt;
        }
    }
    return n;
}

int or_stencil6(int32_t nn, int32_t nt, const real *xy, const int32_t *tri, double x, double y, int32_t linear,
                int32_t *don, real *w)
{
    int fb, d[SDON];
    search_t S;
    search_build(nn, nt, xy, tri, &S);
    int n = stencil_mesh(&S, xy, tri, x, y, linear, d, w, &fb);
    search_free(&S);
    for (int k = 0; k < (n > 0 ? n : 0); ++k) don[k] = d[k];
    return n;
}

/* Nine-node interpolation of eq. (9) on the 3 x 3 block of unit-spaced nodes
 * centred on the nearest node: tensor product of the quadratic Lagrange
 * polynomials through offsets -1, 0, 1.  Linear: the four nodes of the cell.
 * (x, y) relative to the grid origin, unit spacing.  Outputs node offsets. */
static int stencil9(real x, real y, int linear, int *di, int *dj, real *w)
{
    if (!linear) {
        int i = (int)floor(RE(x) + 0.5), j = (int)floor(RE(y) + 0.5);
        real s = x - i, t = y - j;
        real ls[3] = {0.5 * s * (s - 1.0), 1.0 - s * s, 0.5 * s * (s + 1.0)};
        real lt[3] = {0.5 * t * (t - 1.0), 1.0 - t * t, 0.5 * t * (t + 1.0)};
        int k = 0;
        for (int b = 0; b < 3; ++b)
            for (int a = 0; a < 3; ++a) {
                di[k] = i + a - 1; dj[k] = j + b - 1; w[k] = ls[a] * lt[b]; k++;
            }
        return 9;
    }
    int i = (int)floor(RE(x)), j = (int)floor(RE(y));
    real s = x - i, t = y - j;
    di[0] = i; dj[0] = j; w[0] = (1 - s) * (1 - t);
    di[1] = i + 1; dj[1] = j; w[1] = s * (1 - t);
    di[2] = i; dj[2] = j + 1; w[2] = (1 - s) * t;
    di[3] = i + 1; dj[3] = j + 1; w[3] = s * t;
    return 4;
}

int or_stencil9(double x, double y, int32_t linear, int32_t *di, int32_t *dj, real *w)
{
    int a[9], b[9];
    int n = stencil9(x, y, linear, a, b, w);
    for (int k = 0; k < n; ++k) { di[k] = a[k]; dj[k] = b[k]; }
    return n;
}

/* ------------------------------------------------------------------ */
/* creation                                                              */
/* ------------------------------------------------------------------ */

void or_destroy(void *h);

static int default_nsub(real tau_u)
{
    int n = (int)ceil(1.0 / RE(tau_u));
    return n > 10 ? n : 10;
}

void *or_create(const or_cfg *cfg, char *err_out, int32_t err_len)
{
    oracle_t *o = (oracle_t *)calloc(1, sizeof(oracle_t));
    o->cfg = *cfg;
    o->L = cfg->nx_cells > 0 ? cfg->n_refine : 0;
    o->tau_u = cfg->tau_s - 0.5;
    o->n_sub = cfg->n_sub > 0 ? cfg->n_sub : default_nsub(o->tau_u);
#define FAIL(...) do { snprintf(o->err, 256, __VA_ARGS__); if (err_out) snprintf(err_out, err_len, "%s", o->err); or_destroy(o); return NULL; } while (0)
    if (!(RE(cfg->tau_s) > 0.5)) FAIL("tau_s must exceed 1/2");
    if (cfg->n_refine < 0 || cfg->n_refine > 3) FAIL("n_refine out of range");
    if (cfg->nx_cells > 0) {
        int L = o->L, base_sp = 1 << L;
        olevel *b = &o->lev[0];
        b->nx = cfg->nx_cells + (cfg->periodic ? 0 : 1);
        b->ny = cfg->ny_cells + (cfg->periodic ? 0 : 1);
        b->sp = base_sp; b->ox = 0; b->oy = 0;
        for (int l = 1; l <= L; ++l) {
            olevel *lv = &o->lev[l], *pa = &o->lev[l - 1];
            lv->i0 = cfg->patch_i0[l - 1]; lv->j0 = cfg->patch_j0[l - 1];
            if (cfg->patch_nx[l - 1] % 2 || cfg->patch_ny[l - 1] % 2) FAIL("box sizes must be even");
            lv->nx = cfg->patch_nx[l - 1] + 1; lv->ny = cfg->patch_ny[l - 1] + 1;
            lv->sp = pa->sp / 2;
            lv->ox = pa->ox + lv->i0 * pa->sp; lv->oy = pa->oy + lv->j0 * pa->sp;
            int ci1 = lv->i0 + (lv->nx - 1) / 2, cj1 = lv->j0 + (lv->ny - 1) / 2;
            if (lv->i0 < 2 || lv->j0 < 2 || ci1 > pa->nx - 3 || cj1 > pa->ny - 3)
                FAIL("box %d does not fit inside its parent with a two-node margin", l);
        }
        /* acoustic scaling: tau_l - 1/2 = (tau_s - 1/2) / 2^(L - l) */
        for (int l = 0; l <= L; ++l) {
            o->lev[l].tau = 0.5 + (cfg->tau_s - 0.5) / (real)(1 << (L - l));
            if (!(RE(o->lev[l].tau) > 0.5)) FAIL("tau <= 1/2 on level %d", l);
            size_t n = (size_t)o->lev[l].nx * o->lev[l].ny;
            o->lev[l].cls = (uint8_t *)calloc(n, 1);
            o->lev[l].f = (real *)malloc(sizeof(real) * Q * n);
            o->lev[l].post = (real *)malloc(sizeof(real) * Q * n);
            o->lev[l].save = (real *)malloc(sizeof(real) * Q * n);
            if (!o->lev[l].f || !o->lev[l].post || !o->lev[l].save) FAIL("oom");
        }
        classify(o);
        if (cfg->body_n > 0) {
            /* every solid node is surrounded by active or solid nodes of the level */
            olevel *fl = &o->lev[L];
            int per = L == 0 && cfg->periodic, nsolid = 0;
            if (cfg->n_nodes > 0 || cfg->ein[2] > 0.0) FAIL("a body resolved by bounce-back excludes a mesh");
            for (int j = 0; j < fl->ny; ++j)
                for (int i = 0; i < fl->nx; ++i) {
                    if (fl->cls[(size_t)j * fl->nx + i] != CL_SOLID) continue;
                    nsolid++;
                    for (int q = 1; q < Q; ++q) {
                        int a = i + CX[q], b = j + CY[q];
                        if (per) { a = (a + fl->nx) % fl->nx; b = (b + fl->ny) % fl->ny; }
                        else if (a < 1 || b < 1 || a > fl->nx - 2 || b > fl->ny - 2)
                            FAIL("the body touches the edge of the finest level");
                        uint8_t c = fl->cls[(size_t)b * fl->nx + a];
                        if (c != CL_ACTIVE && c != CL_SOLID) FAIL("the body touches a box boundary");
                    }
                }
            if (nsolid == 0) FAIL("the body covers no node of the finest level");
        }
    }
    /* mesh */
    o->nn = cfg->n_nodes; o->nt = cfg->n_tris;
    if (o->nn > 0) {
        o->xy = (real *)malloc(sizeof(real) * 2 * o->nn);
        o->tri = (int32_t *)malloc(sizeof(int32_t) * 3 * o->nt);
        o->kind = (uint8_t *)malloc(o->nn);
        memcpy(o->xy, cfg->xy, sizeof(real) * 2 * o->nn);
        memcpy(o->tri, cfg->tri, sizeof(int32_t) * 3 * o->nt);
        memcpy(o->kind, cfg->kind, o->nn);
        for (int t = 0; t < 3 * o->nt; ++t)
            if (o->tri[t] < 0 || o->tri[t] >= o->nn) FAIL("triangle index out of range");
        int rc = fv_geometry(o->nn, o->nt, o->xy, o->tri, o->kind, cfg->mesh_period, &o->rowptr, &o->col,
                             &o->gx, &o->gy, &o->cc, &o->area, &o->n_wall_edges, &o->wedge, o->err);
        if (rc) FAIL("%s", o->err);
        o->fu = (real *)malloc(sizeof(real) * Q * o->nn);
        o->fu_new = (real *)malloc(sizeof(real) * Q * o->nn);
        o->uint_slot = (int *)malloc(sizeof(int) * o->nn);
        int nu = 0;
        for (int p = 0; p < o->nn; ++p) o->uint_slot[p] = o->kind[p] == KIND_INTERP ? nu++ : -1;
        o->n_uint = nu;
        o->uint_node = (int *)malloc(sizeof(int) * (nu > 0 ? nu : 1));
        for (int p = 0; p < o->nn; ++p) if (o->uint_slot[p] >= 0) o->uint_node[o->uint_slot[p]] = p;
    }
    /* coupling stencils (only with both a structured grid and a mesh) */
    if (cfg->nx_cells > 0 && o->nn > 0) {
        olevel *fl = &o->lev[o->L];
        int linear = cfg->interp == 1;
        /* structured interpolation nodes <- mesh, eq. (8) */
        int ns = 0;
        for (size_t a = 0; a < (size_t)fl->nx * fl->ny; ++a) ns += fl->cls[a] == CL_INTERP;
        o->n_sint = ns;
        o->sint_ij = (int *)malloc(sizeof(int) * 2 * (ns > 0 ? ns : 1));
        o->sint_don = (int *)malloc(sizeof(int) * SDON * (ns > 0 ? ns : 1));
        o->sint_w = (real *)malloc(sizeof(real) * SDON * (ns > 0 ? ns : 1));
        int k = 0;
        search_t S;
        search_build(o->nn, o->nt, o->xy, o->tri, &S);
        for (int j = 0; j < fl->ny; ++j)
            for (int i = 0; i < fl->nx; ++i) {
                if (fl->cls[(size_t)j * fl->nx + i] != CL_INTERP) continue;
                double x = fl->ox + i * fl->sp, y = fl->oy + j * fl->sp;
                int don[SDON];
                real w[SDON];
                int fb = 0;
                int nd = stencil_mesh(&S, o->xy, o->tri, x, y, linear, don, w, &fb);
                if (nd < 0) { search_free(&S); FAIL("structured interpolation node (%d,%d) lies outside the mesh", i, j); }
                o->n_fallback += fb;
                o->sint_ij[2 * k] = i; o->sint_ij[2 * k + 1] = j;
                for (int d = 0; d < SDON; ++d) {
                    o->sint_don[SDON * k + d] = d < nd ? don[d] : -1;
                    o->sint_w[SDON * k + d] = d < nd ? w[d] : 0.0;
                }
                k++;
            }
        search_free(&S);
        /* mesh interpolation nodes <- finest level, eq. (9) */
        o->uint_don = (int *)malloc(sizeof(int) * 9 * (o->n_uint > 0 ? o->n_uint : 1));
        o->uint_w = (real *)malloc(sizeof(real) * 9 * (o->n_uint > 0 ? o->n_uint : 1));
        for (int s = 0; s < o->n_uint; ++s) {
            int p = o->uint_node[s];
            int di[9], dj[9];
            real w[9];
            int nd = stencil9(o->xy[2 * p] - fl->ox, o->xy[2 * p + 1] - fl->oy, linear, di, dj, w);
            for (int d = 0; d < 9; ++d) {
                if (d < nd) {
                    if (di[d] < 1 || dj[d] < 1 || di[d] > fl->nx - 2 || dj[d] > fl->ny - 2 ||
                        fl->cls[(size_t)dj[d] * fl->nx + di[d]] != CL_ACTIVE)
                        FAIL("mesh interpolation node %d has a donor that is not an active structured node", p);
                    o->uint_don[9 * s + d] = di[d] + fl->nx * dj[d];
                    o->uint_w[9 * s + d] = w[d];
                } else {
                    o->uint_don[9 * s + d] = -1;
                    o->uint_w[9 * s + d] = 0.0;
                }
            }
        }
    } else if (cfg->nx_cells > 0 && cfg->ein[2] > 0.0) {
        FAIL("an inactive region needs a mesh");
    }
    /* initial state: f^eq(rho0, u_inf) everywhere, f^eq(rho0, 0) at wall nodes */
    real ux = cfg->u_inf * cos(cfg->aoa), uy = cfg->u_inf * sin(cfg->aoa);
    real feq[Q], feq0[Q];
    equilibrium(cfg->rho0, ux, uy, feq);
    equilibrium(cfg->rho0, 0.0, 0.0, feq0);
    for (int l = 0; cfg->nx_cells > 0 && l <= o->L; ++l) {
        olevel *lv = &o->lev[l];
        size_t plane = (size_t)lv->nx * lv->ny;
        for (int q = 0; q < Q; ++q)       /* one population plane at a time */
            for (size_t a = 0; a < plane; ++a) {
                lv->f[q * plane + a] = feq[q];
                lv->post[q * plane + a] = feq[q];
                lv->save[q * plane + a] = feq[q];
            }
    }
    for (int p = 0; p < o->nn; ++p)
        for (int q = 0; q < Q; ++q)
            o->fu[(size_t)q * o->nn + p] = (o->kind[p] == KIND_WALL && cfg->wall_bc) ? feq0[q] : feq[q];
    o->hist_cap = 1024;
    o->cd = (real *)malloc(sizeof(real) * o->hist_cap);
    o->cl = (real *)malloc(sizeof(real) * o->hist_cap);
    return o;
#undef FAIL
}

void or_destroy(void *h)
{
    oracle_t *o = (oracle_t *)h;
    if (!o) return;
    for (int l = 0; l < 4; ++l) { free(o->lev[l].cls); free(o->lev[l].f); free(o->lev[l].post); free(o->lev[l].save); }
    free(o->xy); free(o->tri); free(o->kind); free(o->rowptr); free(o->col); free(o->gx); free(o->gy);
    free(o->cc); free(o->area); free(o->wedge); free(o->fu); free(o->fu_new);
    free(o->sint_ij); free(o->sint_don); free(o->sint_w); free(o->uint_node); free(o->uint_slot);
    free(o->uint_don); free(o->uint_w); free(o->cd); free(o->cl);
    free(o->ws_sum); free(o->ws_tmp);
    free(o);
}

/* ------------------------------------------------------------------ */
/* one structured step                                                   */
/* ------------------------------------------------------------------ */

static void mesh_advance(oracle_t *o);
static void record_forces(oracle_t *o);

/* Coarse -> fine interface (Sec. 4, Filippova-Haenel): the fine perimeter
 * gets the coarse (rho, u, f^neq), linear in time at theta and linear in
 * space at odd fine nodes; f^neq is rescaled by tau_f / (2 tau_c) to the fine
 * pre-collision value, which is then collided at tau_f. */
static void coarse_to_fine(oracle_t *o, int l, double theta)
{
    olevel *pa = &o->lev[l], *ch = &o->lev[l + 1];
    real scale = plant[2] * ch->tau / (2.0 * pa->tau);
    for (int jc = 0; jc < ch->ny; ++jc)
        for (int ic = 0; ic < ch->nx; ++ic) {
            if (ch->cls[(size_t)jc * ch->nx + ic] != CL_PERIM) continue;
            int pi[2], pj[2], np = 1;
            if (ic % 2 == 0 && jc % 2 == 0) { pi[0] = ch->i0 + ic / 2; pj[0] = ch->j0 + jc / 2; }
            else if (ic % 2 == 1) { pi[0] = ch->i0 + (ic - 1) / 2; pi[1] = pi[0] + 1; pj[0] = pj[1] = ch->j0 + jc / 2; np = 2; }
            else { pj[0] = ch->j0 + (jc - 1) / 2; pj[1] = pj[0] + 1; pi[0] = pi[1] = ch->i0 + ic / 2; np = 2; }
            real rho = 0, ux = 0, uy = 0, neq[Q] = {0};
            for (int a = 0; a < np; ++a) {
                real f0[Q], f1[Q], r0, x0, y0, n0[Q], r1, x1, y1, n1[Q];
                get_node(pa, pa->save, pi[a], pj[a], f0);
                get_node(pa, pa->f, pi[a], pj[a], f1);
                macro_neq(f0, &r0, &x0, &y0, n0);
                macro_neq(f1, &r1, &x1, &y1, n1);
                real wa = 1.0 / np;
                rho += wa * ((1.0 - theta) * r0 + theta * r1);
                ux += wa * ((1.0 - theta) * x0 + theta * x1);
                uy += wa * ((1.0 - theta) * y0 + theta * y1);
                for (int q = 0; q < Q; ++q) neq[q] += wa * ((1.0 - theta) * n0[q] + theta * n1[q]);
            }
            real feq[Q], pre[Q], post[Q];
            equilibrium(rho, ux, uy, feq);
            for (int q = 0; q < Q; ++q) pre[q] = feq[q] + scale * neq[q];
            for (int q = 0; q < Q; ++q) post[q] = pre[q] - (pre[q] - feq[q]) / ch->tau;
            put_node(ch, ch->post, ic, jc, post);
        }
}

/* Fine -> coarse (Sec. 4): coarse nodes on the first ring inside the box get
 * the fine (rho, u) and the fine f^neq rescaled by 2 tau_c / tau_f, collided
 * at tau_c.  With f2c_filter the f^neq is first averaged over the 3 x 3 fine
 * nodes around the coincident one with full-weighting weights
 * (2 - |di|)(2 - |dj|) / 16, which sum to one and reproduce fields linear in
 * space; (rho, u) stay those of the coincident node. */
static void fine_to_coarse(oracle_t *o, int l)
{
    olevel *pa = &o->lev[l], *ch = &o->lev[l + 1];
    real scale = plant[3] * 2.0 * pa->tau / ch->tau;
    for (int j = 0; j < pa->ny; ++j)
        for (int i = 0; i < pa->nx; ++i) {
            if (pa->cls[(size_t)j * pa->nx + i] != CL_RING) continue;
            real f[Q], rho, ux, uy, neq[Q], feq[Q], pre[Q], post[Q];
            const int fi = 2 * (i - ch->i0), fj = 2 * (j - ch->j0);
            get_node(ch, ch->f, fi, fj, f);
            macro_neq(f, &rho, &ux, &uy, neq);
            if (o->cfg.f2c_filter) {
                for (int q = 0; q < Q; ++q) neq[q] = 0.0;
                for (int dj = -1; dj <= 1; ++dj)
                    for (int di = -1; di <= 1; ++di) {
                        real g[Q], r2, x2, y2, n2[Q];
                        const double w = (2 - abs(di)) * (2 - abs(dj)) / 16.0;
                        get_node(ch, ch->f, fi + di, fj + dj, g);
                        macro_neq(g, &r2, &x2, &y2, n2);
                        for (int q = 0; q < Q; ++q) neq[q] += w * n2[q];
                    }
            }
            equilibrium(rho, ux, uy, feq);
            for (int q = 0; q < Q; ++q) pre[q] = feq[q] + scale * neq[q];
            for (int q = 0; q < Q; ++q) post[q] = pre[q] - (pre[q] - feq[q]) / pa->tau;
            put_node(pa, pa->post, i, j, post);
        }
}

/* Structured interpolation nodes, eq. (4): f~ = f^eq(rho, u) +
 * 2 (tau_s - 1) / (2 tau_s - 1) f^neq, with rho, u and f^neq interpolated from
 * the mesh state at time t (eq. (8)). */
static void mesh_to_structured(oracle_t *o)
{
    olevel *fl = &o->lev[o->L];
    real ts = fl->tau;
    real factor = plant[0] * 2.0 * (ts - 1.0) / (2.0 * ts - 1.0);
    for (int s = 0; s < o->n_sint; ++s) {
        real rho = 0, ux = 0, uy = 0, neq[Q] = {0};
        for (int d = 0; d < SDON; ++d) {
            int k = o->sint_don[SDON * s + d];
            if (k < 0) continue;
            real f[Q], r, x, y, n[Q];
            for (int q = 0; q < Q; ++q) f[q] = o->fu[(size_t)q * o->nn + k];
            macro_neq(f, &r, &x, &y, n);
            real w = o->sint_w[SDON * s + d];
            rho += w * r; ux += w * x; uy += w * y;
            for (int q = 0; q < Q; ++q) neq[q] += w * n[q];
        }
        real feq[Q], post[Q];
        equilibrium(rho, ux, uy, feq);
        for (int q = 0; q < Q; ++q) post[q] = feq[q] + factor * neq[q];
        put_node(fl, fl->post, o->sint_ij[2 * s], o->sint_ij[2 * s + 1], post);
    }
}

/* Far-field conditions on the base level (Sec. 4), applied to the streamed
 * populations: top and bottom copy the inner neighbour; then inlet and outlet
 * columns (corners included) use non-equilibrium extrapolation. */
static void farfield(oracle_t *o)
{
    olevel *b = &o->lev[0];
    int nx = b->nx, ny = b->ny;
    real f[Q];
    if (!o->cfg.channel) {
        for (int i = 1; i < nx - 1; ++i) {
            get_node(b, b->f, i, 1, f); put_node(b, b->f, i, 0, f);
            get_node(b, b->f, i, ny - 2, f); put_node(b, b->f, i, ny - 1, f);
        }
    } else {
        /* no-slip walls: u = 0, rho and f^neq from the inner neighbour */
        for (int i = 1; i < nx - 1; ++i) {
            for (int side = 0; side < 2; ++side) {
                int jb = side ? ny - 1 : 0, jn = side ? ny - 2 : 1;
                real rho, ux, uy, neq[Q], feq[Q], out[Q];
                get_node(b, b->f, i, jn, f);
                macro_neq(f, &rho, &ux, &uy, neq);
                equilibrium(rho, 0.0, 0.0, feq);
                for (int q = 0; q < Q; ++q) out[q] = feq[q] + neq[q];
                put_node(b, b->f, i, jb, out);
            }
        }
    }
    real uinx = o->cfg.u_inf * cos(o->cfg.aoa), uiny = o->cfg.u_inf * sin(o->cfg.aoa);
    for (int j = 0; j < ny; ++j) {
        real fn[Q], rho, ux, uy, neq[Q], feq[Q], out[Q];
        /* inlet: u given, rho from the neighbour */
        get_node(b, b->f, 1, j, fn);
        macro_neq(fn, &rho, &ux, &uy, neq);
        real ui = uinx, vi = uiny;
        if (o->cfg.channel) {
            real H = ny - 1.0, y = j;
            ui = 4.0 * o->cfg.u_inf * y * (H - y) / (H * H);
            vi = 0.0;
        }
        equilibrium(rho, ui, vi, feq);
        for (int q = 0; q < Q; ++q) out[q] = feq[q] + neq[q];
        put_node(b, b->f, 0, j, out);
        /* outlet: rho given, u from the neighbour */
        get_node(b, b->f, nx - 2, j, fn);
        macro_neq(fn, &rho, &ux, &uy, neq);
        equilibrium(o->cfg.rho0, ux, uy, feq);
        for (int q = 0; q < Q; ++q) out[q] = feq[q] + neq[q];
        put_node(b, b->f, nx - 1, j, out);
    }
}

/* Advance level l by one of its own time steps (2^(L-l) finest steps). */
static void level_step(oracle_t *o, int l)
{
    olevel *lv = &o->lev[l];
    int nx = lv->nx, ny = lv->ny;
    int periodic = (l == 0 && o->cfg.periodic);
    memcpy(lv->save, lv->f, sizeof(real) * Q * nx * ny);
    /* 1. BGK collision of the active nodes, eq. (1) */
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            if (lv->cls[(size_t)j * nx + i] != CL_ACTIVE) continue;
            real f[Q], out[Q];
            get_node(lv, lv->f, i, j, f);
            bgk(f, lv->tau, out);
            put_node(lv, lv->post, i, j, out);
        }
    /* 2. restriction from the finer box onto the ring */
    if (l < o->L) fine_to_coarse(o, l);
    /* 3. structured interpolation nodes from the mesh at time t, eq. (4) */
    if (l == o->L && o->n_sint > 0) mesh_to_structured(o);
    /* 4. streaming: f_i(x, t+1) = f~_i(x - c_i, t) */
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            if (lv->cls[(size_t)j * nx + i] != CL_ACTIVE) continue;
            if (!periodic && l == 0 && (i == 0 || j == 0 || i == nx - 1 || j == ny - 1)) continue;
            for (int q = 0; q < Q; ++q) {
                int a = i - CX[q], b = j - CY[q];
                if (periodic) { a = (a + nx) % nx; b = (b + ny) % ny; }
                if (lv->cls[(size_t)b * nx + a] == CL_SOLID) {
                    /* halfway bounce-back: what left (i, j) towards the body returns */
                    int back = plant[7] != 0.0 ? OPPOSITE[q] : q;
                    lv->f[LIDX(lv, q, i, j)] = lv->post[LIDX(lv, back, i, j)];
                } else {
                    lv->f[LIDX(lv, q, i, j)] = lv->post[LIDX(lv, q, a, b)];
                }
            }
        }
    /* 5. far field on the base level */
    if (l == 0 && !periodic) farfield(o);
    /* 6. the finer box takes two steps, then the mesh when this is the finest level */
    if (l < o->L) {
        for (int s = 0; s < 2; ++s) {
            coarse_to_fine(o, l, 0.5 * s);
            level_step(o, l + 1);
        }
    } else {
        if (o->nn > 0) {
            mesh_advance(o);
            record_forces(o);
        } else {
            record_forces(o);
        }
    }
}

/* ------------------------------------------------------------------ */
/* mesh: n finite-volume sub-steps per finest step                       */
/* ------------------------------------------------------------------ */

/* (rho, u, f^neq) at the mesh interpolation nodes from a finest-level array, eq. (9) */
static void structured_to_mesh(oracle_t *o, const real *src, real *out /* [12 * n_uint] */)
{
    olevel *fl = &o->lev[o->L];
    for (int s = 0; s < o->n_uint; ++s) {
        real rho = 0, ux = 0, uy = 0, neq[Q] = {0};
        for (int d = 0; d < 9; ++d) {
            int node = o->uint_don[9 * s + d];
            if (node < 0) continue;
            int i = node % fl->nx, j = node / fl->nx;
            real f[Q], r, x, y, n[Q];
            get_node(fl, src, i, j, f);
            macro_neq(f, &r, &x, &y, n);
            real w = o->uint_w[9 * s + d];
            rho += w * r; ux += w * x; uy += w * y;
            for (int q = 0; q < Q; ++q) neq[q] += w * n[q];
        }
        out[12 * s + 0] = rho; out[12 * s + 1] = ux; out[12 * s + 2] = uy;
        for (int q = 0; q < Q; ++q) out[12 * s + 3 + q] = neq[q];
    }
}

/* One sub-step of eq. (3) on every mesh node, eq. (5) at interpolation
 * nodes.  star[] holds, for interpolation nodes, f* = f^eq,s + (1 - 1/(2 tau_s))
 * f^neq,s and nstar[] its non-equilibrium part (eq. (6)); every other node
 * contributes its stored value (eq. (7)). */
static void fv_substep(oracle_t *o, const real *star, const real *nstar)
{
    int nn = o->nn;
    double dt = 1.0 / o->n_sub;
    real tau_u = o->tau_u;
    real *neq_u = (real *)malloc(sizeof(real) * Q * nn);
    /* non-equilibrium part of every stored mesh value */
#pragma omp parallel for schedule(static)
    for (int p = 0; p < nn; ++p) {
        real f[Q], r, x, y, n[Q];
        for (int q = 0; q < Q; ++q) f[q] = o->fu[(size_t)q * nn + p];
        macro_neq(f, &r, &x, &y, n);
        for (int q = 0; q < Q; ++q) neq_u[(size_t)q * nn + p] = n[q];
    }
#pragma omp parallel for schedule(static)
    for (int p = 0; p < nn; ++p) {
        int sp = o->uint_slot[p];
        int use_star = sp >= 0 && star != NULL;
        real fnew[Q];
        for (int q = 0; q < Q; ++q) {
            real base = use_star ? star[Q * sp + q] : o->fu[(size_t)q * nn + p];
            real sum_s = 0.0, sum_c = 0.0;
            for (int z = o->rowptr[p]; z < o->rowptr[p + 1]; ++z) {
                int k = o->col[z];
                int sk = o->uint_slot[k];
                real fk, nk;
                if (use_star && sk >= 0) { fk = star[Q * sk + q]; nk = nstar[Q * sk + q]; }
                else { fk = o->fu[(size_t)q * nn + k]; nk = neq_u[(size_t)q * nn + k]; }
                real s_ik = CX[q] * o->gx[z] + CY[q] * o->gy[z];
                sum_s += s_ik * fk;
                sum_c += o->cc[z] * nk;
            }
            fnew[q] = base + dt * sum_s - (dt / tau_u) * sum_c;
        }
        if (o->kind[p] == KIND_WALL && o->cfg.wall_bc && plant[5] != 0.0) {
            /* no-slip: u -> 0 keeping rho and f^neq */
            real r, x, y, feq[Q], feq0[Q];
            moments(fnew, &r, &x, &y);
            equilibrium(r, x, y, feq);
            equilibrium(r, 0.0, 0.0, feq0);
            for (int q = 0; q < Q; ++q) fnew[q] = feq0[q] + plant[4] * (fnew[q] - feq[q]);
        }
        for (int q = 0; q < Q; ++q) o->fu_new[(size_t)q * nn + p] = fnew[q];
    }
    free(neq_u);
    real *tmp = o->fu; o->fu = o->fu_new; o->fu_new = tmp;
}

static void mesh_advance(oracle_t *o)
{
    int nu = o->n_uint;
    real *s0 = NULL, *s1 = NULL, *star = NULL, *nstar = NULL;
    int coupled = o->cfg.nx_cells > 0 && nu > 0;
    if (coupled) {
        s0 = (real *)malloc(sizeof(real) * 12 * nu);
        s1 = (real *)malloc(sizeof(real) * 12 * nu);
        star = (real *)malloc(sizeof(real) * Q * nu);
        nstar = (real *)malloc(sizeof(real) * Q * nu);
        olevel *fl = &o->lev[o->L];
        structured_to_mesh(o, fl->save, s0);   /* time t   */
        structured_to_mesh(o, fl->f, s1);      /* time t+1 */
    }
    real ts = o->cfg.tau_s;
    for (int m = 0; m < o->n_sub; ++m) {
        if (coupled) {
            double th = plant[6] * m / o->n_sub;
            for (int s = 0; s < nu; ++s) {
                real v[12];
                for (int a = 0; a < 12; ++a) v[a] = (1.0 - th) * s0[12 * s + a] + th * s1[12 * s + a];
                real feq[Q];
                equilibrium(v[0], v[1], v[2], feq);
                for (int q = 0; q < Q; ++q) {
                    nstar[Q * s + q] = plant[1] * (1.0 - 1.0 / (2.0 * ts)) * v[3 + q];
                    star[Q * s + q] = feq[q] + nstar[Q * s + q];
                }
            }
        }
        fv_substep(o, star, nstar);
    }
    free(s0); free(s1); free(star); free(nstar);
}

/* Drag and lift, eqs. (10)-(11): momentum flux out of the fluid through the
 * wall edges, sum_i c_i (c_i . N_e) (f_i(a) + f_i(b)) / 2, N_e = outward
 * normal times length; projected on the free-stream direction and its normal. */
static void wall_force(const oracle_t *o, real *fx, real *fy)
{
    real sx = 0.0, sy = 0.0;
    for (int e = 0; e < o->n_wall_edges; ++e) {
        int P = o->wedge[2 * e], Qn = o->wedge[2 * e + 1];
        real dx = wrap(o->xy[2 * Qn] - o->xy[2 * P], o->cfg.mesh_period[0]);
        real dy = wrap(o->xy[2 * Qn + 1] - o->xy[2 * P + 1], o->cfg.mesh_period[1]);
        real nx = dy, ny = -dx;
        for (int q = 0; q < Q; ++q) {
            real fa = o->fu[(size_t)q * o->nn + P], fb = o->fu[(size_t)q * o->nn + Qn];
            real cn = CX[q] * nx + CY[q] * ny;
            sx += CX[q] * cn * 0.5 * (fa + fb);
            sy += CY[q] * cn * 0.5 * (fa + fb);
        }
    }
    *fx = sx; *fy = sy;
}

/* Pressure and wall stresses at the wall nodes, eqs. (12)-(13).  Pressure is
 * p = rho c_s^2, so C_p = (rho - rho0) c_s^2 / q with q = rho0 U^2 / 2.  The FV
 * scheme integrates the continuous BGK equation, whose first-order
 * non-equilibrium moment gives the viscous stress directly:
 *   sigma = -Pi^neq,  Pi^neq = sum_i c_i c_i f_i - rho c_s^2 I - rho u u
 * (viscosity c_s^2 tau_u, no half-step shift).  At wall node P, V_P is half the
 * sum of the outward (into the body) length-normals of its wall edges; n = -V_P
 * / |V_P| points into the fluid and t = (n_y, -n_x) runs along the wall with the
 * fluid on its left.  Per wall node, in node order: C_p, the shear
 * C_f = t.sigma.n / q and the normal viscous stress C_n = n.sigma.n / q. */
static void wall_coefficients(const oracle_t *o, real *cp, real *cf, real *cn)
{
    real *V = (real *)calloc((size_t)2 * o->nn, sizeof(real));
    for (int e = 0; e < o->n_wall_edges; ++e) {
        int P = o->wedge[2 * e], Qn = o->wedge[2 * e + 1];
        real nx = wrap(o->xy[2 * Qn + 1] - o->xy[2 * P + 1], o->cfg.mesh_period[1]);
        real ny = -wrap(o->xy[2 * Qn] - o->xy[2 * P], o->cfg.mesh_period[0]);
        V[2 * P] += 0.5 * nx; V[2 * P + 1] += 0.5 * ny;
        V[2 * Qn] += 0.5 * nx; V[2 * Qn + 1] += 0.5 * ny;
    }
    const double CS2 = 1.0 / 3.0;
    real q = 0.5 * o->cfg.rho0 * o->cfg.u_inf * o->cfg.u_inf;
    int w = 0;
    for (int P = 0; P < o->nn; ++P) {
        if (o->kind[P] != KIND_WALL) continue;
        real f[Q], rho, ux, uy;
        for (int i = 0; i < Q; ++i) f[i] = o->fu[(size_t)i * o->nn + P];
        moments(f, &rho, &ux, &uy);
        real pxx = 0.0, pxy = 0.0, pyy = 0.0;
        for (int i = 0; i < Q; ++i) {
            pxx += CX[i] * CX[i] * f[i];
            pxy += CX[i] * CY[i] * f[i];
            pyy += CY[i] * CY[i] * f[i];
        }
        real sxx = -(pxx - rho * CS2 - rho * ux * ux);
        real sxy = -(pxy - rho * ux * uy);
        real syy = -(pyy - rho * CS2 - rho * uy * uy);
        real len = sqrt(V[2 * P] * V[2 * P] + V[2 * P + 1] * V[2 * P + 1]);
        real nx = -V[2 * P] / len, ny = -V[2 * P + 1] / len;
        real tx = ny, ty = -nx;
        real snx = sxx * nx + sxy * ny, sny = sxy * nx + syy * ny; /* sigma . n */
        cp[w] = (rho - o->cfg.rho0) * CS2 / q;
        cf[w] = (tx * snx + ty * sny) / q;
        cn[w] = (nx * snx + ny * sny) / q;
        w++;
    }
    free(V);
}

/* Force on the body by momentum exchange: every population f~_p that left a
 * fluid node towards a solid one (x + c_p solid) comes back reversed and gives
 * the body 2 c_p f~_p. */
static void body_force(const oracle_t *o, real *fx, real *fy)
{
    const olevel *lv = &o->lev[o->L];
    int nx = lv->nx, ny = lv->ny;
    int periodic = (o->L == 0 && o->cfg.periodic);
    real sx = 0.0, sy = 0.0;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            if (lv->cls[(size_t)j * nx + i] != CL_ACTIVE) continue;
            for (int p = 1; p < Q; ++p) {
                int a = i + CX[p], b = j + CY[p];
                if (periodic) { a = (a + nx) % nx; b = (b + ny) % ny; }
                if (a < 0 || b < 0 || a >= nx || b >= ny || lv->cls[(size_t)b * nx + a] != CL_SOLID) continue;
                real out = lv->post[LIDX(lv, p, i, j)];
                sx += (1.0 + plant[8]) * CX[p] * out;
                sy += (1.0 + plant[8]) * CY[p] * out;
            }
        }
    *fx = sx;
    *fy = sy;
}

static void record_forces(oracle_t *o)
{
    if (o->t >= o->hist_cap) {
        o->hist_cap *= 2;
        o->cd = (real *)realloc(o->cd, sizeof(real) * o->hist_cap);
        o->cl = (real *)realloc(o->cl, sizeof(real) * o->hist_cap);
    }
    real fx = 0, fy = 0;
    if (o->nn > 0) wall_force(o, &fx, &fy);
    else if (o->cfg.body_n > 0) body_force(o, &fx, &fy);
    real ca = cos(o->cfg.aoa), sa = sin(o->cfg.aoa);
    real qd = 0.5 * o->cfg.rho0 * o->cfg.u_inf * o->cfg.u_inf * o->cfg.chord;
    if (!(RE(qd) > 0)) qd = 1.0;
    o->cd[o->t] = (fx * ca + fy * sa) / qd;
    o->cl[o->t] = (-fx * sa + fy * ca) / qd;
    o->t++;
    if (o->ws_on) {
        real *c = o->ws_tmp;
        wall_coefficients(o, c, c + o->n_wn, c + 2 * o->n_wn);
        for (int k = 0; k < 3 * o->n_wn; ++k) o->ws_sum[k] += c[k];
        o->ws_n++;
    }
}

/* ------------------------------------------------------------------ */
/* public entry points                                                   */
/* ------------------------------------------------------------------ */

int or_step(void *h, int64_t n_finest)
{
    oracle_t *o = (oracle_t *)h;
    if (o->cfg.nx_cells > 0) {
        int per = 1 << o->L;
        if (n_finest % per) return -1;
        for (int64_t b = 0; b < n_finest / per; ++b) level_step(o, 0);
    } else {
        for (int64_t s = 0; s < n_finest; ++s) { mesh_advance(o); record_forces(o); }
    }
    return 0;
}

/* pre-collision populations of level l as [Q][ny][nx]; non-active nodes are zero */
int or_get_level(void *h, int32_t l, real *out)
{
    oracle_t *o = (oracle_t *)h;
    if (o->cfg.nx_cells <= 0 || l < 0 || l > o->L) return -1;
    olevel *lv = &o->lev[l];
    for (int q = 0; q < Q; ++q)
        for (int j = 0; j < lv->ny; ++j)
            for (int i = 0; i < lv->nx; ++i)
                out[LIDX(lv, q, i, j)] = lv->cls[(size_t)j * lv->nx + i] == CL_ACTIVE ? lv->f[LIDX(lv, q, i, j)] : 0.0;
    return 0;
}

/* replaces the pre-collision populations of level l (every node) */
int or_set_level(void *h, int32_t l, const real *in)
{
    oracle_t *o = (oracle_t *)h;
    if (o->cfg.nx_cells <= 0 || l < 0 || l > o->L) return -1;
    olevel *lv = &o->lev[l];
    memcpy(lv->f, in, sizeof(real) * Q * lv->nx * lv->ny);
    return 0;
}

int or_get_mesh(void *h, real *out)
{
    oracle_t *o = (oracle_t *)h;
    memcpy(out, o->fu, sizeof(real) * Q * o->nn);
    return 0;
}

int or_set_mesh(void *h, const real *in)
{
    oracle_t *o = (oracle_t *)h;
    memcpy(o->fu, in, sizeof(real) * Q * o->nn);
    return 0;
}

int or_level_class(void *h, int32_t l, uint8_t *out)
{
    oracle_t *o = (oracle_t *)h;
    if (o->cfg.nx_cells <= 0 || l < 0 || l > o->L) return -1;
    memcpy(out, o->lev[l].cls, (size_t)o->lev[l].nx * o->lev[l].ny);
    return 0;
}

int64_t or_history(void *h, real *cd, real *cl, int64_t cap)
{
    oracle_t *o = (oracle_t *)h;
    int64_t n = o->t < cap ? o->t : cap;
    for (int64_t a = 0; a < n; ++a) { cd[a] = o->cd[a]; cl[a] = o->cl[a]; }
    return o->t;
}

/* ints: [0] levels, [1] n_sub, [2] n_sint, [3] n_uint, [4] n_fallback,
 *       [5] n_wall_edges, [6..9] nx per level, [10..13] ny per level
 * dbls: [0] tau_u, [1..4] tau per level */
int or_info(void *h, int32_t *ints, double *dbls)
{
    oracle_t *o = (oracle_t *)h;
    ints[0] = o->cfg.nx_cells > 0 ? o->L + 1 : 0;
    ints[1] = o->n_sub; ints[2] = o->n_sint; ints[3] = o->n_uint; ints[4] = o->n_fallback;
    ints[5] = o->n_wall_edges;
    for (int l = 0; l < 4; ++l) {
        ints[6 + l] = l <= o->L ? o->lev[l].nx : 0;
        ints[10 + l] = l <= o->L ? o->lev[l].ny : 0;
        dbls[1 + l] = l <= o->L ? RE(o->lev[l].tau) : 0.0;
    }
    dbls[0] = RE(o->tau_u);
    return 0;
}

/* structured interpolation node stencils: ij[2n], don[8n], w[8n] */
int or_sint(void *h, int32_t *ij, int32_t *don, real *w)
{
    oracle_t *o = (oracle_t *)h;
    for (int s = 0; s < o->n_sint; ++s) {
        ij[2 * s] = o->sint_ij[2 * s]; ij[2 * s + 1] = o->sint_ij[2 * s + 1];
        for (int d = 0; d < SDON; ++d) { don[SDON * s + d] = o->sint_don[SDON * s + d]; w[SDON * s + d] = o->sint_w[SDON * s + d]; }
    }
    return o->n_sint;
}

/* Starts the time means of the wall coefficients: every finest step from now
 * on adds its post-step values.  Returns the number of wall nodes. */
int or_wall_stats_begin(void *h)
{
    oracle_t *o = (oracle_t *)h;
    int n = 0;
    for (int P = 0; P < o->nn; ++P) n += o->kind[P] == KIND_WALL;
    free(o->ws_sum); free(o->ws_tmp);
    o->n_wn = n;
    o->ws_sum = (real *)calloc((size_t)3 * n + 1, sizeof(real));
    o->ws_tmp = (real *)calloc((size_t)3 * n + 1, sizeof(real));
    o->ws_n = 0;
    o->ws_on = 1;
    return n;
}

/* Time means since or_wall_stats_begin, per wall node in node order:
 * C_p, C_f, C_n (see wall_coefficients).  Returns the number of steps. */
int64_t or_wall_stats(void *h, real *cp, real *cf, real *cn)
{
    oracle_t *o = (oracle_t *)h;
    if (!o->ws_on) return -1;
    for (int w = 0; w < o->n_wn; ++w) {
        cp[w] = o->ws_sum[w] / (real)o->ws_n;
        cf[w] = o->ws_sum[o->n_wn + w] / (real)o->ws_n;
        cn[w] = o->ws_sum[2 * o->n_wn + w] / (real)o->ws_n;
    }
    return o->ws_n;
}

/* the same coefficients for the current mesh state */
int or_wall_coefficients(void *h, real *cp, real *cf, real *cn)
{
    oracle_t *o = (oracle_t *)h;
    wall_coefficients(o, cp, cf, cn);
    return 0;
}

/* wall force of the current mesh state (not normalised) */
int or_wall_force(void *h, real *fx, real *fy)
{
    oracle_t *o = (oracle_t *)h;
    wall_force(o, fx, fy);
    return 0;
}
