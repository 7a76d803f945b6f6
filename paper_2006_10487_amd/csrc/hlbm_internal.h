// hlbm_internal.h -- host plan and device views of the HLBM library.
//
// The plan is built on the host (prep.cpp) from the caller's grid and mesh:
// level sizes and relaxation times, the median-dual finite-volume
// coefficients in reverse Cuthill-McKee node order, interpolation stencils,
// and the byte layout of the caller's workspace.  Kernels (kernels.hip)
// receive small views by value.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <array>
#include <string>
#include <vector>

#include "../../include/hlbm.h"

namespace hlbm {

constexpr int kQ = 9;
constexpr int kSDon = 8;     // donors of a structured interpolation node (two 6-node stencils on an edge)
constexpr int kUDon = 9;     // donors of a mesh interpolation node (3 x 3 block)
constexpr int kMacro = 12;   // (rho or rho - rho0, ux, uy, f^neq[9])
constexpr int kRec = 12;
constexpr int kTileMeta = 10;  // ints per fused-FV tile: node off, edge off, width, n_le[0..4], star off, star count
// fused-FV tile edge tables: local column, or, where an interpolation pivot
// reads the interpolated f* of its neighbour (eqs. (5)-(7)), kFtStar plus the
// neighbour's slot in the tile's list of such nodes
constexpr int32_t kFtStar = 1 << 30;
constexpr int32_t kFtLocal = kFtStar - 1;
constexpr int kStarRec = 20;   // per staged f* node: f*[9], its f^neq part [9], 2 unused (16-byte rows)
constexpr int kFvStage = 2;    // nodes per thread of a fused FV sub-step (results held in registers)
constexpr int kMaxFuse = 4;
constexpr int kAdjRec = 10;   // doubles per mesh node of the adjoint fields (9 used)     // mesh node record: f_0..f_8, rho (or rho - rho0), ux, uy

// LDS bytes of one fused-FV workgroup: node records and plan indices of the
// tile with its rings, then f* of the tile's interpolation nodes at each of the
// launch's sub-steps.
__host__ __device__ inline size_t fv_stg_offset(int maxl, size_t elem) { return (size_t(maxl) * (kRec * elem + 4) + 15) / 16 * 16; }
inline size_t fv_lds_bytes(int maxl, int maxs, int fuse, size_t elem) {
    return fv_stg_offset(maxl, elem) + size_t(fuse) * size_t(maxs) * kStarRec * elem;
}

struct LevelPlan {
    int nx = 0, ny = 0, pitch = 0;  // nodes, row pitch in elements
    int sp = 1;                     // spacing in finest units
    double ox = 0, oy = 0;          // origin in finest units
    double tau = 1;
    int i0 = 0, j0 = 0;             // origin in parent nodes
    bool has_child = false;
    int ci0 = -4, cj0 = -4, ci1 = -4, cj1 = -4;  // child rectangle in this level's nodes
    bool perim_inactive = false;    // refined level: perimeter nodes come from the parent
    bool farfield = false, periodic = false;
    int64_t active = 0;             // collide-stream nodes
    int sj0 = 0, sj1 = 0;           // rows with inactive spans (finest level, inner ellipse)
};

struct Plan {
    // run parameters
    int L = 0, nlev = 0;
    double tau_s = 0, tau_u = 0, dt_u = 0;
    int n_sub = 0, precision = 0, interp = 0;
    bool periodic = false, wall_bc = true, has_grid = false, has_mesh = false, has_body = false;
    double u_inf = 0, aoa = 0, rho0 = 1, chord = 1;
    int check_every = 0, hist_len = 65536;
    LevelPlan lev[4];
    // finest level, inner ellipse: inactive nodes of row sj0 + r are [span[2r], span[2r+1])
    std::vector<int32_t> spans;
    // structured interpolation nodes (finest level), eq. (4)
    std::vector<int32_t> sint_node;      // i + nx * j
    std::vector<int32_t> sint_don;       // kSDon per node, mesh node in plan order, -1 = unused
    std::vector<double> sint_w;
    int n_fallback = 0;
    // body resolved by bounce-back (finest level): solid nodes are the spans; the
    // collide-stream nodes with a solid neighbour, i + nx * j, and per node the bit
    // mask of directions q whose source x - c_q is solid
    int n_solid = 0;
    std::vector<int32_t> bounce_node, bounce_mask;
    // mesh in plan order [wall | interior | interpolation]
    int nn = 0, n_wall = 0, n_core = 0, n_int = 0, nt = 0;
    std::vector<int32_t> perm;           // perm[new] = caller index
    std::vector<int32_t> rowptr, col;    // CSR, self entry first
    int ell_width = 8;                   // slots per node of the device neighbour table
    int ft_width = 8;                    // slots per node of the fused-FV tile tables (7 when no row is longer)
    std::vector<double> gx, gy, cc;      // G_Pk (x, y) and C_Pk
    std::vector<int32_t> wedge;          // wall edges (P, Q) in plan order, fluid on the left
    std::vector<double> wnorm;           // outward normal times length of each wall edge
    // fused FV sub-steps (temporal blocking): tiles of at most fv_tile plan
    // nodes, each with the rings of neighbours that fv_fuse Jacobi sub-steps
    // reach; per tile kTileMeta ints {node offset, edge offset, edge-table
    // width, n_le[0..fv_fuse]} with n_le[r] = local nodes within ring r
    // fv_threads: workgroup size of the fused kernel, at least fv_maxw / kFvStage
    // fv_maxs: most f* nodes of a tile (their f* is staged in LDS once per sub-step)
    int f2c_filter = 0;
    int fv_fuse = 1, fv_tile = 256, fv_threads = 256, fv_maxl = 0, fv_maxw = 0, fv_maxs = 0, n_tiles = 0;
    std::vector<int32_t> ft_meta, ft_node;
    std::vector<int32_t> ft_star;        // per tile: interpolation slot (plan index - n_core) of its f* nodes
    std::vector<int32_t> ft_col;         // local column per (slot, computed node) of each tile
    std::vector<int32_t> ft_src;         // index into col / gx / gy / cc of that entry, -1 = unused
    std::vector<double> wall_nrm;        // [n_wall][2] unit normal into the fluid at each wall node
    std::vector<int32_t> wall_slot;      // [n_wall] rank of the wall node by caller index
    // mesh interpolation nodes <- finest level, eq. (9)
    std::vector<int32_t> uint_don;       // kUDon per slot, finest node i + nx * j, -1 = unused
    std::vector<double> uint_w;
    // the caller's mesh (caller order), kept for the shape adjoint, and the
    // derivatives of its coordinates with respect to n_shape shape parameters
    // ([n_shape][n_nodes][2], caller order)
    int n_shape = 0;
    std::vector<double> dshape;
    std::vector<double> mxy;
    std::vector<int32_t> mtri;
    std::vector<std::array<int, 2>> mbnd;   // boundary edges, fluid on the left
    // workspace layout (byte offsets)
    struct {
        size_t lev[4][2];
        size_t side[4][2];
        size_t spans, sint_node, sint_don, sint_w, bounce_node, bounce_mask;
        size_t mesh[2], rowptr, edges, wedge, wnorm, prep[2], uint_don, uint_w, hist, stage;
        size_t wall_nrm, wall_slot, wsum, wout;
        size_t ft_meta, ft_node, ft_edges, ft_star;
        size_t total;
    } off{};
    size_t stage_bytes = 0;
    size_t elem = 8;                     // bytes per stored population
};

// Builds the plan; returns HLBM_OK or an error code with a message.
int build_plan(const hlbm_grid* g, const hlbm_mesh* m, double Re, double tau, Plan& p, std::string& err);

// Reverse of the mesh-geometry preprocessing: given the adjoints of the
// finite-volume coefficients (gbar[(z * nn + P) * 3 + {0,1,2}] for (G_x, G_y, C)
// of ELL slot z of plan row P), of the half wall normals summed at each wall
// node (vbar[2 * P + {0,1}]) and of the interpolation weights (w5bar in the
// layout of sint_w, w6bar in the layout of uint_w), adds d J / d(mesh
// coordinates) to grad[2 * caller node + {0,1}].  Returns HLBM_OK or an error.
int mesh_geometry_adjoint(const Plan& p, const double* gbar, const double* vbar, const double* w5bar,
                          const double* w6bar, double* grad, std::string& err);

// ---------------------------------------------------------------------------
// device views
// ---------------------------------------------------------------------------

struct KLevel {
    int nx, ny, pitch;
    long long rs;                    // row stride: 9 * pitch (planes of one row are adjacent)
    double omega;                    // 1 / tau
    int perim_inactive;
    int ci0, cj0, ci1, cj1;          // strictly inside -> not a collide-stream node
    int farfield, periodic;
    const int32_t* spans;            // inner-ellipse or solid-body spans (finest level), or null
    int sj0, sj1;
    int n_bounce;                    // body resolved by bounce-back: nodes with a solid neighbour
    const int32_t* bounce_node;      // i + nx * j
    const int32_t* bounce_mask;      // bit q: the source x - c_q is solid
    double u_in_x, u_in_y, rho0;     // far-field data
};

struct KMesh {
    int nn, n_wall, n_core;
    int ell_width;                   // neighbour slots per node (8 or 16)
    int ft_width;                    // slots per node of the tile tables (7, 8 or 16)
    const void* edges;               // ELL (col, gx, gy, c) records, slot-major
    double dt, dt_over_tau;          // Delta t_u, Delta t_u / tau_u
    double star_neq;                 // 1 - 1 / (2 tau_s), eq. (5)-(6)
    int wall_bc;
    double rho0;
    // fused sub-steps (fuse > 1): tile tables and the LDS size they need
    int fuse, n_sub, n_tiles, maxl, maxw, tile;   // maxw: largest edge-table width (nodes of sub-step 1)
    int maxs;                                     // most staged f* nodes of a tile
    int threads;                                  // workgroup size, kFvStage * threads >= maxw
    const int32_t* ft_meta;
    const int32_t* ft_node;
    const void* ft_edges;
    const int32_t* ft_star;
    // optional: the pre-reset (rho, u_x, u_y) of every wall node after each
    // sub-step of the launch, at wmom + j * wmom_stride + 3 * P (j = sub-step of
    // the launch); read by the adjoint's no-slip reset transpose
    double* wmom;
    size_t wmom_stride;
};

// launchers (kernels.hip); `prec` is HLBM_FP64 or HLBM_FP32_SHIFTED
void launch_fill_uniform(int prec, void* buf, const KLevel& L, double rho, double ux, double uy, hipStream_t s);
void launch_stream_collide(int prec, const KLevel& L, const void* A, void* B, hipStream_t s);
void launch_export_level(int prec, const KLevel& L, const void* A, double* out, int j0, int j1, hipStream_t s);
void launch_import_level(int prec, const KLevel& L, void* A, const double* in, int j0, int j1, hipStream_t s);
void launch_coarse_to_fine(int prec, const KLevel& parent, const KLevel& child, int ci0, int cj0,
                           const void* parentA, void* childA, void* side_cur, const void* side_prev,
                           double theta, int compute_side, double tau_c, double tau_f, hipStream_t s);
void launch_side_init(int prec, const KLevel& parent, int ci0, int cj0, int nxc, int nyc,
                      const void* parentA, void* side, hipStream_t s);
void launch_fine_to_coarse(int prec, const KLevel& parent, const KLevel& child, int ci0, int cj0,
                           int nxc, int nyc, const void* child_prev, void* parent_dst, double tau_c,
                           double tau_f, int filter, hipStream_t s);
void launch_mesh_to_struct(int prec, const KLevel& fine, void* fineA, int n, const int32_t* node,
                           const int32_t* don, const void* w, const void* mesh_f, int nn, double factor,
                           hipStream_t s);
void launch_struct_to_mesh(int prec, const KLevel& fine, const void* fineA, int n, const int32_t* don,
                           const void* w, void* prep, hipStream_t s);
void launch_fv_substep(int prec, const KMesh& M, const void* fin, void* fout, const void* prep0,
                       const void* prep1, double theta, hipStream_t s);
// k = 1..M.fuse sub-steps m0 .. m0 + k - 1 in one launch (tiles with halos in LDS);
// with mid set, also the states after sub-steps m0 .. m0 + k - 2 at
// mid + j * mid_stride_bytes (j = 0..k-2)
void launch_fv_fused(int prec, const KMesh& M, const void* fin, void* fout, const void* prep0, const void* prep1,
                     int m0, int k, hipStream_t s, void* mid = nullptr, size_t mid_stride_bytes = 0);
void launch_wall_stats(int prec, const void* f, int n_wall, const double* nrm, double rho0, double inv_q, double* sum,
                       hipStream_t s);
void launch_wall_stats_final(int n_wall, const double* sum, const int32_t* slot, double n, double* out, hipStream_t s);
// momentum exchanged with a body resolved by bounce-back (finest level L, its
// post-collision buffer A), as C_D, C_L into out[0..1]
void launch_body_force(int prec, const KLevel& L, const void* A, double* out, double ca, double sa, double qn,
                       hipStream_t s);
void launch_wall_force(int prec, const void* f, int n_edges, const int32_t* wedge,
                       const double* wnorm, double* hist_slot, double cos_a, double sin_a, double qnorm,
                       hipStream_t s);
void launch_mesh_convert(int prec, int nn, const double* in, void* out, int to_storage, double rho0,
                         hipStream_t s);

// ---------------------------------------------------------------------------
// adjoint (FP64, single structured level)
// ---------------------------------------------------------------------------

struct KAdj {
    KLevel L;                        // the structured level
    KMesh M;                         // the mesh
    const void* tedges;              // transposed neighbour table: slot z of node k = (P, z_P, G_Pk, C_Pk) with z_P the
                                     // slot of k in row P; slot 0 = (k, 0, sum_{j!=k} G_kj, C_kk)
    double dt, dtt, ddtt_dtau;       // Delta t_u, Delta t_u / tau_u, d(Delta t_u / tau_u)/d tau
    double cst, dcst_dtau;           // 1 - 1/(2 tau), d/d tau
    double omega, domega_dtau;       // 1 / tau, d/d tau
    double phi, dphi_dtau;           // 2 (tau - 1)/(2 tau - 1), d/d tau
    double uin_x, uin_y, duin_x, duin_y;  // inlet velocity and d/d alpha
    double* partial;                 // per-block (d alpha, d tau) partial sums
    // adjoints of the mesh-geometry coefficients, accumulated over the run (null: not wanted)
    double* gbar;                    // [ell_width][nn][3]: (G_x, G_y, C) of the entry in transposed slot z of
                                     // node k (G parts without the pivot's base term, which is in gpivot);
                                     // slot 0 = the pivot k itself, C only
    double* gpivot;                  // [nn][2]: Delta t_u sum_q zbar_Pq c_q base_Pq, per pivot
    double* vbar;                    // [n_wall][2]: half wall normals summed at each wall node
    double* w5bar;                   // eq. (4) weights, per entry of the transposed (donor-major) list
    double* w6bar;                   // eq. (9) weights, per entry of the transposed (donor-major) list
};

void launch_zero(double* p, size_t n, hipStream_t s);
void launch_adj_force(const KAdj& K, double* mbar, const double* vwall, double jx, double jy, const double* fst,
                      hipStream_t s);
// wmom: pre-reset (rho, u) of the wall nodes in the sub-step whose reset is
// transposed (recorded by the forward, KMesh::wmom)
void launch_adj_fv_wall(const KAdj& K, const double* wmom, const double* ybar, double* zwall, hipStream_t s);
void launch_adj_fv(const KAdj& K, const double* Mrec, const double* ybar, const double* zwall, double* mbar,
                   const double* prep0, const double* prep1, double theta, double* p0bar, double* p1bar, int pslot,
                   const double* wmom_prev, double* zwall_prev, hipStream_t s);
void launch_adj_collide(const KAdj& K, const double* A, const double* bbar, double* prebar, int pslot, hipStream_t s);
void launch_adj_s2m(const KAdj& K, const double* A, int nd, const int32_t* node, const int32_t* ptr,
                    const int32_t* slot, const double* w, const double* pbar, double* prebar, hipStream_t s);
void launch_adj_bc(const KAdj& K, const double* A, double* prebar, int pslot, hipStream_t s);
void launch_adj_push(const KAdj& K, const double* prebar, double* abar, hipStream_t s);
void launch_adj_m2s_a(const KAdj& K, const double* Mrec, int n, const int32_t* node, const int32_t* don,
                      const double* w, double* abar, double* m5bar, int pslot, hipStream_t s);
void launch_adj_m2s_b(const KAdj& K, const double* Mrec, const int32_t* ptr, const int32_t* slot, const double* w,
                      const double* m5bar, double* mbar, hipStream_t s);
void launch_adj_alpha_state(const KAdj& K, const double* abar, const double* mbar, const double* dfeq, bool with_mesh,
                            int pslot, hipStream_t s);
void launch_adj_c2f_a(const KLevel& C, const double* side_prev, const double* side_cur, double theta, double* ybar,
                      double* vbar, double coef, double dcoef, double* partial, int pslot, hipStream_t s);
void launch_adj_c2f_b(int nxc, int nyc, const double* vbar, double theta, double* sbar_prev, double* sbar_cur,
                      hipStream_t s);
void launch_adj_f2c(const KLevel& P, const KLevel& C, int ci0, int cj0, int nxc, int nyc, const double* cprev,
                    double* xbar, double* ybar, double coef, double dcoef, double* partial, int pslot, int filter,
                    hipStream_t s);
// threads (and so partial-sum blocks) of launch_adj_f2c: the ring nodes, or with the
// filtered transfer the fine band their 3 x 3 stencils cover
int f2c_adj_threads(int nxc, int nyc, int filter);
void launch_adj_side(const KLevel& P, int ci0, int cj0, int nxc, int nyc, const double* A, const double* sbar,
                     double* prebar, hipStream_t s);
void launch_reduce_partials(const double* partial, int n, double* acc, hipStream_t s);
int adj_blocks_collide(const KLevel& L);
int adj_fv_blocks(const KMesh& M);   // partial slots of one launch_adj_fv
// workgroup size of the FV sub-step adjoint: small meshes are latency-bound,
// and small workgroups spread them over more CUs
constexpr int kAdjFvBlock = 64;
constexpr int kAdjFvSimds = 1024;   // SIMDs of an MI355X (256 CUs x 4)
int adj_blocks_nodes(int n);

}  // namespace hlbm

struct AdjState;
struct hlbm_ctx {
    hlbm::Plan p;
    hipStream_t s = nullptr;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    int cur[4] = {0, 0, 0, 0};   // buffer holding the current post-collision state
    int side_t[4] = {0, 0, 0, 0};  // side slot holding the parent's (rho, u, f^neq) at the parent's time
    int mesh_cur = 0;
    int prep_t = 0;               // prep slot holding the mesh interpolation values at time t
    int64_t t = 0;
    int64_t last_check = 0;
    bool poisoned = false;
    bool dirty = false;           // an import must be finished before stepping
    std::string err;
    hlbm::KLevel kl[4];
    hlbm::KMesh km;
    std::vector<double> tmp;
    // adjoint (objective run and reverse sweep)
    AdjState* adj = nullptr;
    // observer of the step recursion (the adjoint's segment recompute), or null:
    // event 0 = entry of a level-l step (l < L), 1 = the parent's side values of
    // that step are recorded, 2 = entry of a finest step (before eq. (4)), 3 = the
    // finest input after eq. (4), before its collide-stream
    void (*rec)(hlbm_ctx*, int event, int level) = nullptr;
    // with sub_sink set, the FV sub-steps of the next finest step write their
    // states to sub_sink + m * sub_stride (m = 0..n-1, the state after sub-step
    // m + 1); the last one is copied back into the mesh buffer
    char* sub_sink = nullptr;
    size_t sub_stride = 0;
    // with wmom_sink set as well, the pre-reset (rho, u) of the wall nodes after
    // sub-step m go to wmom_sink + m * wmom_stride (doubles)
    double* wmom_sink = nullptr;
    size_t wmom_stride = 0;
    // wall statistics (eqs. (12)-(13)): accumulating, and finest steps summed
    bool wstat = false;
    int64_t wstat_n = 0;
    // instrumentation
    bool prof = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;

    void* lev(int l, int b) { return ws + p.off.lev[l][b]; }
    void* side(int l, int b) { return ws + p.off.side[l][b]; }
    void* mesh(int b) { return ws + p.off.mesh[b]; }
    void* prep(int b) { return ws + p.off.prep[b]; }
    double* hist() { return reinterpret_cast<double*>(ws + p.off.hist); }
    double* stage() { return reinterpret_cast<double*>(ws + p.off.stage); }
};


namespace hlbm {
// Static workspace of hlbm_create_noalloc on the current device (kernels.hip):
// its device address, looked up once per device.  Returns HLBM_OK or HLBM_E_DEVICE.
constexpr size_t kNoAllocBytes = HLBM_NOALLOC_MAX_BYTES;
int noalloc_workspace(void** ptr);
void finish_import(hlbm_ctx* c);
void finest_step(hlbm_ctx* c);
void level_step(hlbm_ctx* c, int l);
void reset_initial_state(hlbm_ctx* c);
hipEvent_t take_event(hlbm_ctx* c);
void adj_free(AdjState* a);
int hip_check(hlbm_ctx* c, hipError_t e, const char* what);
int set_err(hlbm_ctx* c, int code, const std::string& msg);
}  // namespace hlbm
