// capi.cpp -- C ABI of the HLBM library: context, workspace carving, the
// per-step orchestration of the hybrid scheme, state import/export, forces.
//
// One finest step t -> t+1, inside the level recursion (Sec. 4 time
// subcycling: level l advances once per 2^(L-l) finest steps, and each of
// its steps is followed by two steps of the finer box):
//   level_step(l):
//     l == L: structured interpolation nodes <- mesh at t      (eq. (4))
//     collide-stream of level l                                (eq. (1))
//     l <  L: coarse -> fine perimeter at theta = 0; level_step(l+1);
//             coarse -> fine perimeter at theta = 1/2; level_step(l+1);
//             fine -> coarse ring                               (Sec. 4)
//     l == L: mesh interpolation nodes <- finest level at t+1  (eq. (9))
//             n finite-volume sub-steps, theta = m / n         (eqs. (3), (5))
//             drag and lift                                     (eqs. (10)-(11))
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "hlbm_internal.h"

using namespace hlbm;

namespace hlbm {

std::string g_create_err;

hipEvent_t take_event(hlbm_ctx* c) {
    if (!c->ev_pool.empty()) {
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Brackets one kernel launch with events when profiling is on.
struct Timed {
    hlbm_ctx* c;
    int cls;
    hipEvent_t a = nullptr, b = nullptr;
    Timed(hlbm_ctx* c_, int cls_) : c(c_), cls(cls_) {
        if (!c->prof) return;
        a = take_event(c);
        b = take_event(c);
        if (a && b) (void)hipEventRecord(a, c->s);
    }
    ~Timed() {
        if (!c->prof || !a || !b) return;
        (void)hipEventRecord(b, c->s);
        c->ev_pending.push_back({cls, {a, b}});
    }
};

int set_err(hlbm_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    else g_create_err = msg;
    return code;
}

int hip_check(hlbm_ctx* c, hipError_t e, const char* what) {
    if (e == hipSuccess) return HLBM_OK;
    return set_err(c, HLBM_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

template <typename T>
std::vector<char> pack_real(const std::vector<double>& v) {
    std::vector<char> out(v.size() * sizeof(T));
    T* d = reinterpret_cast<T*>(out.data());
    for (size_t a = 0; a < v.size(); ++a) d[a] = T(v[a]);
    return out;
}

int upload(hlbm_ctx* c, size_t off, const void* src, size_t bytes) {
    if (!bytes) return HLBM_OK;
    return hip_check(c, hipMemcpyAsync(c->ws + off, src, bytes, hipMemcpyHostToDevice, c->s), "hipMemcpyAsync");
}

void setup_views(hlbm_ctx* c) {
    const Plan& p = c->p;
    for (int l = 0; l <= p.L; ++l) {
        const LevelPlan& v = p.lev[l];
        KLevel& k = c->kl[l];
        k.nx = v.nx;
        k.ny = v.ny;
        k.pitch = v.pitch;
        k.rs = 9LL * v.pitch;
        k.omega = 1.0 / v.tau;
        k.perim_inactive = v.perim_inactive;
        k.ci0 = v.has_child ? v.ci0 : -4;
        k.cj0 = v.has_child ? v.cj0 : -4;
        k.ci1 = v.has_child ? v.ci1 : -4;
        k.cj1 = v.has_child ? v.cj1 : -4;
        k.farfield = v.farfield;
        k.periodic = v.periodic;
        const bool spans = l == p.L && !p.spans.empty();
        k.spans = spans ? reinterpret_cast<const int32_t*>(c->ws + p.off.spans) : nullptr;
        k.sj0 = v.sj0;
        k.sj1 = v.sj1;
        const bool bounce = l == p.L && !p.bounce_node.empty();
        k.n_bounce = bounce ? int(p.bounce_node.size()) : 0;
        k.bounce_node = bounce ? reinterpret_cast<const int32_t*>(c->ws + p.off.bounce_node) : nullptr;
        k.bounce_mask = bounce ? reinterpret_cast<const int32_t*>(c->ws + p.off.bounce_mask) : nullptr;
        k.u_in_x = p.u_inf * std::cos(p.aoa);
        k.u_in_y = p.u_inf * std::sin(p.aoa);
        k.rho0 = p.rho0;
    }
    KMesh& m = c->km;
    m.nn = p.nn;
    m.n_wall = p.n_wall;
    m.n_core = p.n_core;
    m.ell_width = p.ell_width;
    m.ft_width = p.ft_width;
    m.edges = c->ws + p.off.edges;
    m.dt = p.dt_u;
    m.dt_over_tau = p.dt_u / p.tau_u;
    m.star_neq = 1.0 - 1.0 / (2.0 * p.tau_s);
    m.wall_bc = p.wall_bc;
    m.rho0 = p.rho0;
    m.fuse = p.fv_fuse;
    m.n_sub = p.n_sub;
    m.n_tiles = p.n_tiles;
    m.maxl = p.fv_maxl;
    m.maxs = p.fv_maxs;
    m.maxw = p.fv_maxw;
    m.tile = p.fv_tile;
    m.threads = p.fv_threads;
    m.ft_meta = reinterpret_cast<const int32_t*>(c->ws + p.off.ft_meta);
    m.ft_node = reinterpret_cast<const int32_t*>(c->ws + p.off.ft_node);
    m.ft_edges = c->ws + p.off.ft_edges;
    m.ft_star = reinterpret_cast<const int32_t*>(c->ws + p.off.ft_star);
    m.wmom = nullptr;
    m.wmom_stride = 0;
}

int upload_tables(hlbm_ctx* c) {
    const Plan& p = c->p;
    const bool f64 = p.precision == HLBM_FP64;
    int rc = HLBM_OK;
    auto real = [&](const std::vector<double>& v) { return f64 ? pack_real<double>(v) : pack_real<float>(v); };
    std::vector<std::vector<char>> keep;   // host copies alive until the stream syncs
    rc |= upload(c, p.off.spans, p.spans.data(), p.spans.size() * 4);
    rc |= upload(c, p.off.bounce_node, p.bounce_node.data(), p.bounce_node.size() * 4);
    rc |= upload(c, p.off.bounce_mask, p.bounce_mask.data(), p.bounce_mask.size() * 4);
    rc |= upload(c, p.off.sint_node, p.sint_node.data(), p.sint_node.size() * 4);
    rc |= upload(c, p.off.sint_don, p.sint_don.data(), p.sint_don.size() * 4);
    keep.push_back(real(p.sint_w));
    rc |= upload(c, p.off.sint_w, keep.back().data(), keep.back().size());
    if (p.has_mesh) {
        // ELL neighbour table: slot z of node P at z * nn + P; unused slots col = -1
        const size_t W = size_t(p.ell_width), rs = f64 ? 32 : 16;
        std::vector<char> rec(W * p.nn * rs, 0);
        for (int P = 0; P < p.nn; ++P)
            for (size_t z = 0; z < W; ++z) {
                char* r = rec.data() + (z * p.nn + P) * rs;
                const int zz = p.rowptr[P] + int(z);
                const int32_t col = zz < p.rowptr[P + 1] ? p.col[zz] : -1;
                std::memcpy(r, &col, 4);
                if (col < 0) continue;
                if (f64) {
                    const double v[3] = {p.gx[zz], p.gy[zz], p.cc[zz]};
                    std::memcpy(r + 8, v, 24);
                } else {
                    const float v[3] = {float(p.gx[zz]), float(p.gy[zz]), float(p.cc[zz])};
                    std::memcpy(r + 4, v, 12);
                }
            }
        keep.push_back(std::move(rec));
        rc |= upload(c, p.off.edges, keep.back().data(), keep.back().size());
        rc |= upload(c, p.off.wedge, p.wedge.data(), p.wedge.size() * 4);
        rc |= upload(c, p.off.wnorm, p.wnorm.data(), p.wnorm.size() * 8);
        if (p.fv_fuse > 1) {
            rc |= upload(c, p.off.ft_meta, p.ft_meta.data(), p.ft_meta.size() * 4);
            rc |= upload(c, p.off.ft_node, p.ft_node.data(), p.ft_node.size() * 4);
            rc |= upload(c, p.off.ft_star, p.ft_star.data(), p.ft_star.size() * 4);
            // tile edge tables: the ELL record layout with local columns
            std::vector<char> te(p.ft_col.size() * rs, 0);
            for (size_t e = 0; e < p.ft_col.size(); ++e) {
                char* r = te.data() + e * rs;
                const int32_t col = p.ft_col[e];
                std::memcpy(r, &col, 4);
                const int zz = p.ft_src[e];
                if (zz < 0) continue;
                if (f64) {
                    const double v[3] = {p.gx[zz], p.gy[zz], p.cc[zz]};
                    std::memcpy(r + 8, v, 24);
                } else {
                    const float v[3] = {float(p.gx[zz]), float(p.gy[zz]), float(p.cc[zz])};
                    std::memcpy(r + 4, v, 12);
                }
            }
            keep.push_back(std::move(te));
            rc |= upload(c, p.off.ft_edges, keep.back().data(), keep.back().size());
        }
        rc |= upload(c, p.off.wall_nrm, p.wall_nrm.data(), p.wall_nrm.size() * 8);
        rc |= upload(c, p.off.wall_slot, p.wall_slot.data(), p.wall_slot.size() * 4);
        rc |= upload(c, p.off.uint_don, p.uint_don.data(), p.uint_don.size() * 4);
        keep.push_back(real(p.uint_w));
        rc |= upload(c, p.off.uint_w, keep.back().data(), keep.back().size());
    }
    if (rc) return HLBM_E_DEVICE;
    return hip_check(c, hipStreamSynchronize(c->s), "hipStreamSynchronize");
}

// Derived state after the streamed populations of every level were written
// into its previous buffer (by a scatter) and the mesh into its current one:
// post-collision state, restricted rings, box-boundary values, mesh
// interpolation values at time t.
void finish_import(hlbm_ctx* c) {
    const Plan& p = c->p;
    const int pr = p.precision;
    for (int l = 0; l <= p.L; ++l)
        launch_stream_collide(pr, c->kl[l], c->lev(l, 1 - c->cur[l]), c->lev(l, c->cur[l]), c->s);
    for (int l = 0; l < p.L; ++l) {
        const LevelPlan& v = p.lev[l];
        launch_side_init(pr, c->kl[l], v.ci0, v.cj0, v.ci1 - v.ci0, v.cj1 - v.cj0, c->lev(l, 1 - c->cur[l]),
                         c->side(l, c->side_t[l]), c->s);
        launch_fine_to_coarse(pr, c->kl[l], c->kl[l + 1], v.ci0, v.cj0, v.ci1 - v.ci0, v.cj1 - v.cj0,
                              c->lev(l + 1, 1 - c->cur[l + 1]), c->lev(l, c->cur[l]), v.tau, p.lev[l + 1].tau,
                              p.f2c_filter, c->s);
    }
    if (p.has_mesh && p.n_int > 0)
        launch_struct_to_mesh(pr, c->kl[p.L], c->lev(p.L, 1 - c->cur[p.L]), p.n_int,
                              reinterpret_cast<const int32_t*>(c->ws + p.off.uint_don), c->ws + p.off.uint_w,
                              c->prep(c->prep_t), c->s);
    c->dirty = false;
}


// Initial state: f^eq(rho0, u_inf) on every level and mesh node, f^eq(rho0, 0)
// at wall nodes; time and history restart at 0.
int reset_initial_state_checked(hlbm_ctx* c) {
    const Plan& p = c->p;
    for (int l = 0; l < 4; ++l) c->cur[l] = 0, c->side_t[l] = 0;
    c->mesh_cur = 0;
    c->prep_t = 0;
    c->t = 0;
    c->last_check = 0;
    c->poisoned = false;
    const double ux = p.u_inf * std::cos(p.aoa), uy = p.u_inf * std::sin(p.aoa);
    for (int l = 0; l <= p.L; ++l) launch_fill_uniform(p.precision, c->lev(l, 1), c->kl[l], p.rho0, ux, uy, c->s);
    int rc = HLBM_OK;
    if (p.has_mesh) {
        std::vector<double> f0(size_t(kQ) * p.nn);
        const int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1}, cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
        const double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
        for (int P = 0; P < p.nn; ++P) {
            const bool wall = P < p.n_wall && p.wall_bc;
            const double u = wall ? 0.0 : ux, v = wall ? 0.0 : uy;
            for (int q = 0; q < 9; ++q) {
                const double cu = cx[q] * u + cy[q] * v;
                f0[size_t(q) * p.nn + P] = w[q] * p.rho0 * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * (u * u + v * v));
            }
        }
        rc = upload(c, p.off.stage, f0.data(), f0.size() * 8);
        launch_mesh_convert(p.precision, p.nn, c->stage(), c->mesh(0), 1, p.rho0, c->s);
        rc |= hip_check(c, hipStreamSynchronize(c->s), "init");
        if (rc) return HLBM_E_DEVICE;
    }
    finish_import(c);
    return hip_check(c, hipGetLastError(), "kernel launch");
}

void reset_initial_state(hlbm_ctx* c) { (void)reset_initial_state_checked(c); }

void finest_step(hlbm_ctx* c) {
    const Plan& p = c->p;
    const int pr = p.precision, L = p.L;
    if (c->rec) c->rec(c, 2, L);
    void* A = c->lev(L, c->cur[L]);
    void* B = c->lev(L, 1 - c->cur[L]);
    if (p.has_mesh && !p.sint_node.empty()) {
        const double ts = p.lev[L].tau;
        Timed tm(c, HLBM_K_MESH_TO_STRUCT);
        launch_mesh_to_struct(pr, c->kl[L], A, int(p.sint_node.size()),
                              reinterpret_cast<const int32_t*>(c->ws + p.off.sint_node),
                              reinterpret_cast<const int32_t*>(c->ws + p.off.sint_don), c->ws + p.off.sint_w,
                              c->mesh(c->mesh_cur), p.nn, 2.0 * (ts - 1.0) / (2.0 * ts - 1.0), c->s);
    }
    if (c->rec) c->rec(c, 3, L);   // the finest input as the collide-stream reads it
    {
        Timed tm(c, HLBM_K_COLLIDE_L0 + L);
        launch_stream_collide(pr, c->kl[L], A, B, c->s);
    }
    double* slot = c->hist() + 2 * (c->t % p.hist_len);
    if (p.has_mesh) {
        if (p.n_int > 0) {
            Timed tm(c, HLBM_K_STRUCT_TO_MESH);
            launch_struct_to_mesh(pr, c->kl[L], A, p.n_int, reinterpret_cast<const int32_t*>(c->ws + p.off.uint_don),
                                  c->ws + p.off.uint_w, c->prep(1 - c->prep_t), c->s);
        }
        if (c->sub_sink) {
            // every sub-step's state to the sink (fused launches write their
            // intermediate states there too)
            const void* in = c->mesh(c->mesh_cur);
            KMesh km = c->km;
            km.wmom_stride = c->wmom_stride;
            for (int m = 0; m < p.n_sub;) {
                const int k = std::min(p.fv_fuse, p.n_sub - m);
                void* out = c->sub_sink + size_t(m + k - 1) * c->sub_stride;
                km.wmom = c->wmom_sink ? c->wmom_sink + size_t(m) * c->wmom_stride : nullptr;
                if (k > 1)
                    launch_fv_fused(pr, km, in, out, c->prep(c->prep_t), c->prep(1 - c->prep_t), m, k, c->s,
                                    c->sub_sink + size_t(m) * c->sub_stride, c->sub_stride);
                else
                    launch_fv_substep(pr, km, in, out, c->prep(c->prep_t), c->prep(1 - c->prep_t),
                                      double(m) / p.n_sub, c->s);
                in = out;
                m += k;
            }
            (void)hip_check(c, hipMemcpyAsync(c->mesh(c->mesh_cur), in, size_t(kRec) * p.nn * p.elem,
                                              hipMemcpyDeviceToDevice, c->s), "sub-step states");
        } else if (p.fv_fuse > 1) {
            for (int m = 0; m < p.n_sub; m += p.fv_fuse) {
                Timed tm(c, HLBM_K_FV);
                const int k = std::min(p.fv_fuse, p.n_sub - m);
                if (k > 1)
                    launch_fv_fused(pr, c->km, c->mesh(c->mesh_cur), c->mesh(1 - c->mesh_cur), c->prep(c->prep_t),
                                    c->prep(1 - c->prep_t), m, k, c->s);
                else   // a single remaining sub-step: no halo to stage
                    launch_fv_substep(pr, c->km, c->mesh(c->mesh_cur), c->mesh(1 - c->mesh_cur), c->prep(c->prep_t),
                                      c->prep(1 - c->prep_t), double(m) / p.n_sub, c->s);
                c->mesh_cur ^= 1;
            }
        } else {
            for (int m = 0; m < p.n_sub; ++m) {
                Timed tm(c, HLBM_K_FV);
                launch_fv_substep(pr, c->km, c->mesh(c->mesh_cur), c->mesh(1 - c->mesh_cur), c->prep(c->prep_t),
                                  c->prep(1 - c->prep_t), double(m) / p.n_sub, c->s);
                c->mesh_cur ^= 1;
            }
        }
        const double qn = 0.5 * p.rho0 * p.u_inf * p.u_inf * p.chord;
        {
            Timed tm(c, HLBM_K_FORCE);
            launch_wall_force(pr, c->mesh(c->mesh_cur), int(p.wedge.size() / 2),
                              reinterpret_cast<const int32_t*>(c->ws + p.off.wedge),
                              reinterpret_cast<const double*>(c->ws + p.off.wnorm), slot, std::cos(p.aoa),
                              std::sin(p.aoa), qn > 0 ? qn : 1.0, c->s);
        }
        if (c->wstat && !c->rec) {
            const double q = 0.5 * p.rho0 * p.u_inf * p.u_inf;
            Timed tw(c, HLBM_K_WALL_STATS);
            launch_wall_stats(pr, c->mesh(c->mesh_cur), p.n_wall, reinterpret_cast<const double*>(c->ws + p.off.wall_nrm),
                              p.rho0, q > 0 ? 1.0 / q : 1.0, reinterpret_cast<double*>(c->ws + p.off.wsum), c->s);
            c->wstat_n++;
        }
        c->prep_t ^= 1;
    } else if (c->kl[L].n_bounce > 0) {
        // body resolved by bounce-back: momentum exchanged over its links in this step
        const double qn = 0.5 * p.rho0 * p.u_inf * p.u_inf * p.chord;
        Timed tm(c, HLBM_K_FORCE);
        launch_body_force(pr, c->kl[L], A, slot, std::cos(p.aoa), std::sin(p.aoa), qn > 0 ? qn : 1.0, c->s);
    } else {
        // no wall: zero force (the kernel writes 0 for an empty edge list)
        launch_wall_force(pr, c->mesh(0), 0, nullptr, nullptr, slot, 1.0, 0.0, 1.0, c->s);
    }
    c->cur[L] ^= 1;
    c->t++;
}

void level_step(hlbm_ctx* c, int l) {
    const Plan& p = c->p;
    if (l == p.L) {
        finest_step(c);
        return;
    }
    const int pr = p.precision;
    const LevelPlan& v = p.lev[l];
    void* A = c->lev(l, c->cur[l]);
    void* B = c->lev(l, 1 - c->cur[l]);
    if (c->rec) c->rec(c, 0, l);
    {
        Timed tm(c, HLBM_K_COLLIDE_L0 + l);
        launch_stream_collide(pr, c->kl[l], A, B, c->s);
    }
    for (int half = 0; half < 2; ++half) {
        {
            Timed tm(c, HLBM_K_COARSE_TO_FINE);
            launch_coarse_to_fine(pr, c->kl[l], c->kl[l + 1], v.ci0, v.cj0, A, c->lev(l + 1, c->cur[l + 1]),
                              c->side(l, 1 - c->side_t[l]), c->side(l, c->side_t[l]), 0.5 * half, half == 0,
                              v.tau, p.lev[l + 1].tau, c->s);
        }
        if (half == 0 && c->rec) c->rec(c, 1, l);
        level_step(c, l + 1);
    }
    Timed tm(c, HLBM_K_FINE_TO_COARSE);
    launch_fine_to_coarse(pr, c->kl[l], c->kl[l + 1], v.ci0, v.cj0, v.ci1 - v.ci0, v.cj1 - v.cj0,
                          c->lev(l + 1, 1 - c->cur[l + 1]), B, v.tau, p.lev[l + 1].tau, p.f2c_filter, c->s);
    c->side_t[l] ^= 1;
    c->cur[l] ^= 1;
}

}  // namespace

extern "C" {

int hlbm_validate(const hlbm_grid* grid, const hlbm_mesh* mesh, double Re, double tau) {
    Plan p;
    std::string err;
    const int rc = build_plan(grid, mesh, Re, tau, p, err);
    if (rc) g_create_err = err;
    return rc;
}

int hlbm_workspace_size(const hlbm_grid* grid, const hlbm_mesh* mesh, double Re, double tau, size_t* ws_bytes) {
    if (!ws_bytes) return set_err(nullptr, HLBM_E_ARG, "ws_bytes is null");
    Plan p;
    std::string err;
    const int rc = build_plan(grid, mesh, Re, tau, p, err);
    if (rc) return set_err(nullptr, rc, err);
    *ws_bytes = p.off.total;
    return HLBM_OK;
}

int hlbm_create(const hlbm_grid* grid, const hlbm_mesh* mesh, double Re, double tau, void* d_workspace,
                size_t ws_bytes, void* hip_stream, hlbm_ctx** out) {
    if (!out) return set_err(nullptr, HLBM_E_ARG, "out is null");
    *out = nullptr;
    hlbm_ctx* c = new (std::nothrow) hlbm_ctx();
    if (!c) return set_err(nullptr, HLBM_E_ARG, "out of host memory");
    std::string err;
    int rc = build_plan(grid, mesh, Re, tau, c->p, err);
    if (rc) {
        delete c;
        return set_err(nullptr, rc, err);
    }
    if (!d_workspace || (reinterpret_cast<uintptr_t>(d_workspace) & 255) || ws_bytes < c->p.off.total) {
        const size_t need = c->p.off.total;
        delete c;
        return set_err(nullptr, HLBM_E_WORKSPACE,
                       "workspace must be 256-byte aligned and hold " + std::to_string(need) + " bytes");
    }
    if (c->p.fv_fuse > 1) {   // the fused FV tiles against this device's LDS per workgroup
        int dev = 0, lds_max = 0;
        const size_t lds = fv_lds_bytes(c->p.fv_maxl, c->p.fv_maxs, c->p.fv_fuse, c->p.elem);
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
            delete c;
            return set_err(nullptr, HLBM_E_DEVICE, "cannot read the device's LDS per workgroup");
        }
        if (lds > size_t(lds_max)) {
            delete c;
            return set_err(nullptr, HLBM_E_DEVICE,
                           "fused FV tiles need " + std::to_string(lds) + " bytes of LDS per workgroup; the device "
                           "allows " + std::to_string(lds_max) + " (request fewer sub-steps per launch, fv_fuse)");
        }
    }
    c->ws = static_cast<char*>(d_workspace);
    c->ws_bytes = ws_bytes;
    c->s = static_cast<hipStream_t>(hip_stream);
    setup_views(c);
    rc = upload_tables(c);
    if (rc) {
        g_create_err = c->err;
        delete c;
        return rc;
    }
    rc = reset_initial_state_checked(c);
    if (rc) {
        g_create_err = c->err;
        delete c;
        return rc;
    }
    *out = c;
    return HLBM_OK;
}

int hlbm_create_noalloc(const hlbm_grid* grid, const hlbm_mesh* mesh, double Re, double tau, void* hip_stream,
                        hlbm_ctx** out) {
    if (!out) return set_err(nullptr, HLBM_E_ARG, "out is null");
    *out = nullptr;
    size_t need = 0;
    int rc = hlbm_workspace_size(grid, mesh, Re, tau, &need);
    if (rc) return rc;
    if (need > kNoAllocBytes)
        return set_err(nullptr, HLBM_E_WORKSPACE,
                       "problem needs a workspace of " + std::to_string(need) + " bytes; the static workspace of "
                       "hlbm_create_noalloc holds " + std::to_string(kNoAllocBytes));
    void* ws = nullptr;
    rc = noalloc_workspace(&ws);
    if (rc) return set_err(nullptr, rc, "hipGetSymbolAddress of the static workspace failed");
    return hlbm_create(grid, mesh, Re, tau, ws, kNoAllocBytes, hip_stream, out);
}

int hlbm_step(hlbm_ctx* c, int64_t n) {
    if (!c) return HLBM_E_ARG;
    if (c->poisoned) return set_err(c, HLBM_E_STATE, "context poisoned by a non-finite state");
    const int64_t per = int64_t(1) << c->p.L;
    if (n < 0 || n % per) return set_err(c, HLBM_E_ARG, "step count must be a non-negative multiple of 2^n_refine");
    if (c->dirty) finish_import(c);
    for (int64_t b = 0; b < n / per; ++b) {
        level_step(c, 0);
        if (c->p.check_every > 0 && c->t - c->last_check >= c->p.check_every) {
            c->last_check = c->t;
            double v[2];
            int rc = hip_check(c, hipMemcpyAsync(v, c->hist() + 2 * ((c->t - 1) % c->p.hist_len), 16,
                                                 hipMemcpyDeviceToHost, c->s), "check");
            rc |= hip_check(c, hipStreamSynchronize(c->s), "check");
            if (rc) return HLBM_E_DEVICE;
            if (!std::isfinite(v[0]) || !std::isfinite(v[1])) {
                c->poisoned = true;
                return set_err(c, HLBM_E_NONFINITE, "non-finite force at step " + std::to_string(c->t));
            }
        }
    }
    return hip_check(c, hipGetLastError(), "kernel launch");
}

int hlbm_forces(hlbm_ctx* c, double* cd, double* cl) {
    if (!c || !cd || !cl) return HLBM_E_ARG;
    if (c->t == 0) {
        *cd = *cl = 0.0;
        return HLBM_OK;
    }
    return hlbm_force_history(c, c->t - 1, c->t, cd, cl);
}

int hlbm_force_history(hlbm_ctx* c, int64_t t0, int64_t t1, double* cd, double* cl) {
    if (!c || !cd || !cl) return HLBM_E_ARG;
    if (t0 < 0 || t1 > c->t || t0 > t1 || t1 - t0 > c->p.hist_len || t0 < c->t - c->p.hist_len)
        return set_err(c, HLBM_E_ARG, "history range outside the recorded window");
    std::vector<double> buf(size_t(c->p.hist_len) * 2);
    int rc = hip_check(c, hipMemcpyAsync(buf.data(), c->hist(), buf.size() * 8, hipMemcpyDeviceToHost, c->s), "history");
    rc |= hip_check(c, hipStreamSynchronize(c->s), "history");
    if (rc) return HLBM_E_DEVICE;
    for (int64_t t = t0; t < t1; ++t) {
        cd[t - t0] = buf[2 * (t % c->p.hist_len)];
        cl[t - t0] = buf[2 * (t % c->p.hist_len) + 1];
    }
    return HLBM_OK;
}

int hlbm_get_state(hlbm_ctx* c, int32_t part, double* host, size_t count) {
    if (!c || !host) return HLBM_E_ARG;
    const Plan& p = c->p;
    if (part == HLBM_PART_MESH) {
        if (!p.has_mesh || count != size_t(kQ) * p.nn) return set_err(c, HLBM_E_ARG, "bad mesh count");
        launch_mesh_convert(p.precision, p.nn, c->stage(), c->mesh(c->mesh_cur), 0, p.rho0, c->s);
        c->tmp.resize(count);
        int rc = hip_check(c, hipMemcpyAsync(c->tmp.data(), c->stage(), count * 8, hipMemcpyDeviceToHost, c->s), "get");
        rc |= hip_check(c, hipStreamSynchronize(c->s), "get");
        if (rc) return HLBM_E_DEVICE;
        for (int q = 0; q < kQ; ++q)
            for (int P = 0; P < p.nn; ++P) host[size_t(q) * p.nn + p.perm[P]] = c->tmp[size_t(q) * p.nn + P];
        return HLBM_OK;
    }
    if (part < 0 || part > p.L) return set_err(c, HLBM_E_ARG, "bad part");
    const LevelPlan& v = p.lev[part];
    if (count != size_t(kQ) * v.nx * v.ny) return set_err(c, HLBM_E_ARG, "bad level count");
    const int rows = int(std::max<size_t>(1, p.stage_bytes / (size_t(kQ) * v.nx * 8)));
    for (int j0 = 0; j0 < v.ny; j0 += rows) {
        const int j1 = std::min(v.ny, j0 + rows);
        launch_export_level(p.precision, c->kl[part], c->lev(part, 1 - c->cur[part]), c->stage(), j0, j1, c->s);
        const size_t n = size_t(kQ) * (j1 - j0) * v.nx;
        c->tmp.resize(n);
        int rc = hip_check(c, hipMemcpyAsync(c->tmp.data(), c->stage(), n * 8, hipMemcpyDeviceToHost, c->s), "get");
        rc |= hip_check(c, hipStreamSynchronize(c->s), "get");
        if (rc) return HLBM_E_DEVICE;
        for (int q = 0; q < kQ; ++q)
            std::memcpy(host + (size_t(q) * v.ny + j0) * v.nx, c->tmp.data() + size_t(q) * (j1 - j0) * v.nx,
                        size_t(j1 - j0) * v.nx * 8);
    }
    return HLBM_OK;
}

int hlbm_set_state(hlbm_ctx* c, int32_t part, const double* host, size_t count) {
    if (!c || !host) return HLBM_E_ARG;
    if (c->poisoned) return set_err(c, HLBM_E_STATE, "context poisoned by a non-finite state");
    const Plan& p = c->p;
    c->wstat = false;
    if (part == HLBM_PART_MESH) {
        if (!p.has_mesh || count != size_t(kQ) * p.nn) return set_err(c, HLBM_E_ARG, "bad mesh count");
        c->tmp.resize(count);
        for (int q = 0; q < kQ; ++q)
            for (int P = 0; P < p.nn; ++P) c->tmp[size_t(q) * p.nn + P] = host[size_t(q) * p.nn + p.perm[P]];
        int rc = hip_check(c, hipMemcpyAsync(c->stage(), c->tmp.data(), count * 8, hipMemcpyHostToDevice, c->s), "set");
        launch_mesh_convert(p.precision, p.nn, c->stage(), c->mesh(c->mesh_cur), 1, p.rho0, c->s);
        rc |= hip_check(c, hipStreamSynchronize(c->s), "set");
        if (rc) return HLBM_E_DEVICE;
        c->dirty = true;
        return HLBM_OK;
    }
    if (part < 0 || part > p.L) return set_err(c, HLBM_E_ARG, "bad part");
    const LevelPlan& v = p.lev[part];
    if (count != size_t(kQ) * v.nx * v.ny) return set_err(c, HLBM_E_ARG, "bad level count");
    const int rows = int(std::max<size_t>(1, p.stage_bytes / (size_t(kQ) * v.nx * 8)));
    for (int j0 = 0; j0 < v.ny; j0 += rows) {
        const int j1 = std::min(v.ny, j0 + rows);
        const size_t n = size_t(kQ) * (j1 - j0) * v.nx;
        c->tmp.resize(n);
        for (int q = 0; q < kQ; ++q)
            std::memcpy(c->tmp.data() + size_t(q) * (j1 - j0) * v.nx, host + (size_t(q) * v.ny + j0) * v.nx,
                        size_t(j1 - j0) * v.nx * 8);
        int rc = hip_check(c, hipMemcpyAsync(c->stage(), c->tmp.data(), n * 8, hipMemcpyHostToDevice, c->s), "set");
        launch_import_level(p.precision, c->kl[part], c->lev(part, 1 - c->cur[part]), c->stage(), j0, j1, c->s);
        rc |= hip_check(c, hipStreamSynchronize(c->s), "set");
        if (rc) return HLBM_E_DEVICE;
    }
    c->dirty = true;
    return HLBM_OK;
}

int hlbm_info(hlbm_ctx* c, hlbm_info_t* o) {
    if (!c || !o) return HLBM_E_ARG;
    const Plan& p = c->p;
    std::memset(o, 0, sizeof(*o));
    o->n_levels = p.nlev;
    o->n_sub = p.n_sub;
    const int64_t E = int64_t(p.elem);
    int64_t bytes = 0;
    for (int l = 0; l <= p.L; ++l) {
        o->nx[l] = p.lev[l].nx;
        o->ny[l] = p.lev[l].ny;
        o->pitch[l] = p.lev[l].pitch;
        o->tau[l] = p.lev[l].tau;
        o->active_nodes[l] = p.lev[l].active;
        o->k1_bytes[l] = p.lev[l].active * 2 * kQ * E;
        bytes += o->k1_bytes[l] << l;   // level l runs 2^l times per base step
    }
    o->tau_u = p.tau_u;
    o->n_mesh_nodes = p.nn;
    o->n_wall_nodes = p.n_wall;
    o->n_interp_mesh = p.n_int;
    o->n_interp_struct = int(p.sint_node.size());
    o->n_fallback = p.n_fallback;
    o->n_wall_edges = int(p.wedge.size() / 2);
    o->nnz = int(p.col.size());
    // FV sub-step of eq. (3), algorithmic: per node 9 populations in and out, its own
    // (G_x, G_y, C) and a row pointer; per neighbour entry a column index and (G_x, G_y, C)
    const int64_t nn = p.nn, nbr = int64_t(p.col.size()) - nn;
    o->fv_bytes = nn * (2 * kQ * E + 3 * E + 4) + nbr * (4 + 3 * E);
    // what this layout moves: records with stored moments in and out, every padded table slot
    o->fv_layout_bytes = nn * 2 * kRec * E + nn * p.ell_width * (E == 8 ? 32 : 16);
    o->n_solid = p.n_solid;
    o->n_bounce = int32_t(p.bounce_node.size());
    o->bytes_per_finest_step = bytes / (int64_t(1) << p.L) + int64_t(p.n_sub) * o->fv_bytes;
    o->t = c->t;
    o->workspace_bytes = p.off.total;
    o->fv_fuse = p.has_mesh ? p.fv_fuse : 0;
    const bool fused = p.has_mesh && p.fv_fuse > 1;
    o->fv_tiles = fused ? p.n_tiles : 0;
    o->fv_tile_nodes = fused ? p.fv_tile : 0;
    o->fv_threads = fused ? p.fv_threads : 0;
    return HLBM_OK;
}

int hlbm_wall_stats_begin(hlbm_ctx* c) {
    if (!c) return HLBM_E_ARG;
    if (c->poisoned) return set_err(c, HLBM_E_STATE, "context poisoned by a non-finite state");
    const Plan& p = c->p;
    if (!p.has_mesh || p.n_wall == 0) return set_err(c, HLBM_E_ARG, "no wall nodes");
    launch_zero(reinterpret_cast<double*>(c->ws + p.off.wsum), size_t(3) * p.n_wall, c->s);
    c->wstat = true;
    c->wstat_n = 0;
    return hip_check(c, hipGetLastError(), "wall statistics");
}

int hlbm_wall_stats(hlbm_ctx* c, int64_t* n_steps, double* cp, double* cf, double* cn) {
    if (!c || !n_steps || !cp || !cf) return HLBM_E_ARG;
    const Plan& p = c->p;
    if (!c->wstat || c->wstat_n == 0) return set_err(c, HLBM_E_STATE, "no wall statistics accumulated");
    double* out = reinterpret_cast<double*>(c->ws + p.off.wout);
    launch_wall_stats_final(p.n_wall, reinterpret_cast<const double*>(c->ws + p.off.wsum),
                            reinterpret_cast<const int32_t*>(c->ws + p.off.wall_slot), double(c->wstat_n), out, c->s);
    std::vector<double> h(size_t(3) * p.n_wall);
    int rc = hip_check(c, hipMemcpyAsync(h.data(), out, h.size() * 8, hipMemcpyDeviceToHost, c->s), "wall statistics");
    rc |= hip_check(c, hipStreamSynchronize(c->s), "wall statistics");
    if (rc) return HLBM_E_DEVICE;
    std::memcpy(cp, h.data(), size_t(p.n_wall) * 8);
    std::memcpy(cf, h.data() + p.n_wall, size_t(p.n_wall) * 8);
    if (cn) std::memcpy(cn, h.data() + 2 * size_t(p.n_wall), size_t(p.n_wall) * 8);
    *n_steps = c->wstat_n;
    return HLBM_OK;
}

int hlbm_profile(hlbm_ctx* c, int enable) {
    if (!c) return HLBM_E_ARG;
    c->prof = enable != 0;
    return HLBM_OK;
}

int hlbm_profile_read(hlbm_ctx* c, double* ms, int64_t* launches) {
    if (!c || !ms || !launches) return HLBM_E_ARG;
    for (int k = 0; k < HLBM_K_COUNT; ++k) ms[k] = 0.0, launches[k] = 0;
    int rc = hip_check(c, hipStreamSynchronize(c->s), "profile");
    for (auto& e : c->ev_pending) {
        float t = 0.0f;
        if (hipEventElapsedTime(&t, e.second.first, e.second.second) == hipSuccess) {
            ms[e.first] += t;
            launches[e.first] += 1;
        }
        c->ev_pool.push_back(e.second.first);
        c->ev_pool.push_back(e.second.second);
    }
    c->ev_pending.clear();
    return rc;
}

int hlbm_kernel_bench(hlbm_ctx* c, int kclass, int n, double* avg_ms) {
    if (!c || !avg_ms || n <= 0) return HLBM_E_ARG;
    const Plan& p = c->p;
    const bool fv = kclass == HLBM_K_FV;
    const int l = kclass - HLBM_K_COLLIDE_L0;
    if (!fv && (l < 0 || l > p.L)) return set_err(c, HLBM_E_ARG, "unsupported kernel class");
    if (fv && !p.has_mesh) return set_err(c, HLBM_E_ARG, "no mesh");
    if (c->dirty) finish_import(c);
    hipEvent_t a = take_event(c), b = take_event(c);
    if (!a || !b) return set_err(c, HLBM_E_DEVICE, "hipEventCreate failed");
    int rc = hip_check(c, hipEventRecord(a, c->s), "event");
    for (int k = 0; k < n; ++k) {
        if (fv && p.fv_fuse > 1) {
            launch_fv_fused(p.precision, c->km, c->mesh(c->mesh_cur), c->mesh(1 - c->mesh_cur), c->prep(c->prep_t),
                            c->prep(1 - c->prep_t), 0, std::min(p.fv_fuse, p.n_sub), c->s);
            c->mesh_cur ^= 1;
        } else if (fv) {
            launch_fv_substep(p.precision, c->km, c->mesh(c->mesh_cur), c->mesh(1 - c->mesh_cur), c->prep(c->prep_t),
                              c->prep(1 - c->prep_t), double(k % p.n_sub) / p.n_sub, c->s);
            c->mesh_cur ^= 1;
        } else {
            launch_stream_collide(p.precision, c->kl[l], c->lev(l, c->cur[l]), c->lev(l, 1 - c->cur[l]), c->s);
            c->cur[l] ^= 1;
        }
    }
    rc |= hip_check(c, hipEventRecord(b, c->s), "event");
    rc |= hip_check(c, hipEventSynchronize(b), "event");
    float ms = 0.0f;
    rc |= hip_check(c, hipEventElapsedTime(&ms, a, b), "event");
    c->ev_pool.push_back(a);
    c->ev_pool.push_back(b);
    *avg_ms = double(ms) / n;
    return rc ? HLBM_E_DEVICE : HLBM_OK;
}

const char* hlbm_last_error(const hlbm_ctx* c) { return c ? c->err.c_str() : g_create_err.c_str(); }

void hlbm_destroy(hlbm_ctx* c) {
    if (!c) return;
    if (!c->ev_pending.empty()) (void)hipStreamSynchronize(c->s);
    for (auto& e : c->ev_pending) c->ev_pool.push_back(e.second.first), c->ev_pool.push_back(e.second.second);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    adj_free(c->adj);
    delete c;
}

}  // extern "C"
