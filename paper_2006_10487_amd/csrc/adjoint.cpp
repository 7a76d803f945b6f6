// adjoint.cpp -- objective run and discrete adjoint of the HLBM step.
//
// Objective: J = mean over finest steps h in [t0, t1) of w_cd C_D(h) + w_cl C_L(h)
// (eqs. (10)-(11)), for a run of t_end finest steps from the initial state.
// Gradient: dJ/d(angle of attack) and dJ/d(tau) with the number of FV
// sub-steps held fixed.  Reverse mode over the exact sequence of GPU kernels
// of the forward step (single structured level, FP64):
//   forward   K5 (eq. 4) -> collide-stream -> K6 (eq. 9) -> n FV sub-steps -> force
//   reverse   force^T -> FV^T (n sub-steps, states recomputed) -> K6^T + collide^T
//             + boundary^T + pull^T -> K5^T
// Memory: revolve-style two-level checkpointing: the forward stores the state
// every K steps; the reverse sweep recomputes each K-step segment forward from
// its checkpoint (storing every step of the segment) and, inside every step,
// the n sub-step states from the step's mesh state.
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "hlbm_internal.h"

using namespace hlbm;

struct AdjState {
    hlbm_objective obj{};
    char* ws = nullptr;
    size_t bytes = 0;
    size_t lev_bytes = 0, mesh_bytes = 0, prep_bytes = 0, adjlev_bytes = 0, adjmesh_bytes = 0;
    int n_ckpt = 0, seg_len = 0, n_slots = 0, nd6 = 0;
    struct {
        size_t ckpt, seg_lev, seg_mesh, seg_prep, sub, awork, abar[2], prebar, mbar[2], zbar, pbar[2], m5bar;
        size_t partial, acc, tedges, vwall, t5ptr, t5s, t5w, t6node, t6ptr, t6s, t6w, dfeq;
        size_t gbar, vbar, w5bar, w6bar, total;
    } off{};
    bool tables = false, ran = false;
    std::vector<int32_t> t5map, t6map;   // transposed entry -> index into sint_w / uint_w
    double J = 0.0;
    std::vector<double> cd, cl;
    template <typename T> T* at(size_t o) { return reinterpret_cast<T*>(ws + o); }
};

namespace {

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

int check_supported(hlbm_ctx* c, const hlbm_objective* o) {
    const Plan& p = c->p;
    if (!o) return set_err(c, HLBM_E_ARG, "objective is null");
    if (p.precision != HLBM_FP64) return set_err(c, HLBM_E_ARG, "the adjoint runs in FP64 contexts");
    if (p.L != 0) return set_err(c, HLBM_E_ARG, "the adjoint covers a single structured level (n_refine = 0)");
    if (!p.has_mesh || p.wedge.empty()) return set_err(c, HLBM_E_ARG, "the adjoint needs a mesh with a wall");
    if (o->t_end <= 0 || o->t0 < 0 || o->t1 <= o->t0 || o->t1 > o->t_end || o->ckpt_every <= 0)
        return set_err(c, HLBM_E_ARG, "objective window must satisfy 0 <= t0 < t1 <= t_end, ckpt_every > 0");
    if (o->t_end > p.hist_len) return set_err(c, HLBM_E_ARG, "t_end exceeds the force history length");
    return HLBM_OK;
}

// Workspace layout of the objective run and the reverse sweep.
void layout(hlbm_ctx* c, AdjState& a) {
    const Plan& p = c->p;
    const LevelPlan& v = p.lev[0];
    const int K = int(a.obj.ckpt_every);
    a.seg_len = K;
    a.n_ckpt = int((a.obj.t_end + K - 1) / K);
    a.lev_bytes = size_t(kQ) * v.ny * v.pitch * 8;
    a.mesh_bytes = size_t(kRec) * p.nn * 8;
    a.prep_bytes = size_t(std::max(p.n_int, 1)) * kMacro * 8;
    a.adjlev_bytes = a.lev_bytes;
    a.adjmesh_bytes = size_t(kQ) * p.nn * 8;
    const size_t ck = a256(a.lev_bytes) + a256(a.mesh_bytes) + a256(a.prep_bytes);
    size_t off = 0;
    auto take = [&](size_t b) { const size_t o = off; off = a256(off + std::max<size_t>(b, 8)); return o; };
    a.off.ckpt = take(ck * a.n_ckpt);
    a.off.seg_lev = take(a256(a.lev_bytes) * K);
    a.off.seg_mesh = take(a256(a.mesh_bytes) * K);
    a.off.seg_prep = take(a256(a.prep_bytes) * (K + 1));
    a.off.sub = take(a256(a.mesh_bytes) * (p.n_sub + 1));
    a.off.awork = take(a.lev_bytes);
    a.off.abar[0] = take(a.adjlev_bytes);
    a.off.abar[1] = take(a.adjlev_bytes);
    a.off.prebar = take(a.adjlev_bytes);
    a.off.mbar[0] = take(a.adjmesh_bytes);
    a.off.mbar[1] = take(a.adjmesh_bytes);
    a.off.zbar = take(a.adjmesh_bytes);
    a.off.pbar[0] = take(a.prep_bytes);
    a.off.pbar[1] = take(a.prep_bytes);
    a.off.m5bar = take(std::max<size_t>(p.sint_node.size(), 1) * kMacro * 8);
    // partial-sum slots of one reverse step (the largest user)
    const int bn = adj_blocks_nodes(p.nn), bi = adj_blocks_nodes(p.n_int);
    const int bc = adj_blocks_nodes(2 * (v.nx - 2)) + adj_blocks_nodes(2 * (v.ny - 2)) + 1;
    a.n_slots = p.n_sub * (bn + bi) + adj_blocks_collide(c->kl[0]) + bc +
                adj_blocks_nodes(int(p.sint_node.size())) + adj_blocks_nodes(int(v.ny) * 9 * v.pitch + p.nn) + 64;
    a.off.partial = take(size_t(a.n_slots) * 2 * 8);
    a.off.acc = take(2 * 8);
    a.off.tedges = take(size_t(p.ell_width) * p.nn * 32);
    a.off.vwall = take(size_t(2) * std::max(p.n_wall, 1) * 8);
    a.off.t5ptr = take(size_t(p.nn + 1) * 4);
    a.off.t5s = take(std::max<size_t>(p.sint_don.size(), 1) * 4);
    a.off.t5w = take(std::max<size_t>(p.sint_don.size(), 1) * 8);
    a.off.t6node = take(std::max<size_t>(p.uint_don.size(), 1) * 4);
    a.off.t6ptr = take((std::max<size_t>(p.uint_don.size(), 1) + 1) * 4);
    a.off.t6s = take(std::max<size_t>(p.uint_don.size(), 1) * 4);
    a.off.t6w = take(std::max<size_t>(p.uint_don.size(), 1) * 8);
    a.off.dfeq = take(9 * 8);
    if (a.obj.mesh_grad) {
        a.off.gbar = take(size_t(3) * p.ell_width * p.nn * 8);
        a.off.vbar = take(size_t(2) * std::max(p.n_wall, 1) * 8);
        a.off.w5bar = take(std::max<size_t>(p.sint_don.size(), 1) * 8);
        a.off.w6bar = take(std::max<size_t>(p.uint_don.size(), 1) * 8);
    }
    a.off.total = off;
}

size_t ckpt_lev(const AdjState& a, int k) {
    return a.off.ckpt + size_t(k) * (a256(a.lev_bytes) + a256(a.mesh_bytes) + a256(a.prep_bytes));
}
size_t ckpt_mesh(const AdjState& a, int k) { return ckpt_lev(a, k) + a256(a.lev_bytes); }
size_t ckpt_prep(const AdjState& a, int k) { return ckpt_mesh(a, k) + a256(a.mesh_bytes); }

int d2d(hlbm_ctx* c, void* dst, const void* src, size_t bytes) {
    return hip_check(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c->s), "hipMemcpyAsync");
}

// Transposed tables of the reverse sweep, built from the plan.
int upload_tables(hlbm_ctx* c, AdjState& a) {
    const Plan& p = c->p;
    const int nn = p.nn, W = p.ell_width;
    // FV transpose: slot z of node k = (P, G_Pk, C_Pk) for the pivots P whose row holds k;
    // slot 0 = (k, sum_{j != k} G_kj, C_kk) (the pivot's own base and collision terms)
    std::vector<std::vector<std::array<double, 4>>> rows(nn);
    for (int P = 0; P < nn; ++P) {
        double sx = 0.0, sy = 0.0, ckk = 0.0;
        for (int z = p.rowptr[P]; z < p.rowptr[P + 1]; ++z) {
            if (p.col[z] == P) {
                ckk = p.cc[z];
                continue;
            }
            sx += p.gx[z];
            sy += p.gy[z];
            rows[p.col[z]].push_back({double(P), p.gx[z], p.gy[z], p.cc[z]});
        }
        rows[P].insert(rows[P].begin(), {double(P), sx, sy, ckk});
    }
    std::vector<char> te(size_t(W) * nn * 32, 0);
    for (int k = 0; k < nn; ++k) {
        if (int(rows[k].size()) > W) return set_err(c, HLBM_E_GEOMETRY, "mesh connectivity is not symmetric");
        for (int z = 0; z < W; ++z) {
            char* r = te.data() + (size_t(z) * nn + k) * 32;
            const int32_t col = z < int(rows[k].size()) ? int32_t(rows[k][z][0]) : -1;
            std::memcpy(r, &col, 4);
            if (col >= 0) std::memcpy(r + 8, &rows[k][z][1], 24);
        }
    }
    // wall force weights: half the outward normals of the wall edges at each wall node
    std::vector<double> vw(size_t(2) * std::max(p.n_wall, 1), 0.0);
    for (size_t e = 0; e < p.wedge.size() / 2; ++e)
        for (int s = 0; s < 2; ++s) {
            const int P = p.wedge[2 * e + s];
            vw[2 * P] += 0.5 * p.wnorm[2 * e];
            vw[2 * P + 1] += 0.5 * p.wnorm[2 * e + 1];
        }
    // eq. (4) transpose: mesh donor -> (structured interpolation node, weight)
    std::vector<int32_t> t5ptr(nn + 1, 0), t5s;
    std::vector<double> t5w;
    a.t5map.clear();
    {
        std::vector<std::vector<std::pair<int, int>>> lst(nn);   // (s, d)
        for (size_t s = 0; s < p.sint_node.size(); ++s)
            for (int d = 0; d < kSDon; ++d) {
                const int k = p.sint_don[s * kSDon + d];
                if (k >= 0) lst[k].push_back({int(s), d});
            }
        for (int k = 0; k < nn; ++k) {
            for (auto& pr : lst[k]) {
                t5s.push_back(pr.first);
                t5w.push_back(p.sint_w[size_t(pr.first) * kSDon + pr.second]);
                a.t5map.push_back(pr.first * kSDon + pr.second);
            }
            t5ptr[k + 1] = int(t5s.size());
        }
    }
    // eq. (9) transpose: structured donor -> (mesh interpolation slot, weight)
    std::vector<int32_t> t6node, t6ptr{0}, t6s;
    std::vector<double> t6w;
    a.t6map.clear();
    {
        std::map<int, std::vector<std::pair<int, int>>> lst;   // (slot, d)
        for (int s = 0; s < p.n_int; ++s)
            for (int d = 0; d < kUDon; ++d) {
                const int id = p.uint_don[size_t(s) * kUDon + d];
                if (id >= 0) lst[id].push_back({s, d});
            }
        for (auto& kv : lst) {
            t6node.push_back(kv.first);
            for (auto& pr : kv.second) {
                t6s.push_back(pr.first);
                t6w.push_back(p.uint_w[size_t(pr.first) * kUDon + pr.second]);
                a.t6map.push_back(pr.first * kUDon + pr.second);
            }
            t6ptr.push_back(int(t6s.size()));
        }
        a.nd6 = int(t6node.size());
    }
    auto up = [&](size_t off, const void* src, size_t b) {
        return b ? hip_check(c, hipMemcpyAsync(a.ws + off, src, b, hipMemcpyHostToDevice, c->s), "upload") : 0;
    };
    int rc = up(a.off.tedges, te.data(), te.size());
    rc |= up(a.off.vwall, vw.data(), vw.size() * 8);
    rc |= up(a.off.t5ptr, t5ptr.data(), t5ptr.size() * 4);
    rc |= up(a.off.t5s, t5s.data(), t5s.size() * 4);
    rc |= up(a.off.t5w, t5w.data(), t5w.size() * 8);
    rc |= up(a.off.t6node, t6node.data(), t6node.size() * 4);
    rc |= up(a.off.t6ptr, t6ptr.data(), t6ptr.size() * 4);
    rc |= up(a.off.t6s, t6s.data(), t6s.size() * 4);
    rc |= up(a.off.t6w, t6w.data(), t6w.size() * 8);
    rc |= hip_check(c, hipStreamSynchronize(c->s), "upload");
    if (rc) return HLBM_E_DEVICE;
    a.tables = true;
    return HLBM_OK;
}

KAdj make_kadj(hlbm_ctx* c, AdjState& a) {
    const Plan& p = c->p;
    KAdj K;
    K.L = c->kl[0];
    K.M = c->km;
    K.tedges = a.ws + a.off.tedges;
    const double tau = p.tau_s, tu = p.tau_u;
    K.dt = p.dt_u;
    K.dtt = p.dt_u / tu;
    K.ddtt_dtau = -p.dt_u / (tu * tu);
    K.cst = 1.0 - 1.0 / (2.0 * tau);
    K.dcst_dtau = 1.0 / (2.0 * tau * tau);
    K.omega = 1.0 / tau;
    K.domega_dtau = -1.0 / (tau * tau);
    K.phi = 2.0 * (tau - 1.0) / (2.0 * tau - 1.0);
    K.dphi_dtau = 2.0 / ((2.0 * tau - 1.0) * (2.0 * tau - 1.0));
    K.uin_x = p.u_inf * std::cos(p.aoa);
    K.uin_y = p.u_inf * std::sin(p.aoa);
    K.duin_x = -p.u_inf * std::sin(p.aoa);
    K.duin_y = p.u_inf * std::cos(p.aoa);
    K.partial = a.at<double>(a.off.partial);
    const bool g = a.obj.mesh_grad != 0;
    K.gbar = g ? a.at<double>(a.off.gbar) : nullptr;
    K.vbar = g ? a.at<double>(a.off.vbar) : nullptr;
    K.w5bar = g ? a.at<double>(a.off.w5bar) : nullptr;
    K.w6bar = g ? a.at<double>(a.off.w6bar) : nullptr;
    return K;
}

// One reverse step: adjoint of finest step t, whose stored inputs are segment slot k.
void reverse_step(hlbm_ctx* c, AdjState& a, const KAdj& K, int64_t t, int k, int& ab, int& mb, int& pb,
                  double& alpha_host) {
    const Plan& p = c->p;
    const hlbm_objective& o = a.obj;
    hipStream_t s = c->s;
    const double* Mt = a.at<double>(a.off.seg_mesh + a256(a.mesh_bytes) * k);
    const double* prep0 = a.at<double>(a.off.seg_prep + a256(a.prep_bytes) * k);
    const double* prep1 = a.at<double>(a.off.seg_prep + a256(a.prep_bytes) * (k + 1));
    double* Aw = a.at<double>(a.off.awork);
    double* Bbar = a.at<double>(a.off.abar[ab]);
    double* Anew = a.at<double>(a.off.abar[1 - ab]);
    double* prebar = a.at<double>(a.off.prebar);
    double* Pcur = a.at<double>(a.off.pbar[pb]);       // adjoint of prep(t+1)
    double* Pnext = a.at<double>(a.off.pbar[1 - pb]);  // adjoint of prep(t)
    int slot = 0;
    // A as read by the collide-stream kernel: stored post(t) with eq. (4) applied
    (void)d2d(c, Aw, a.ws + a.off.seg_lev + a256(a.lev_bytes) * k, a.lev_bytes);
    if (!p.sint_node.empty()) {
        const double ts = p.tau_s;
        launch_mesh_to_struct(HLBM_FP64, c->kl[0], Aw, int(p.sint_node.size()),
                              reinterpret_cast<const int32_t*>(c->ws + p.off.sint_node),
                              reinterpret_cast<const int32_t*>(c->ws + p.off.sint_don), c->ws + p.off.sint_w, Mt,
                              p.nn, 2.0 * (ts - 1.0) / (2.0 * ts - 1.0), s);
    }
    // sub-step states M^0..M^n of this step
    const size_t ms = a256(a.mesh_bytes);
    (void)d2d(c, a.ws + a.off.sub, Mt, a.mesh_bytes);
    for (int m = 0; m < p.n_sub; ++m)
        launch_fv_substep(HLBM_FP64, c->km, a.ws + a.off.sub + ms * m, a.ws + a.off.sub + ms * (m + 1), prep0, prep1,
                          double(m) / p.n_sub, s);
    // force^T (history entry t belongs to the state after step t, M^n)
    if (t >= o.t0 && t < o.t1) {
        const double span = double(o.t1 - o.t0);
        const double jcd = o.w_cd / span, jcl = o.w_cl / span;   // times J_bar, applied below via scaling
        const double qn = 0.5 * p.rho0 * p.u_inf * p.u_inf * p.chord;
        const double ca = std::cos(p.aoa), sa = std::sin(p.aoa);
        launch_adj_force(K, a.at<double>(a.off.mbar[mb]), a.at<double>(a.off.vwall), (jcd * ca - jcl * sa) / qn,
                         (jcd * sa + jcl * ca) / qn, a.at<double>(a.off.sub + ms * p.n_sub), s);
        // projection directions depend on alpha: dC_D/dalpha = C_L, dC_L/dalpha = -C_D
        alpha_host += jcd * a.cl[t] - jcl * a.cd[t];
    }
    // FV^T, last sub-step first
    const int bn = adj_blocks_nodes(p.nn), bi = adj_blocks_nodes(p.n_int);
    for (int m = p.n_sub - 1; m >= 0; --m) {
        const double th = double(m) / p.n_sub;
        const double* Mm = a.at<double>(a.off.sub + ms * m);
        launch_adj_fv_a(K, Mm, a.at<double>(a.off.mbar[mb]), a.at<double>(a.off.zbar), prep0, prep1, th, slot, s);
        slot += bn;
        launch_adj_fv_b(K, Mm, a.at<double>(a.off.zbar), a.at<double>(a.off.mbar[1 - mb]), s);
        if (p.n_int > 0) {
            launch_adj_fv_c(K, a.at<double>(a.off.zbar), prep0, prep1, th, Pnext, Pcur, slot, s);
            slot += bi;
        }
        mb ^= 1;
    }
    // collide-stream^T with eq. (9)^T and the boundary conditions^T, then pull^T
    launch_adj_collide(K, Aw, Bbar, prebar, slot, s);
    slot += adj_blocks_collide(c->kl[0]);
    launch_adj_s2m(K, Aw, a.nd6, a.at<int32_t>(a.off.t6node), a.at<int32_t>(a.off.t6ptr), a.at<int32_t>(a.off.t6s),
                   a.at<double>(a.off.t6w), Pcur, prebar, s);
    launch_adj_bc(K, Aw, prebar, slot, s);
    slot += adj_blocks_nodes(2 * (c->kl[0].nx - 2)) + adj_blocks_nodes(2 * (c->kl[0].ny - 2)) + 1;
    launch_adj_push(K, prebar, Anew, s);
    // eq. (4)^T
    if (!p.sint_node.empty()) {
        launch_adj_m2s_a(K, Mt, int(p.sint_node.size()), reinterpret_cast<const int32_t*>(c->ws + p.off.sint_node),
                         reinterpret_cast<const int32_t*>(c->ws + p.off.sint_don),
                         reinterpret_cast<const double*>(c->ws + p.off.sint_w), Anew, a.at<double>(a.off.m5bar), slot, s);
        slot += adj_blocks_nodes(int(p.sint_node.size()));
        launch_adj_m2s_b(K, Mt, a.at<int32_t>(a.off.t5ptr), a.at<int32_t>(a.off.t5s), a.at<double>(a.off.t5w),
                         a.at<double>(a.off.m5bar), a.at<double>(a.off.mbar[mb]), s);
    }
    launch_reduce_partials(a.at<double>(a.off.partial), slot, a.at<double>(a.off.acc), s);
    // carried adjoints: post(t), M_t, prep(t)
    ab ^= 1;
    launch_zero(Pcur, a.prep_bytes / 8, s);
    pb ^= 1;
}

}  // namespace

namespace hlbm {
void adj_free(AdjState* a) { delete a; }
}  // namespace hlbm

extern "C" {

int hlbm_objective_workspace_size(hlbm_ctx* c, const hlbm_objective* o, size_t* bytes) {
    if (!c || !bytes) return HLBM_E_ARG;
    const int rc = check_supported(c, o);
    if (rc) return rc;
    AdjState a;
    a.obj = *o;
    layout(c, a);
    *bytes = a.off.total;
    return HLBM_OK;
}

int hlbm_run_objective(hlbm_ctx* c, const hlbm_objective* o, void* d_ckpt, size_t ckpt_bytes, double* J) {
    if (!c || !J) return HLBM_E_ARG;
    int rc = check_supported(c, o);
    if (rc) return rc;
    if (!c->adj) c->adj = new AdjState();
    AdjState& a = *c->adj;
    const bool same_ws = a.ws == static_cast<char*>(d_ckpt);
    a.obj = *o;
    a.ran = false;
    layout(c, a);
    if (!d_ckpt || (reinterpret_cast<uintptr_t>(d_ckpt) & 255) || ckpt_bytes < a.off.total)
        return set_err(c, HLBM_E_WORKSPACE, "objective workspace must be 256-byte aligned and hold " +
                                                std::to_string(a.off.total) + " bytes");
    if (!same_ws) a.tables = false;
    a.ws = static_cast<char*>(d_ckpt);
    a.bytes = ckpt_bytes;
    if (!a.tables && (rc = upload_tables(c, a))) return rc;
    reset_initial_state(c);
    const Plan& p = c->p;
    const int K = int(o->ckpt_every);
    for (int64_t t = 0; t < o->t_end; ++t) {
        if (t % K == 0) {
            const int k = int(t / K);
            rc |= d2d(c, a.ws + ckpt_lev(a, k), c->lev(0, c->cur[0]), a.lev_bytes);
            rc |= d2d(c, a.ws + ckpt_mesh(a, k), c->mesh(c->mesh_cur), a.mesh_bytes);
            rc |= d2d(c, a.ws + ckpt_prep(a, k), c->prep(c->prep_t), a.prep_bytes);
        }
        finest_step(c);
    }
    if (rc) return HLBM_E_DEVICE;
    a.cd.assign(size_t(o->t_end), 0.0);
    a.cl.assign(size_t(o->t_end), 0.0);
    rc = hlbm_force_history(c, 0, o->t_end, a.cd.data(), a.cl.data());
    if (rc) return rc;
    double s = 0.0;
    for (int64_t h = o->t0; h < o->t1; ++h) s += o->w_cd * a.cd[h] + o->w_cl * a.cl[h];
    a.J = s / double(o->t1 - o->t0);
    *J = a.J;
    a.ran = true;
    (void)p;
    return hip_check(c, hipGetLastError(), "objective");
}

int hlbm_adjoint(hlbm_ctx* c, double J_bar, double* grad, double* grad_xy) {
    if (!c || !grad) return HLBM_E_ARG;
    if (!c->adj || !c->adj->ran) return set_err(c, HLBM_E_STATE, "hlbm_run_objective must run first");
    AdjState& a = *c->adj;
    if ((grad_xy != nullptr) != (a.obj.mesh_grad != 0))
        return set_err(c, HLBM_E_ARG, "grad_xy must be given exactly when the objective asked for mesh_grad");
    const Plan& p = c->p;
    const hlbm_objective& o = a.obj;
    hipStream_t s = c->s;
    const KAdj K = make_kadj(c, a);
    for (double* z : {a.at<double>(a.off.abar[0]), a.at<double>(a.off.abar[1]), a.at<double>(a.off.prebar)})
        launch_zero(z, a.adjlev_bytes / 8, s);
    for (double* z : {a.at<double>(a.off.mbar[0]), a.at<double>(a.off.mbar[1]), a.at<double>(a.off.zbar)})
        launch_zero(z, a.adjmesh_bytes / 8, s);
    launch_zero(a.at<double>(a.off.pbar[0]), a.prep_bytes / 8, s);
    launch_zero(a.at<double>(a.off.pbar[1]), a.prep_bytes / 8, s);
    launch_zero(a.at<double>(a.off.acc), 2, s);
    if (a.obj.mesh_grad) {
        launch_zero(a.at<double>(a.off.gbar), size_t(3) * p.ell_width * p.nn, s);
        launch_zero(a.at<double>(a.off.vbar), size_t(2) * std::max(p.n_wall, 1), s);
        launch_zero(a.at<double>(a.off.w5bar), std::max<size_t>(p.sint_don.size(), 1), s);
        launch_zero(a.at<double>(a.off.w6bar), std::max<size_t>(p.uint_don.size(), 1), s);
    }
    int ab = 0, mb = 0, pb = 0;
    double alpha_host = 0.0;
    int rc = 0;
    const int Kc = int(o.ckpt_every);
    for (int seg = a.n_ckpt - 1; seg >= 0; --seg) {
        const int64_t ta = int64_t(seg) * Kc, tb = std::min<int64_t>(o.t_end, ta + Kc);
        // restore the checkpoint into the context and recompute the segment, storing every step
        c->cur[0] = 0;
        c->mesh_cur = 0;
        c->prep_t = 0;
        c->t = ta;
        rc |= d2d(c, c->lev(0, 0), a.ws + ckpt_lev(a, seg), a.lev_bytes);
        rc |= d2d(c, c->mesh(0), a.ws + ckpt_mesh(a, seg), a.mesh_bytes);
        rc |= d2d(c, c->prep(0), a.ws + ckpt_prep(a, seg), a.prep_bytes);
        for (int64_t t = ta; t < tb; ++t) {
            const int k = int(t - ta);
            rc |= d2d(c, a.ws + a.off.seg_lev + a256(a.lev_bytes) * k, c->lev(0, c->cur[0]), a.lev_bytes);
            rc |= d2d(c, a.ws + a.off.seg_mesh + a256(a.mesh_bytes) * k, c->mesh(c->mesh_cur), a.mesh_bytes);
            rc |= d2d(c, a.ws + a.off.seg_prep + a256(a.prep_bytes) * k, c->prep(c->prep_t), a.prep_bytes);
            finest_step(c);
        }
        rc |= d2d(c, a.ws + a.off.seg_prep + a256(a.prep_bytes) * int(tb - ta), c->prep(c->prep_t), a.prep_bytes);
        for (int64_t t = tb - 1; t >= ta; --t) reverse_step(c, a, K, t, int(t - ta), ab, mb, pb, alpha_host);
    }
    // the initial state: uniform f^eq(rho0, u_inf) fill, its collide-stream and
    // eq. (9) (post(0) and prep(0)), and the mesh initial values
    {
        double* Aw = a.at<double>(a.off.awork);
        double* prebar = a.at<double>(a.off.prebar);
        double* Anew = a.at<double>(a.off.abar[1 - ab]);
        const double ux = p.u_inf * std::cos(p.aoa), uy = p.u_inf * std::sin(p.aoa);
        launch_fill_uniform(HLBM_FP64, Aw, c->kl[0], p.rho0, ux, uy, s);
        int slot = 0;
        launch_adj_collide(K, Aw, a.at<double>(a.off.abar[ab]), prebar, slot, s);
        slot += adj_blocks_collide(c->kl[0]);
        launch_adj_s2m(K, Aw, a.nd6, a.at<int32_t>(a.off.t6node), a.at<int32_t>(a.off.t6ptr),
                       a.at<int32_t>(a.off.t6s), a.at<double>(a.off.t6w), a.at<double>(a.off.pbar[pb]), prebar, s);
        launch_adj_bc(K, Aw, prebar, slot, s);
        slot += adj_blocks_nodes(2 * (c->kl[0].nx - 2)) + adj_blocks_nodes(2 * (c->kl[0].ny - 2)) + 1;
        launch_adj_push(K, prebar, Anew, s);
        double dfeq[9];
        const int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1}, cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
        const double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
        for (int q = 0; q < 9; ++q) {
            const double cu = cx[q] * ux + cy[q] * uy;
            dfeq[q] = w[q] * p.rho0 *
                      ((3.0 * cx[q] + 9.0 * cu * cx[q] - 3.0 * ux) * K.duin_x +
                       (3.0 * cy[q] + 9.0 * cu * cy[q] - 3.0 * uy) * K.duin_y);
        }
        rc |= hip_check(c, hipMemcpyAsync(a.ws + a.off.dfeq, dfeq, sizeof(dfeq), hipMemcpyHostToDevice, s), "dfeq");
        launch_adj_alpha_state(K, Anew, a.at<double>(a.off.mbar[mb]), a.at<double>(a.off.dfeq), slot, s);
        slot += adj_blocks_nodes(int(c->kl[0].ny * c->kl[0].rs) + p.nn);
        launch_reduce_partials(a.at<double>(a.off.partial), slot, a.at<double>(a.off.acc), s);
    }
    double acc[2] = {0, 0};
    rc |= hip_check(c, hipMemcpyAsync(acc, a.ws + a.off.acc, 16, hipMemcpyDeviceToHost, s), "grad");
    rc |= hip_check(c, hipStreamSynchronize(s), "grad");
    rc |= hip_check(c, hipGetLastError(), "adjoint");
    if (rc) return HLBM_E_DEVICE;
    grad[0] = J_bar * (acc[0] + alpha_host);
    grad[1] = J_bar * acc[1];
    if (a.obj.mesh_grad) {
        // coefficient adjoints -> mesh coordinates (host, forward mode per local coordinate)
        std::vector<double> gb(size_t(3) * p.ell_width * p.nn), vb(size_t(2) * std::max(p.n_wall, 1));
        std::vector<double> t5(a.t5map.size()), t6(a.t6map.size());
        std::vector<double> w5(p.sint_w.size(), 0.0), w6(p.uint_w.size(), 0.0);
        rc |= hip_check(c, hipMemcpyAsync(gb.data(), a.ws + a.off.gbar, gb.size() * 8, hipMemcpyDeviceToHost, s), "gbar");
        rc |= hip_check(c, hipMemcpyAsync(vb.data(), a.ws + a.off.vbar, vb.size() * 8, hipMemcpyDeviceToHost, s), "vbar");
        if (!t5.empty())
            rc |= hip_check(c, hipMemcpyAsync(t5.data(), a.ws + a.off.w5bar, t5.size() * 8, hipMemcpyDeviceToHost, s), "w5bar");
        if (!t6.empty())
            rc |= hip_check(c, hipMemcpyAsync(t6.data(), a.ws + a.off.w6bar, t6.size() * 8, hipMemcpyDeviceToHost, s), "w6bar");
        rc |= hip_check(c, hipStreamSynchronize(s), "mesh grad");
        if (rc) return HLBM_E_DEVICE;
        for (size_t z = 0; z < t5.size(); ++z) w5[a.t5map[z]] = t5[z];
        for (size_t z = 0; z < t6.size(); ++z) w6[a.t6map[z]] = t6[z];
        std::vector<double> gx(2 * size_t(p.nn), 0.0);
        std::string err;
        const int grc = mesh_geometry_adjoint(p, gb.data(), vb.data(), w5.data(), w6.data(), gx.data(), err);
        if (grc) return set_err(c, grc, err);
        for (size_t z = 0; z < gx.size(); ++z) grad_xy[z] = J_bar * gx[z];
    }
    // the context now holds the state at the end of the first segment; restart from t_end
    // requires a new objective run
    a.ran = false;
    return HLBM_OK;
}

}  // extern "C"
