// adjoint.cpp -- objective run and discrete adjoint of the HLBM step.
//
// Objective: J = mean over finest steps h in [t0, t1) of w_cd C_D(h) + w_cl C_L(h)
// (eqs. (10)-(11)), for a run of t_end finest steps from the initial state.
// Gradient: dJ/d(angle of attack), dJ/d(tau) with the number of FV sub-steps
// held fixed, and optionally dJ/d(mesh coordinates).  Reverse mode over the
// exact sequence of GPU kernels of the forward step (FP64), level by level:
//   forward level l < L: collide-stream, [coarse -> fine, child step] x 2, fine -> coarse
//   forward finest:      eq. (4) -> collide-stream -> eq. (9) -> n FV sub-steps -> force
//   reverse level l < L: [child step^T, (fine -> coarse^T after the second), coarse -> fine^T]
//                        x 2 (second half first), collide-stream^T with the recorded side values^T
//   reverse finest:      force^T -> FV^T (n sub-steps, states recomputed; per sub-step the
//                        no-slip reset^T at wall pivots, then one gather per node) -> eq. (9)^T +
//                        collide^T + boundary^T + pull^T -> eq. (4)^T
// The restriction at the end of a level-l step pulls from the child's buffer
// between its two steps (the input of the second), so its transpose is added
// to the adjoint of that buffer.
// Memory: revolve-style two-level checkpointing: the forward stores the state
// every K finest steps; the reverse sweep recomputes each K-step segment
// forward from its checkpoint (recording the input of every step of every
// level) and, inside every finest step, the n sub-step states from the step's
// mesh state.
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "hlbm_internal.h"

using namespace hlbm;

struct AdjState {
    static size_t a256(size_t x) { return (x + 255) & ~size_t(255); }
    hlbm_objective obj{};
    char* ws = nullptr;
    size_t bytes = 0;
    int L = 0, per = 1;                       // levels - 1; finest steps per base step
    int n_ckpt = 0, seg_len = 0, seg_base = 0;
    size_t lev_bytes[4] = {}, side_bytes[4] = {}, mesh_bytes = 0, prep_bytes = 0, adjmesh_bytes = 0;
    int n_slots = 0, nd6 = 0;
    struct {
        size_t ckpt, ckpt_stride, ck_lev[4], ck_side[4], ck_mesh, ck_prep;
        size_t fin, fin_prev[4];   // state at t_end: a checkpoint plus every level's previous buffer
        size_t seg_lev[4], seg_side[4], seg_mesh, seg_prep, seg_sub, sub, awork;
        size_t seg_wmom, wmom;   // pre-reset (rho, u) of the wall nodes per sub-step
        size_t abar[4][2], prebar[4], sbar[4][2], vperim[4];
        size_t mbar[2], zwall[2], pbar[2], m5bar;
        size_t partial, acc, tedges, vwall, t5ptr, t5s, t5w, t6node, t6ptr, t6s, t6w, dfeq;
        size_t gbar, gpivot, vbar, w5bar, w6bar, total;
    } off{};
    bool tables = false, ran = false;
    size_t tables_at[9] = {};            // offsets of the transposed tables when they were uploaded
    std::vector<int32_t> t5map, t6map;   // transposed entry -> index into sint_w / uint_w
    std::vector<int64_t> gmap;           // transposed FV slot z * nn + k -> forward slot z_P * nn + P, -1 = unused
    double J = 0.0;
    std::vector<double> cd, cl;
    // reverse-sweep state: current slot of each ping-pong pair
    int ab[4] = {}, sb[4] = {}, mb = 0, pb = 0;
    int ridx[4] = {};                    // recorder: next snapshot slot per level
    int rec_rc = 0;
    template <typename T> T* at(size_t o) { return reinterpret_cast<T*>(ws + o); }
    size_t seg_lev_at(int l, int k) const { return off.seg_lev[l] + a256(lev_bytes[l]) * size_t(k); }
    size_t seg_side_at(int l, int k, int w) const { return off.seg_side[l] + a256(side_bytes[l]) * size_t(2 * k + w); }
    size_t seg_mesh_at(int k) const { return off.seg_mesh + a256(mesh_bytes) * size_t(k); }
    size_t seg_prep_at(int k) const { return off.seg_prep + a256(prep_bytes) * size_t(k); }
    int n_sub = 0;
    // state after FV sub-step m + 1 of segment step k (stored sub-steps)
    size_t seg_sub_at(int k, int m) const { return off.seg_sub + a256(mesh_bytes) * (size_t(k) * n_sub + m); }
    size_t wmom_bytes = 0;   // one sub-step's wall-node moments
    size_t seg_wmom_at(int k, int m) const { return off.seg_wmom + a256(wmom_bytes) * (size_t(k) * n_sub + m); }
};

namespace {

size_t a256(size_t x) { return AdjState::a256(x); }

int check_supported(hlbm_ctx* c, const hlbm_objective* o) {
    const Plan& p = c->p;
    if (!o) return set_err(c, HLBM_E_ARG, "objective is null");
    if (p.precision != HLBM_FP64) return set_err(c, HLBM_E_ARG, "the adjoint runs in FP64 contexts");
    if (p.periodic) return set_err(c, HLBM_E_ARG, "the adjoint needs the far-field base level");
    if (!p.has_mesh || p.wedge.empty()) return set_err(c, HLBM_E_ARG, "the adjoint needs a mesh with a wall");
    const int64_t per = int64_t(1) << p.L;
    if (o->t_end <= 0 || o->t0 < 0 || o->t1 <= o->t0 || o->t1 > o->t_end || o->ckpt_every <= 0)
        return set_err(c, HLBM_E_ARG, "objective window must satisfy 0 <= t0 < t1 <= t_end, ckpt_every > 0");
    if (o->t_end % per || o->ckpt_every % per)
        return set_err(c, HLBM_E_ARG, "t_end and ckpt_every must be multiples of 2^n_refine");
    if (o->t_end > p.hist_len) return set_err(c, HLBM_E_ARG, "t_end exceeds the force history length");
    return HLBM_OK;
}

int box_nodes(const LevelPlan& v) { return 2 * ((v.ci1 - v.ci0) + (v.cj1 - v.cj0)); }
int perim_nodes(const KLevel& C) { return 2 * ((C.nx - 1) + (C.ny - 1)); }
int bc_blocks(const KLevel& L) {
    return L.farfield ? adj_blocks_nodes(2 * (L.nx - 2)) + adj_blocks_nodes(2 * (L.ny - 2)) + 1 : 0;
}

// Workspace layout of the objective run and the reverse sweep.
void layout(hlbm_ctx* c, AdjState& a) {
    const Plan& p = c->p;
    const int K = int(a.obj.ckpt_every);
    a.L = p.L;
    a.per = 1 << p.L;
    a.seg_len = K;
    a.seg_base = K / a.per;
    a.n_ckpt = int((a.obj.t_end + K - 1) / K);
    size_t maxlev = 0;
    for (int l = 0; l <= p.L; ++l) {
        a.lev_bytes[l] = size_t(kQ) * p.lev[l].ny * p.lev[l].pitch * 8;
        a.side_bytes[l] = l < p.L ? size_t(box_nodes(p.lev[l])) * kMacro * 8 : 0;
        maxlev = std::max(maxlev, a.lev_bytes[l]);
    }
    a.mesh_bytes = size_t(kRec) * p.nn * 8;
    a.prep_bytes = size_t(std::max(p.n_int, 1)) * kMacro * 8;
    a.adjmesh_bytes = size_t(kAdjRec) * p.nn * 8;
    size_t off = 0;
    auto take = [&](size_t b) { const size_t o = off; off = a256(off + std::max<size_t>(b, 8)); return o; };
    // one checkpoint: every level's post buffer and side values, the mesh, prep(t)
    size_t ck = 0;
    for (int l = 0; l <= p.L; ++l) {
        a.off.ck_lev[l] = ck;
        ck += a256(a.lev_bytes[l]);
        a.off.ck_side[l] = ck;
        ck += a256(a.side_bytes[l]);
    }
    a.off.ck_mesh = ck;
    ck += a256(a.mesh_bytes);
    a.off.ck_prep = ck;
    ck += a256(a.prep_bytes);
    a.off.ckpt_stride = ck;
    a.off.ckpt = take(ck * a.n_ckpt);
    // the state at t_end, restored after the reverse sweep; state export pulls
    // from the previous buffer of each level, so that one is kept as well
    a.off.fin = take(ck);
    for (int l = 0; l <= p.L; ++l) a.off.fin_prev[l] = take(a.lev_bytes[l]);
    // one segment: level l takes seg_base 2^l steps; one more slot for its state after the segment
    for (int l = 0; l <= p.L; ++l) {
        const int n = a.seg_base << l;
        a.off.seg_lev[l] = take(a256(a.lev_bytes[l]) * (n + 1));
        a.off.seg_side[l] = l < p.L ? take(a256(a.side_bytes[l]) * 2 * n) : 0;
    }
    a.off.seg_mesh = take(a256(a.mesh_bytes) * K);
    a.off.seg_prep = take(a256(a.prep_bytes) * (K + 1));
    a.n_sub = p.n_sub;
    a.off.seg_sub = a.obj.store_substeps ? take(a256(a.mesh_bytes) * size_t(K) * p.n_sub) : 0;
    a.off.sub = take(a256(a.mesh_bytes) * (p.n_sub + 1));
    a.wmom_bytes = size_t(std::max(p.n_wall, 1)) * 3 * 8;
    a.off.seg_wmom = a.obj.store_substeps ? take(a256(a.wmom_bytes) * size_t(K) * p.n_sub) : 0;
    a.off.wmom = take(a256(a.wmom_bytes) * p.n_sub);
    a.off.awork = take(maxlev);
    for (int l = 0; l <= p.L; ++l) {
        a.off.abar[l][0] = take(a.lev_bytes[l]);
        a.off.abar[l][1] = take(a.lev_bytes[l]);
        a.off.prebar[l] = take(a.lev_bytes[l]);
        if (l < p.L) {
            a.off.sbar[l][0] = take(a.side_bytes[l]);
            a.off.sbar[l][1] = take(a.side_bytes[l]);
            a.off.vperim[l] = take(size_t(perim_nodes(c->kl[l + 1])) * kMacro * 8);
        }
    }
    a.off.mbar[0] = take(a.adjmesh_bytes);
    a.off.mbar[1] = take(a.adjmesh_bytes);
    a.off.zwall[0] = take(size_t(kAdjRec) * std::max(p.n_wall, 1) * 8);
    a.off.zwall[1] = take(size_t(kAdjRec) * std::max(p.n_wall, 1) * 8);
    a.off.pbar[0] = take(a.prep_bytes);
    a.off.pbar[1] = take(a.prep_bytes);
    a.off.m5bar = take(std::max<size_t>(p.sint_node.size(), 1) * kMacro * 8);
    // partial-sum slots between two reductions (the largest user)
    const KLevel& F = c->kl[p.L];
    const int bn = adj_fv_blocks(c->km);
    const int fine = p.n_sub * bn + adj_blocks_collide(F) + bc_blocks(F) +
                     adj_blocks_nodes(int(p.sint_node.size()));
    int coarse = 0, init = 0;
    for (int l = 0; l <= p.L; ++l) {
        const int cs = adj_blocks_collide(c->kl[l]) + bc_blocks(c->kl[l]);
        const int tr = l < p.L ? std::max(adj_blocks_nodes(f2c_adj_threads(p.lev[l].ci1 - p.lev[l].ci0,
                                                                             p.lev[l].cj1 - p.lev[l].cj0, p.f2c_filter)),
                                          adj_blocks_nodes(perim_nodes(c->kl[l + 1])))
                               : 0;
        coarse = std::max(coarse, std::max(cs, tr));
        init += cs + tr + adj_blocks_nodes(int(c->kl[l].ny * c->kl[l].rs) + p.nn);
    }
    a.n_slots = std::max(fine, std::max(coarse, init)) + 64;
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
        a.off.gpivot = take(size_t(2) * p.nn * 8);
        a.off.vbar = take(size_t(2) * std::max(p.n_wall, 1) * 8);
        a.off.w5bar = take(std::max<size_t>(p.sint_don.size(), 1) * 8);
        a.off.w6bar = take(std::max<size_t>(p.uint_don.size(), 1) * 8);
    }
    a.off.total = off;
}

int d2d(hlbm_ctx* c, void* dst, const void* src, size_t bytes) {
    if (!bytes) return HLBM_OK;
    return hip_check(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c->s), "hipMemcpyAsync");
}

// Copies the context's current state into the final-state region.
int save_final(hlbm_ctx* c, AdjState& a) {
    const Plan& p = c->p;
    int rc = HLBM_OK;
    for (int l = 0; l <= p.L; ++l) {
        rc |= d2d(c, a.ws + a.off.fin + a.off.ck_lev[l], c->lev(l, c->cur[l]), a.lev_bytes[l]);
        rc |= d2d(c, a.ws + a.off.fin_prev[l], c->lev(l, 1 - c->cur[l]), a.lev_bytes[l]);
        if (l < p.L) rc |= d2d(c, a.ws + a.off.fin + a.off.ck_side[l], c->side(l, c->side_t[l]), a.side_bytes[l]);
    }
    rc |= d2d(c, a.ws + a.off.fin + a.off.ck_mesh, c->mesh(c->mesh_cur), a.mesh_bytes);
    rc |= d2d(c, a.ws + a.off.fin + a.off.ck_prep, c->prep(c->prep_t), a.prep_bytes);
    return rc;
}

// Puts the state saved by save_final back into the context (time t_end).
int restore_final(hlbm_ctx* c, AdjState& a) {
    const Plan& p = c->p;
    int rc = HLBM_OK;
    for (int l = 0; l <= p.L; ++l) {
        c->cur[l] = 0;
        c->side_t[l] = 0;
        rc |= d2d(c, c->lev(l, 0), a.ws + a.off.fin + a.off.ck_lev[l], a.lev_bytes[l]);
        rc |= d2d(c, c->lev(l, 1), a.ws + a.off.fin_prev[l], a.lev_bytes[l]);
        if (l < p.L) rc |= d2d(c, c->side(l, 0), a.ws + a.off.fin + a.off.ck_side[l], a.side_bytes[l]);
    }
    c->mesh_cur = 0;
    c->prep_t = 0;
    rc |= d2d(c, c->mesh(0), a.ws + a.off.fin + a.off.ck_mesh, a.mesh_bytes);
    rc |= d2d(c, c->prep(0), a.ws + a.off.fin + a.off.ck_prep, a.prep_bytes);
    c->t = a.obj.t_end;
    return rc;
}

// Transposed tables of the reverse sweep, built from the plan.
int upload_tables(hlbm_ctx* c, AdjState& a) {
    const Plan& p = c->p;
    const int nn = p.nn, W = p.ell_width;
    // FV transpose: slot z of node k = (P, z_P, G_Pk, C_Pk) for the pivots P whose row holds k
    // in its slot z_P; slot 0 = (k, 0, sum_{j != k} G_kj, C_kk) (the pivot's own base and
    // collision terms)
    struct TEnt {
        int32_t P, zf;
        double gx, gy, c;
    };
    std::vector<std::vector<TEnt>> rows(nn);
    for (int P = 0; P < nn; ++P) {
        double sx = 0.0, sy = 0.0, ckk = 0.0;
        for (int z = p.rowptr[P]; z < p.rowptr[P + 1]; ++z) {
            if (p.col[z] == P) {
                ckk = p.cc[z];
                continue;
            }
            sx += p.gx[z];
            sy += p.gy[z];
            rows[p.col[z]].push_back({P, z - p.rowptr[P], p.gx[z], p.gy[z], p.cc[z]});
        }
        rows[P].insert(rows[P].begin(), TEnt{P, 0, sx, sy, ckk});
    }
    std::vector<char> te(size_t(W) * nn * 32, 0);
    a.gmap.assign(size_t(W) * nn, -1);
    for (int k = 0; k < nn; ++k) {
        if (int(rows[k].size()) > W) return set_err(c, HLBM_E_GEOMETRY, "mesh connectivity is not symmetric");
        for (int z = 0; z < W; ++z) {
            char* r = te.data() + (size_t(z) * nn + k) * 32;
            const bool used = z < int(rows[k].size());
            const int32_t col = used ? rows[k][z].P : -1, zf = used ? rows[k][z].zf : 0;
            if (used) a.gmap[size_t(z) * nn + k] = int64_t(zf) * nn + col;
            std::memcpy(r, &col, 4);
            std::memcpy(r + 4, &zf, 4);
            if (used) {
                const double v[3] = {rows[k][z].gx, rows[k][z].gy, rows[k][z].c};
                std::memcpy(r + 8, v, 24);
            }
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

// d tau_l / d tau_s under acoustic scaling tau_l - 1/2 = (tau_s - 1/2) / 2^(L - l)
double dtau_level(const Plan& p, int l) { return 1.0 / double(1 << (p.L - l)); }

// Reverse-mode view of level l (the mesh fields are those of the finest level).
KAdj make_kadj(hlbm_ctx* c, AdjState& a, int l) {
    const Plan& p = c->p;
    KAdj K;
    K.L = c->kl[l];
    K.M = c->km;
    K.tedges = a.ws + a.off.tedges;
    const double tau = p.tau_s, tu = p.tau_u, tl = p.lev[l].tau;
    K.dt = p.dt_u;
    K.dtt = p.dt_u / tu;
    K.ddtt_dtau = -p.dt_u / (tu * tu);
    K.cst = 1.0 - 1.0 / (2.0 * tau);
    K.dcst_dtau = 1.0 / (2.0 * tau * tau);
    K.omega = 1.0 / tl;
    K.domega_dtau = -dtau_level(p, l) / (tl * tl);
    K.phi = 2.0 * (tau - 1.0) / (2.0 * tau - 1.0);
    K.dphi_dtau = 2.0 / ((2.0 * tau - 1.0) * (2.0 * tau - 1.0));
    K.uin_x = p.u_inf * std::cos(p.aoa);
    K.uin_y = p.u_inf * std::sin(p.aoa);
    K.duin_x = -p.u_inf * std::sin(p.aoa);
    K.duin_y = p.u_inf * std::cos(p.aoa);
    K.partial = a.at<double>(a.off.partial);
    const bool g = a.obj.mesh_grad != 0;
    K.gbar = g ? a.at<double>(a.off.gbar) : nullptr;
    K.gpivot = g ? a.at<double>(a.off.gpivot) : nullptr;
    K.vbar = g ? a.at<double>(a.off.vbar) : nullptr;
    K.w5bar = g ? a.at<double>(a.off.w5bar) : nullptr;
    K.w6bar = g ? a.at<double>(a.off.w6bar) : nullptr;
    return K;
}

// Coefficients of the refinement transfers between levels l and l + 1 (the
// f^neq factors after collision) and their tau derivatives.
struct Transfer {
    double c2f, dc2f, f2c, df2c;
};
Transfer transfer(const Plan& p, int l) {
    const double tc = p.lev[l].tau, tf = p.lev[l + 1].tau;
    const double dc = dtau_level(p, l), df = dtau_level(p, l + 1);
    Transfer t;
    t.c2f = (tf - 1.0) / (2.0 * tc);   // (1 - 1/tau_f) tau_f / (2 tau_c)
    t.dc2f = (df * 2.0 * tc - (tf - 1.0) * 2.0 * dc) / (4.0 * tc * tc);
    t.f2c = 2.0 * (tc - 1.0) / tf;     // (1 - 1/tau_c) 2 tau_c / tau_f
    t.df2c = 2.0 * (dc * tf - (tc - 1.0) * df) / (tf * tf);
    return t;
}

// Step recorder of the segment recompute (see hlbm_ctx::rec).
void recorder(hlbm_ctx* c, int ev, int l) {
    AdjState& a = *c->adj;
    int& k = a.ridx[l];
    if (ev == 0) {
        a.rec_rc |= d2d(c, a.ws + a.seg_lev_at(l, k), c->lev(l, c->cur[l]), a.lev_bytes[l]);
        a.rec_rc |= d2d(c, a.ws + a.seg_side_at(l, k, 0), c->side(l, c->side_t[l]), a.side_bytes[l]);
    } else if (ev == 1) {
        a.rec_rc |= d2d(c, a.ws + a.seg_side_at(l, k, 1), c->side(l, 1 - c->side_t[l]), a.side_bytes[l]);
        ++k;
    } else if (ev == 2) {
        a.rec_rc |= d2d(c, a.ws + a.seg_mesh_at(k), c->mesh(c->mesh_cur), a.mesh_bytes);
        a.rec_rc |= d2d(c, a.ws + a.seg_prep_at(k), c->prep(c->prep_t), a.prep_bytes);
        if (a.obj.store_substeps) {
            c->sub_sink = a.ws + a.seg_sub_at(k, 0);
            c->sub_stride = a256(a.mesh_bytes);
            c->wmom_sink = a.at<double>(a.seg_wmom_at(k, 0));
            c->wmom_stride = a256(a.wmom_bytes) / 8;
        }
    } else {
        // finest input after eq. (4), as the collide-stream reads it: the reverse
        // step uses it as is
        a.rec_rc |= d2d(c, a.ws + a.seg_lev_at(l, k), c->lev(l, c->cur[l]), a.lev_bytes[l]);
        ++k;
    }
}

// Collide-stream^T of level l (recorded input X, output adjoint Bbar) with the far
// field^T on the base level: fills prebar (adjoint of the pulled values).
// Returns the partial slots used from slot on.
int collide_adj(hlbm_ctx* c, const KAdj& K, const double* X, const double* Bbar, double* prebar, int slot) {
    launch_adj_collide(K, X, Bbar, prebar, slot, c->s);
    return adj_blocks_collide(K.L);
}
int bc_adj(hlbm_ctx* c, const KAdj& K, const double* X, double* prebar, int slot) {
    if (!K.L.farfield) return 0;
    launch_adj_bc(K, X, prebar, slot, c->s);
    return bc_blocks(K.L);
}

// One reverse finest step: adjoint of finest step t, whose recorded inputs are segment slot k.
void reverse_finest(hlbm_ctx* c, AdjState& a, int64_t t, int k, double& alpha_host) {
    const Plan& p = c->p;
    const hlbm_objective& o = a.obj;
    const int L = p.L;
    const KAdj K = make_kadj(c, a, L);
    hipStream_t s = c->s;
    const double* Mt = a.at<double>(a.seg_mesh_at(k));
    const double* prep0 = a.at<double>(a.seg_prep_at(k));
    const double* prep1 = a.at<double>(a.seg_prep_at(k + 1));
    const double* Aw = a.at<double>(a.seg_lev_at(L, k));   // the input the collide-stream read
    double* Bbar = a.at<double>(a.off.abar[L][a.ab[L]]);
    double* Anew = a.at<double>(a.off.abar[L][1 - a.ab[L]]);
    double* prebar = a.at<double>(a.off.prebar[L]);
    double* Pcur = a.at<double>(a.off.pbar[a.pb]);       // adjoint of prep(t+1)
    double* Pnext = a.at<double>(a.off.pbar[1 - a.pb]);  // adjoint of prep(t)
    int slot = 0;
    // sub-step states M^0..M^n of this step: recorded by the segment recompute, or recomputed
    const size_t ms = a256(a.mesh_bytes);
    const bool stored = a.obj.store_substeps != 0;
    auto Msub = [&](int m) -> const double* {
        if (m == 0) return Mt;
        return stored ? a.at<double>(a.seg_sub_at(k, m - 1)) : a.at<double>(a.off.sub + ms * m);
    };
    // pre-reset (rho, u) of the wall nodes in sub-step m, recorded by the forward
    auto Wmom = [&](int m) -> const double* {
        return stored ? a.at<double>(a.seg_wmom_at(k, m)) : a.at<double>(a.off.wmom + a256(a.wmom_bytes) * m);
    };
    if (!stored) {
        (void)d2d(c, a.ws + a.off.sub, Mt, a.mesh_bytes);
        KMesh km = c->km;
        for (int m = 0; m < p.n_sub; ++m) {
            km.wmom = a.at<double>(a.off.wmom + a256(a.wmom_bytes) * m);
            launch_fv_substep(HLBM_FP64, km, a.ws + a.off.sub + ms * m, a.ws + a.off.sub + ms * (m + 1), prep0,
                              prep1, double(m) / p.n_sub, s);
        }
    }
    // force^T (history entry t belongs to the state after step t, M^n)
    if (t >= o.t0 && t < o.t1) {
        const double span = double(o.t1 - o.t0);
        const double jcd = o.w_cd / span, jcl = o.w_cl / span;   // times J_bar, applied at the end
        const double qn = 0.5 * p.rho0 * p.u_inf * p.u_inf * p.chord;
        const double ca = std::cos(p.aoa), sa = std::sin(p.aoa);
        launch_adj_force(K, a.at<double>(a.off.mbar[a.mb]), a.at<double>(a.off.vwall), (jcd * ca - jcl * sa) / qn,
                         (jcd * sa + jcl * ca) / qn, Msub(p.n_sub), s);
        // projection directions depend on alpha: dC_D/dalpha = C_L, dC_L/dalpha = -C_D
        alpha_host += jcd * a.cl[t] - jcl * a.cd[t];
    }
    // FV^T, last sub-step first: one gather per node and sub-step; the no-slip reset
    // transpose of a sub-step is taken by the wall threads of the launch after it
    const int bn = adj_fv_blocks(c->km);
    int zw = 0;
    launch_adj_fv_wall(K, Wmom(p.n_sub - 1), a.at<double>(a.off.mbar[a.mb]), a.at<double>(a.off.zwall[zw]), s);
    for (int m = p.n_sub - 1; m >= 0; --m) {
        const double th = double(m) / p.n_sub;
        const double* Mm = Msub(m);
        launch_adj_fv(K, Mm, a.at<double>(a.off.mbar[a.mb]), a.at<double>(a.off.zwall[zw]),
                      a.at<double>(a.off.mbar[1 - a.mb]), prep0, prep1, th, Pnext, Pcur, slot,
                      m > 0 ? Wmom(m - 1) : nullptr, a.at<double>(a.off.zwall[1 - zw]), s);
        slot += bn;
        a.mb ^= 1;
        zw ^= 1;
    }
    // collide-stream^T with eq. (9)^T and the boundary conditions^T, then pull^T
    slot += collide_adj(c, K, Aw, Bbar, prebar, slot);
    launch_adj_s2m(K, Aw, a.nd6, a.at<int32_t>(a.off.t6node), a.at<int32_t>(a.off.t6ptr), a.at<int32_t>(a.off.t6s),
                   a.at<double>(a.off.t6w), Pcur, prebar, s);
    slot += bc_adj(c, K, Aw, prebar, slot);
    launch_adj_push(K, prebar, Anew, s);
    // eq. (4)^T
    if (!p.sint_node.empty()) {
        launch_adj_m2s_a(K, Mt, int(p.sint_node.size()), reinterpret_cast<const int32_t*>(c->ws + p.off.sint_node),
                         reinterpret_cast<const int32_t*>(c->ws + p.off.sint_don),
                         reinterpret_cast<const double*>(c->ws + p.off.sint_w), Anew, a.at<double>(a.off.m5bar), slot, s);
        slot += adj_blocks_nodes(int(p.sint_node.size()));
        launch_adj_m2s_b(K, Mt, a.at<int32_t>(a.off.t5ptr), a.at<int32_t>(a.off.t5s), a.at<double>(a.off.t5w),
                         a.at<double>(a.off.m5bar), a.at<double>(a.off.mbar[a.mb]), s);
    }
    launch_reduce_partials(a.at<double>(a.off.partial), slot, a.at<double>(a.off.acc), s);
    // carried adjoints: finest input buffer, M_t, prep(t)
    a.ab[L] ^= 1;
    launch_zero(Pcur, a.prep_bytes / 8, s);
    a.pb ^= 1;
}

// Adjoint of step idx (within the segment that starts at finest time ta) of level l.
void reverse_level(hlbm_ctx* c, AdjState& a, int l, int idx, int64_t ta, double& alpha_host) {
    const Plan& p = c->p;
    if (l == p.L) {
        reverse_finest(c, a, ta + idx, idx, alpha_host);
        return;
    }
    hipStream_t s = c->s;
    const LevelPlan& v = p.lev[l];
    const int nxc = v.ci1 - v.ci0, nyc = v.cj1 - v.cj0;
    const Transfer tr = transfer(p, l);
    const KAdj K = make_kadj(c, a, l);
    double* partial = a.at<double>(a.off.partial);
    double* acc = a.at<double>(a.off.acc);
    const double* sp = a.at<double>(a.seg_side_at(l, idx, 0));
    const double* sc = a.at<double>(a.seg_side_at(l, idx, 1));
    for (int half = 1; half >= 0; --half) {
        reverse_level(c, a, l + 1, 2 * idx + half, ta, alpha_host);
        if (half == 1) {
            // fine -> coarse^T: the restriction pulls from the child's buffer that is the
            // input of its second step (interior nodes, untouched by the transfers)
            launch_adj_f2c(c->kl[l], c->kl[l + 1], v.ci0, v.cj0, nxc, nyc,
                           a.at<double>(a.seg_lev_at(l + 1, 2 * idx + 1)), a.at<double>(a.off.abar[l][a.ab[l]]),
                           a.at<double>(a.off.abar[l + 1][a.ab[l + 1]]), tr.f2c, tr.df2c, partial, 0, p.f2c_filter, s);
            launch_reduce_partials(partial, adj_blocks_nodes(f2c_adj_threads(nxc, nyc, p.f2c_filter)), acc, s);
        }
        // coarse -> fine^T onto the side values at the parent's two times
        launch_adj_c2f_a(c->kl[l + 1], sp, sc, 0.5 * half, a.at<double>(a.off.abar[l + 1][a.ab[l + 1]]),
                         a.at<double>(a.off.vperim[l]), tr.c2f, tr.dc2f, partial, 0, s);
        launch_adj_c2f_b(nxc, nyc, a.at<double>(a.off.vperim[l]), 0.5 * half, a.at<double>(a.off.sbar[l][1 - a.sb[l]]),
                         a.at<double>(a.off.sbar[l][a.sb[l]]), s);
        launch_reduce_partials(partial, adj_blocks_nodes(perim_nodes(c->kl[l + 1])), acc, s);
    }
    // collide-stream^T of level l, with the side values it recorded^T and the far field^T
    const double* X = a.at<double>(a.seg_lev_at(l, idx));
    double* prebar = a.at<double>(a.off.prebar[l]);
    int slot = collide_adj(c, K, X, a.at<double>(a.off.abar[l][a.ab[l]]), prebar, 0);
    launch_adj_side(c->kl[l], v.ci0, v.cj0, nxc, nyc, X, a.at<double>(a.off.sbar[l][a.sb[l]]), prebar, s);
    slot += bc_adj(c, K, X, prebar, slot);
    launch_adj_push(K, prebar, a.at<double>(a.off.abar[l][1 - a.ab[l]]), s);
    launch_reduce_partials(partial, slot, acc, s);
    a.ab[l] ^= 1;
    // the side values recorded by this step are consumed; the other slot holds the
    // adjoint of the values recorded by the previous step
    launch_zero(a.at<double>(a.off.sbar[l][a.sb[l]]), a.side_bytes[l] / 8, s);
    a.sb[l] ^= 1;
}

// Adjoint of the initial state with respect to the angle of attack and tau:
// the uniform f^eq(rho0, u_inf) fill of every level's previous buffer, its
// collide-stream, side values and restriction, eq. (9) at t = 0, and the mesh
// initial values.
int reverse_initial(hlbm_ctx* c, AdjState& a) {
    const Plan& p = c->p;
    hipStream_t s = c->s;
    const int L = p.L;
    double* Aw = a.at<double>(a.off.awork);
    double* partial = a.at<double>(a.off.partial);
    const double ux = p.u_inf * std::cos(p.aoa), uy = p.u_inf * std::sin(p.aoa);
    int slot = 0;
    // finest level: collide-stream^T + eq. (9)^T at prep(0) + far field^T (single level) + pull^T
    {
        const KAdj K = make_kadj(c, a, L);
        double* prebar = a.at<double>(a.off.prebar[L]);
        launch_fill_uniform(HLBM_FP64, Aw, c->kl[L], p.rho0, ux, uy, s);
        slot += collide_adj(c, K, Aw, a.at<double>(a.off.abar[L][a.ab[L]]), prebar, slot);
        launch_adj_s2m(K, Aw, a.nd6, a.at<int32_t>(a.off.t6node), a.at<int32_t>(a.off.t6ptr),
                       a.at<int32_t>(a.off.t6s), a.at<double>(a.off.t6w), a.at<double>(a.off.pbar[a.pb]), prebar, s);
        slot += bc_adj(c, K, Aw, prebar, slot);
        launch_adj_push(K, prebar, a.at<double>(a.off.abar[L][1 - a.ab[L]]), s);
    }
    // coarser levels, finest first: restriction^T into the child's fill, side values^T, collide-stream^T
    for (int l = L - 1; l >= 0; --l) {
        const LevelPlan& v = p.lev[l];
        const int nxc = v.ci1 - v.ci0, nyc = v.cj1 - v.cj0;
        const Transfer tr = transfer(p, l);
        const KAdj K = make_kadj(c, a, l);
        double* prebar = a.at<double>(a.off.prebar[l]);
        launch_fill_uniform(HLBM_FP64, Aw, c->kl[l + 1], p.rho0, ux, uy, s);
        launch_adj_f2c(c->kl[l], c->kl[l + 1], v.ci0, v.cj0, nxc, nyc, Aw, a.at<double>(a.off.abar[l][a.ab[l]]),
                       a.at<double>(a.off.abar[l + 1][1 - a.ab[l + 1]]), tr.f2c, tr.df2c, partial, slot,
                       p.f2c_filter, s);
        slot += adj_blocks_nodes(f2c_adj_threads(nxc, nyc, p.f2c_filter));
        launch_fill_uniform(HLBM_FP64, Aw, c->kl[l], p.rho0, ux, uy, s);
        slot += collide_adj(c, K, Aw, a.at<double>(a.off.abar[l][a.ab[l]]), prebar, slot);
        launch_adj_side(c->kl[l], v.ci0, v.cj0, nxc, nyc, Aw, a.at<double>(a.off.sbar[l][a.sb[l]]), prebar, s);
        slot += bc_adj(c, K, Aw, prebar, slot);
        launch_adj_push(K, prebar, a.at<double>(a.off.abar[l][1 - a.ab[l]]), s);
    }
    // angle of attack through the fills and the mesh initial values
    double dfeq[9];
    const KAdj K0 = make_kadj(c, a, 0);
    const int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1}, cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    const double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    for (int q = 0; q < 9; ++q) {
        const double cu = cx[q] * ux + cy[q] * uy;
        dfeq[q] = w[q] * p.rho0 *
                  ((3.0 * cx[q] + 9.0 * cu * cx[q] - 3.0 * ux) * K0.duin_x +
                   (3.0 * cy[q] + 9.0 * cu * cy[q] - 3.0 * uy) * K0.duin_y);
    }
    int rc = hip_check(c, hipMemcpyAsync(a.ws + a.off.dfeq, dfeq, sizeof(dfeq), hipMemcpyHostToDevice, s), "dfeq");
    for (int l = 0; l <= L; ++l) {
        const KAdj K = make_kadj(c, a, l);
        launch_adj_alpha_state(K, a.at<double>(a.off.abar[l][1 - a.ab[l]]), a.at<double>(a.off.mbar[a.mb]),
                               a.at<double>(a.off.dfeq), l == L, slot, s);
        slot += adj_blocks_nodes(int(c->kl[l].ny * c->kl[l].rs) + (l == L ? p.nn : 0));
    }
    launch_reduce_partials(partial, slot, a.at<double>(a.off.acc), s);
    // dfeq is a stack array: wait for its upload before returning
    rc |= hip_check(c, hipStreamSynchronize(s), "initial state");
    return rc;
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
    c->wstat = false;
    a.obj = *o;
    a.ran = false;
    layout(c, a);
    if (!d_ckpt || (reinterpret_cast<uintptr_t>(d_ckpt) & 255) || ckpt_bytes < a.off.total)
        return set_err(c, HLBM_E_WORKSPACE, "objective workspace must be 256-byte aligned and hold " +
                                                std::to_string(a.off.total) + " bytes");
    // the tables sit after the checkpoints and segment buffers, so their offsets move
    // with t_end, ckpt_every and store_substeps: upload again whenever they do
    const size_t at[9] = {a.off.tedges, a.off.vwall, a.off.t5ptr, a.off.t5s, a.off.t5w,
                          a.off.t6node, a.off.t6ptr, a.off.t6s, a.off.t6w};
    if (!same_ws || std::memcmp(at, a.tables_at, sizeof(at)) != 0) a.tables = false;
    std::memcpy(a.tables_at, at, sizeof(at));
    a.ws = static_cast<char*>(d_ckpt);
    a.bytes = ckpt_bytes;
    if (!a.tables && (rc = upload_tables(c, a))) return rc;
    reset_initial_state(c);
    const Plan& p = c->p;
    const int K = int(o->ckpt_every);
    for (int64_t t = 0; t < o->t_end; t += a.per) {
        if (t % K == 0) {
            const size_t ck = a.off.ckpt + a.off.ckpt_stride * size_t(t / K);
            for (int l = 0; l <= p.L; ++l) {
                rc |= d2d(c, a.ws + ck + a.off.ck_lev[l], c->lev(l, c->cur[l]), a.lev_bytes[l]);
                if (l < p.L) rc |= d2d(c, a.ws + ck + a.off.ck_side[l], c->side(l, c->side_t[l]), a.side_bytes[l]);
            }
            rc |= d2d(c, a.ws + ck + a.off.ck_mesh, c->mesh(c->mesh_cur), a.mesh_bytes);
            rc |= d2d(c, a.ws + ck + a.off.ck_prep, c->prep(c->prep_t), a.prep_bytes);
        }
        level_step(c, 0);
    }
    rc |= save_final(c, a);
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
    return hip_check(c, hipGetLastError(), "objective");
}

int hlbm_adjoint(hlbm_ctx* c, double J_bar, double* grad, double* grad_xy) {
    if (!c || !grad) return HLBM_E_ARG;
    if (!c->adj || !c->adj->ran) return set_err(c, HLBM_E_STATE, "hlbm_run_objective must run first");
    AdjState& a = *c->adj;
    if (grad_xy && !a.obj.mesh_grad)
        return set_err(c, HLBM_E_ARG, "grad_xy needs an objective run with mesh_grad set");
    const Plan& p = c->p;
    const hlbm_objective& o = a.obj;
    hipStream_t s = c->s;
    for (int l = 0; l <= p.L; ++l) {
        launch_zero(a.at<double>(a.off.abar[l][0]), a.lev_bytes[l] / 8, s);
        launch_zero(a.at<double>(a.off.abar[l][1]), a.lev_bytes[l] / 8, s);
        launch_zero(a.at<double>(a.off.prebar[l]), a.lev_bytes[l] / 8, s);
        if (l < p.L) {
            launch_zero(a.at<double>(a.off.sbar[l][0]), a.side_bytes[l] / 8, s);
            launch_zero(a.at<double>(a.off.sbar[l][1]), a.side_bytes[l] / 8, s);
        }
        a.ab[l] = 0;
        a.sb[l] = 0;
    }
    for (double* z : {a.at<double>(a.off.mbar[0]), a.at<double>(a.off.mbar[1])}) launch_zero(z, a.adjmesh_bytes / 8, s);
    for (double* z : {a.at<double>(a.off.zwall[0]), a.at<double>(a.off.zwall[1])})
        launch_zero(z, size_t(kAdjRec) * std::max(p.n_wall, 1), s);
    launch_zero(a.at<double>(a.off.pbar[0]), a.prep_bytes / 8, s);
    launch_zero(a.at<double>(a.off.pbar[1]), a.prep_bytes / 8, s);
    launch_zero(a.at<double>(a.off.acc), 2, s);
    if (a.obj.mesh_grad) {
        launch_zero(a.at<double>(a.off.gbar), size_t(3) * p.ell_width * p.nn, s);
        launch_zero(a.at<double>(a.off.gpivot), size_t(2) * p.nn, s);
        launch_zero(a.at<double>(a.off.vbar), size_t(2) * std::max(p.n_wall, 1), s);
        launch_zero(a.at<double>(a.off.w5bar), std::max<size_t>(p.sint_don.size(), 1), s);
        launch_zero(a.at<double>(a.off.w6bar), std::max<size_t>(p.uint_don.size(), 1), s);
    }
    a.mb = 0;
    a.pb = 0;
    double alpha_host = 0.0;
    int rc = 0;
    const int Kc = int(o.ckpt_every);
    for (int seg = a.n_ckpt - 1; seg >= 0; --seg) {
        const int64_t ta = int64_t(seg) * Kc, tb = std::min<int64_t>(o.t_end, ta + Kc);
        // restore the checkpoint into the context and recompute the segment, recording every step
        const size_t ck = a.off.ckpt + a.off.ckpt_stride * size_t(seg);
        for (int l = 0; l <= p.L; ++l) {
            c->cur[l] = 0;
            c->side_t[l] = 0;
            rc |= d2d(c, c->lev(l, 0), a.ws + ck + a.off.ck_lev[l], a.lev_bytes[l]);
            if (l < p.L) rc |= d2d(c, c->side(l, 0), a.ws + ck + a.off.ck_side[l], a.side_bytes[l]);
            a.ridx[l] = 0;
        }
        c->mesh_cur = 0;
        c->prep_t = 0;
        c->t = ta;
        rc |= d2d(c, c->mesh(0), a.ws + ck + a.off.ck_mesh, a.mesh_bytes);
        rc |= d2d(c, c->prep(0), a.ws + ck + a.off.ck_prep, a.prep_bytes);
        a.rec_rc = 0;
        c->rec = recorder;
        for (int64_t t = ta; t < tb; t += a.per) level_step(c, 0);
        c->rec = nullptr;
        c->sub_sink = nullptr;
        c->wmom_sink = nullptr;
        rc |= a.rec_rc;
        // states after the segment: the post buffer of every refined level, prep at tb
        for (int l = 1; l <= p.L; ++l)
            rc |= d2d(c, a.ws + a.seg_lev_at(l, a.ridx[l]), c->lev(l, c->cur[l]), a.lev_bytes[l]);
        rc |= d2d(c, a.ws + a.seg_prep_at(int(tb - ta)), c->prep(c->prep_t), a.prep_bytes);
        const int nb = int((tb - ta) / a.per);
        for (int b = nb - 1; b >= 0; --b) reverse_level(c, a, 0, b, ta, alpha_host);
    }
    rc |= reverse_initial(c, a);
    double acc[2] = {0, 0};
    rc |= hip_check(c, hipMemcpyAsync(acc, a.ws + a.off.acc, 16, hipMemcpyDeviceToHost, s), "grad");
    rc |= hip_check(c, hipStreamSynchronize(s), "grad");
    rc |= hip_check(c, hipGetLastError(), "adjoint");
    if (rc) return HLBM_E_DEVICE;
    grad[0] = J_bar * (acc[0] + alpha_host);
    grad[1] = J_bar * acc[1];
    for (int m = 0; m < p.n_shape; ++m) grad[2 + m] = std::nan("");
    if (a.obj.mesh_grad) {
        // coefficient adjoints -> mesh coordinates (host, forward mode per local coordinate)
        std::vector<double> gt(size_t(3) * p.ell_width * p.nn), gb(gt.size(), 0.0);
        std::vector<double> vb(size_t(2) * std::max(p.n_wall, 1));
        std::vector<double> gp(size_t(2) * p.nn);
        std::vector<double> t5(a.t5map.size()), t6(a.t6map.size());
        std::vector<double> w5(p.sint_w.size(), 0.0), w6(p.uint_w.size(), 0.0);
        rc |= hip_check(c, hipMemcpyAsync(gt.data(), a.ws + a.off.gbar, gt.size() * 8, hipMemcpyDeviceToHost, s), "gbar");
        rc |= hip_check(c, hipMemcpyAsync(vb.data(), a.ws + a.off.vbar, vb.size() * 8, hipMemcpyDeviceToHost, s), "vbar");
        rc |= hip_check(c, hipMemcpyAsync(gp.data(), a.ws + a.off.gpivot, gp.size() * 8, hipMemcpyDeviceToHost, s), "gpivot");
        if (!t5.empty())
            rc |= hip_check(c, hipMemcpyAsync(t5.data(), a.ws + a.off.w5bar, t5.size() * 8, hipMemcpyDeviceToHost, s), "w5bar");
        if (!t6.empty())
            rc |= hip_check(c, hipMemcpyAsync(t6.data(), a.ws + a.off.w6bar, t6.size() * 8, hipMemcpyDeviceToHost, s), "w6bar");
        rc |= hip_check(c, hipStreamSynchronize(s), "mesh grad");
        if (rc) return HLBM_E_DEVICE;
        // transposed slots -> forward ELL slots
        for (size_t e = 0; e < a.gmap.size(); ++e)
            if (a.gmap[e] >= 0)
                for (int j = 0; j < 3; ++j) gb[size_t(a.gmap[e]) * 3 + j] = gt[e * 3 + j];
        // G_Pk adjoints of the difference form: neighbour part minus the pivot's base part
        for (int P = 0; P < p.nn; ++P)
            for (int z = 1; z < p.rowptr[P + 1] - p.rowptr[P]; ++z) {
                double* g = gb.data() + (size_t(z) * p.nn + P) * 3;
                g[0] -= gp[2 * size_t(P)];
                g[1] -= gp[2 * size_t(P) + 1];
            }
        for (size_t z = 0; z < t5.size(); ++z) w5[a.t5map[z]] = t5[z];
        for (size_t z = 0; z < t6.size(); ++z) w6[a.t6map[z]] = t6[z];
        std::vector<double> gx(2 * size_t(p.nn), 0.0);
        std::string err;
        const int grc = mesh_geometry_adjoint(p, gb.data(), vb.data(), w5.data(), w6.data(), gx.data(), err);
        if (grc) return set_err(c, grc, err);
        if (grad_xy)
            for (size_t z = 0; z < gx.size(); ++z) grad_xy[z] = J_bar * gx[z];
        // shape parameters: contraction with the caller's d(x, y)/d a_m
        for (int m = 0; m < p.n_shape; ++m) {
            const double* d = p.dshape.data() + size_t(m) * gx.size();
            double sum = 0.0;
            for (size_t z = 0; z < gx.size(); ++z) sum += gx[z] * d[z];
            grad[2 + m] = J_bar * sum;
        }
    }
    // back to the state at t_end of the objective run; another adjoint needs a new run
    a.ran = false;
    rc = restore_final(c, a);
    rc |= hip_check(c, hipStreamSynchronize(s), "restore");
    return rc ? HLBM_E_DEVICE : HLBM_OK;
}

}  // extern "C"
