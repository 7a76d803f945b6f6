// prep.cpp -- host preprocessing of the HLBM library.
//
// Builds, from the caller's grid and mesh:
//   * the levels of the structured grid (Sec. 4: nested factor-two boxes,
//     the finest one with unit spacing), their relaxation times under
//     acoustic scaling and the inactive region inside the inner ellipse;
//   * the finite-volume coefficients of eq. (3) on median-dual control
//     volumes, S_ik = c_i . G_Pk and C_Pk, with boundary control volumes
//     closed by half boundary edges;
//   * a reverse Cuthill-McKee order of the mesh nodes, stably partitioned
//     into [wall | interior | interpolation] so that the finite-volume kernel
//     reads neighbours close in memory and tells node kinds by index;
//   * the interpolation stencils of eq. (8) (structured <- mesh) and eq. (9)
//     (mesh <- structured), or their linear variants;
//   * the byte layout of the device workspace.
#include <algorithm>
#include <cstdarg>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <queue>
#include <tuple>
#include <type_traits>

#include "hlbm_internal.h"

namespace hlbm {
namespace {

constexpr int kCx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int kCy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

// Is (x, y) inside the polygon: crossing number of the ray towards +x, an edge
// counted when exactly one of its end points has y' <= y, odd = inside.  No
// floating-point contraction, so the crossing abscissae round as written.
bool polygon_contains(int n, const double* xy, double x, double y) {
#pragma clang fp contract(off)
    bool in = false;
    for (int e = 0; e < n; ++e) {
        const double* a = xy + 2 * e;
        const double* b = xy + 2 * ((e + 1) % n);
        if ((a[1] <= y) == (b[1] <= y)) continue;
        const double xc = a[0] + (y - a[1]) * (b[0] - a[0]) / (b[1] - a[1]);
        if (x < xc) in = !in;
    }
    return in;
}

// Forward-mode dual number: value and derivative along one seeded input.  The
// geometry and stencil code below is written once for a scalar type S and
// evaluated with S = double (the plan) and S = Dual (derivatives of the
// coefficients with respect to one mesh coordinate, for the shape adjoint).
struct Dual {
    double v, d;
};
inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
inline Dual operator/(Dual a, Dual b) { return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)}; }
inline Dual operator*(double s, Dual a) { return {s * a.v, s * a.d}; }
inline Dual operator*(Dual a, double s) { return {a.v * s, a.d * s}; }
inline Dual operator+(Dual a, double b) { return {a.v + b, a.d}; }
inline Dual operator-(double a, Dual b) { return {a - b.v, -b.d}; }
inline Dual operator-(Dual a, double b) { return {a.v - b, a.d}; }
inline Dual& operator+=(Dual& a, Dual b) { return a = a + b; }
inline Dual& operator-=(Dual& a, Dual b) { return a = a - b; }
inline Dual& operator*=(Dual& a, Dual b) { return a = a * b; }
inline Dual operator/(Dual a, double b) { return {a.v / b, a.d / b}; }
inline double val(double a) { return a; }
inline double val(Dual a) { return a.v; }
inline double sqrt_(double a) { return std::sqrt(a); }
inline Dual sqrt_(Dual a) {
    const double r = std::sqrt(a.v);
    return {r, a.d / (2.0 * r)};
}
template <class S> inline S abs_(S a) { return val(a) < 0.0 ? -a : a; }
template <class S> inline S lift(double v);
template <> inline double lift<double>(double v) { return v; }
template <> inline Dual lift<Dual>(double v) { return {v, 0.0}; }

template <class S> struct V2T {
    S x, y;
};
template <class S> inline V2T<S> operator-(V2T<S> a, V2T<S> b) { return {a.x - b.x, a.y - b.y}; }
template <class S> inline V2T<S> operator+(V2T<S> a, V2T<S> b) { return {a.x + b.x, a.y + b.y}; }
template <class S> inline V2T<S> operator*(double s, V2T<S> a) { return {s * a.x, s * a.y}; }
template <class S> inline S cross(V2T<S> a, V2T<S> b) { return a.x * b.y - a.y * b.x; }
// outward normal of a counter-clockwise boundary piece
template <class S> inline V2T<S> rot_cw(V2T<S> a) { return {a.y, -a.x}; }
using V2 = V2T<double>;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int fail(std::string& err, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(std::string& err, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    err = buf;
    return code;
}

// ---------------------------------------------------------------------------
// finite-volume coefficients on the median dual
// ---------------------------------------------------------------------------

struct Entry {
    int p, k;
    double gx, gy, c;
};

// Contributions of corner P (neighbours A, B counter-clockwise) of a triangle of
// area at to the rows of P: out[0..5] = G parts of (P,P), (P,A), (P,B) (x, y),
// out[6..8] = C parts of the same entries (before division by A_P).
template <class S> void corner_terms(V2T<S> p, V2T<S> a, V2T<S> b, S at, S out[9]) {
    const V2T<S> e = a - p, f = b - p;
    // segments M_PA -> centroid and centroid -> M_PB of P's piece
    const V2T<S> n1 = (1.0 / 6.0) * rot_cw((2.0 * f) - e);
    const V2T<S> n2 = (1.0 / 6.0) * rot_cw(f - (2.0 * e));
    // hat functions at the two segment midpoints: P 5/12, 5/12; A 5/12, 1/6; B 1/6, 5/12
    const V2T<S> gP = (5.0 / 12.0) * (n1 + n2);
    const V2T<S> gA = (5.0 / 12.0) * n1 + (1.0 / 6.0) * n2;
    const V2T<S> gB = (1.0 / 6.0) * n1 + (5.0 / 12.0) * n2;
    out[0] = -gP.x, out[1] = -gP.y, out[2] = -gA.x, out[3] = -gA.y, out[4] = -gB.x, out[5] = -gB.y;
    out[6] = at * (11.0 / 54.0);
    out[7] = at * (7.0 / 108.0);
    out[8] = at * (7.0 / 108.0);
}

// Coefficients of eq. (3) for every node P (caller order), sorted by (P, k):
// G_Pk = -(1/A_P) sum over control-volume segments of N_seg psi_k(mid_seg),
// C_Pk = (1/A_P) integral of psi_k over the control volume, psi = linear hat.
int median_dual(int nn, int nt, const double* xy, const int32_t* tri, std::vector<Entry>& out,
                std::vector<double>& area, std::vector<std::array<int, 2>>& bnd_edges,
                std::string& err) {
    std::vector<Entry> acc;
    acc.reserve(size_t(nt) * 9 + 64);
    area.assign(nn, 0.0);
    auto P_of = [&](int v) { return V2{xy[2 * v], xy[2 * v + 1]}; };
    for (int t = 0; t < nt; ++t) {
        const int v[3] = {tri[3 * t], tri[3 * t + 1], tri[3 * t + 2]};
        for (int a = 0; a < 3; ++a)
            if (v[a] < 0 || v[a] >= nn) return fail(err, HLBM_E_GEOMETRY, "triangle %d: vertex index out of range", t);
        const double at2 = cross(P_of(v[1]) - P_of(v[0]), P_of(v[2]) - P_of(v[0]));
        if (!(at2 > 0.0)) return fail(err, HLBM_E_GEOMETRY, "triangle %d is not counter-clockwise or is degenerate", t);
        const double at = 0.5 * at2;
        for (int r = 0; r < 3; ++r) {
            const int P = v[r], A = v[(r + 1) % 3], B = v[(r + 2) % 3];
            double o[9];
            corner_terms<double>(P_of(P), P_of(A), P_of(B), at, o);
            acc.push_back({P, P, o[0], o[1], o[6]});
            acc.push_back({P, A, o[2], o[3], o[7]});
            acc.push_back({P, B, o[4], o[5], o[8]});
            area[P] += at / 3.0;
        }
    }
    // boundary edges: undirected edges used by a single triangle, kept with
    // the direction they have in that (counter-clockwise) triangle
    std::vector<std::tuple<int, int, int, int>> edges;  // (min, max, from, to)
    edges.reserve(size_t(nt) * 3);
    for (int t = 0; t < nt; ++t)
        for (int r = 0; r < 3; ++r) {
            const int a = tri[3 * t + r], b = tri[3 * t + (r + 1) % 3];
            edges.emplace_back(std::min(a, b), std::max(a, b), a, b);
        }
    std::sort(edges.begin(), edges.end());
    bnd_edges.clear();
    for (size_t s = 0; s < edges.size();) {
        size_t e = s + 1;
        while (e < edges.size() && std::get<0>(edges[e]) == std::get<0>(edges[s]) &&
               std::get<1>(edges[e]) == std::get<1>(edges[s]))
            ++e;
        if (e - s == 1) bnd_edges.push_back({std::get<2>(edges[s]), std::get<3>(edges[s])});
        else if (e - s > 2) return fail(err, HLBM_E_GEOMETRY, "edge (%d,%d) shared by more than two triangles",
                                        std::get<0>(edges[s]), std::get<1>(edges[s]));
        s = e;
    }
    // half boundary edges close the control volumes of boundary nodes:
    // P -> midpoint with hat values (3/4, 1/4), midpoint -> Q with (1/4, 3/4)
    for (const auto& be : bnd_edges) {
        const int P = be[0], Qn = be[1];
        const V2 nh = 0.5 * rot_cw(P_of(Qn) - P_of(P));
        acc.push_back({P, P, -0.75 * nh.x, -0.75 * nh.y, 0.0});
        acc.push_back({P, Qn, -0.25 * nh.x, -0.25 * nh.y, 0.0});
        acc.push_back({Qn, Qn, -0.75 * nh.x, -0.75 * nh.y, 0.0});
        acc.push_back({Qn, P, -0.25 * nh.x, -0.25 * nh.y, 0.0});
    }
    std::sort(acc.begin(), acc.end(), [](const Entry& a, const Entry& b) {
        return a.p != b.p ? a.p < b.p : a.k < b.k;
    });
    out.clear();
    for (const Entry& e : acc) {
        if (!out.empty() && out.back().p == e.p && out.back().k == e.k) {
            out.back().gx += e.gx;
            out.back().gy += e.gy;
            out.back().c += e.c;
        } else {
            out.push_back(e);
        }
    }
    for (int p = 0; p < nn; ++p)
        if (!(area[p] > 0.0)) return fail(err, HLBM_E_GEOMETRY, "mesh node %d belongs to no triangle", p);
    for (Entry& e : out) {
        e.gx /= area[e.p];
        e.gy /= area[e.p];
        e.c /= area[e.p];
    }
    return HLBM_OK;
}

// Reverse Cuthill-McKee order of the mesh graph, started from a minimum-degree
// node of the lowest-numbered component seed (wall nodes first when present).
std::vector<int> rcm_order(int nn, const std::vector<int>& rp, const std::vector<int>& cl,
                           const uint8_t* kind) {
    std::vector<int> deg(nn), order;
    order.reserve(nn);
    for (int p = 0; p < nn; ++p) deg[p] = rp[p + 1] - rp[p];
    std::vector<char> seen(nn, 0);
    std::vector<int> nb;
    while ((int)order.size() < nn) {
        int seed = -1;
        for (int pass = 0; pass < 2 && seed < 0; ++pass)
            for (int p = 0; p < nn; ++p) {
                if (seen[p]) continue;
                if (pass == 0 && !(kind && kind[p] == 1)) continue;
                if (seed < 0 || deg[p] < deg[seed]) seed = p;
            }
        std::queue<int> q;
        q.push(seed);
        seen[seed] = 1;
        while (!q.empty()) {
            const int p = q.front();
            q.pop();
            order.push_back(p);
            nb.clear();
            for (int z = rp[p]; z < rp[p + 1]; ++z)
                if (!seen[cl[z]]) nb.push_back(cl[z]);
            std::sort(nb.begin(), nb.end(), [&](int a, int b) { return deg[a] != deg[b] ? deg[a] < deg[b] : a < b; });
            for (int k : nb) {
                seen[k] = 1;
                q.push(k);
            }
        }
    }
    std::reverse(order.begin(), order.end());
    return order;
}

// ---------------------------------------------------------------------------
// interpolation stencils
// ---------------------------------------------------------------------------

struct TriIndex {
    double x0, y0, h;
    int nbx, nby;
    std::vector<int> head, list;          // bucket -> triangles (increasing index)
    std::vector<int> n2t_head, n2t;       // node -> incident triangles
};

void build_tri_index(int nn, int nt, const double* xy, const int32_t* tri, TriIndex& T) {
    double xmin = 1e300, ymin = 1e300, xmax = -1e300, ymax = -1e300;
    for (int p = 0; p < nn; ++p) {
        xmin = std::min(xmin, xy[2 * p]);
        xmax = std::max(xmax, xy[2 * p]);
        ymin = std::min(ymin, xy[2 * p + 1]);
        ymax = std::max(ymax, xy[2 * p + 1]);
    }
    T.h = std::max(1e-9, 1.5 * std::sqrt((xmax - xmin) * (ymax - ymin) / std::max(1, nt)));
    T.x0 = xmin - 0.5 * T.h;
    T.y0 = ymin - 0.5 * T.h;
    T.nbx = int((xmax - T.x0) / T.h) + 2;
    T.nby = int((ymax - T.y0) / T.h) + 2;
    std::vector<std::pair<int, int>> pairs;   // (bucket, triangle)
    for (int t = 0; t < nt; ++t) {
        double bx0 = 1e300, by0 = 1e300, bx1 = -1e300, by1 = -1e300;
        for (int r = 0; r < 3; ++r) {
            const int v = tri[3 * t + r];
            bx0 = std::min(bx0, xy[2 * v]);
            bx1 = std::max(bx1, xy[2 * v]);
            by0 = std::min(by0, xy[2 * v + 1]);
            by1 = std::max(by1, xy[2 * v + 1]);
        }
        const int i0 = std::max(0, int(std::floor((bx0 - 1e-9 - T.x0) / T.h)));
        const int i1 = std::min(T.nbx - 1, int(std::floor((bx1 + 1e-9 - T.x0) / T.h)));
        const int j0 = std::max(0, int(std::floor((by0 - 1e-9 - T.y0) / T.h)));
        const int j1 = std::min(T.nby - 1, int(std::floor((by1 + 1e-9 - T.y0) / T.h)));
        for (int j = j0; j <= j1; ++j)
            for (int i = i0; i <= i1; ++i) pairs.emplace_back(j * T.nbx + i, t);
    }
    std::sort(pairs.begin(), pairs.end());
    T.head.assign(size_t(T.nbx) * T.nby + 1, 0);
    T.list.resize(pairs.size());
    for (size_t a = 0; a < pairs.size(); ++a) {
        T.head[pairs[a].first + 1]++;
        T.list[a] = pairs[a].second;
    }
    for (size_t b = 0; b + 1 < T.head.size(); ++b) T.head[b + 1] += T.head[b];
    T.n2t_head.assign(nn + 1, 0);
    for (int a = 0; a < 3 * nt; ++a) T.n2t_head[tri[a] + 1]++;
    for (int p = 0; p < nn; ++p) T.n2t_head[p + 1] += T.n2t_head[p];
    T.n2t.resize(size_t(3) * nt);
    std::vector<int> cur(T.n2t_head.begin(), T.n2t_head.end() - 1);
    for (int t = 0; t < nt; ++t)
        for (int r = 0; r < 3; ++r) T.n2t[cur[tri[3 * t + r]]++] = t;
}

// barycentric coordinates of (x, y) in triangle t (vertex order of the triangle)
template <class S> void bary(const S* xy, const int32_t* tri, int t, double x, double y, S l[3]) {
    const V2T<S> a{xy[2 * tri[3 * t]], xy[2 * tri[3 * t] + 1]};
    const V2T<S> b{xy[2 * tri[3 * t + 1]], xy[2 * tri[3 * t + 1] + 1]};
    const V2T<S> c{xy[2 * tri[3 * t + 2]], xy[2 * tri[3 * t + 2] + 1]};
    const V2T<S> p{lift<S>(x), lift<S>(y)};
    const S d = cross(b - a, c - a);
    l[1] = cross(p - a, c - a) / d;
    l[2] = cross(b - a, p - a) / d;
    l[0] = 1.0 - l[1] - l[2];
}

// Solves M w = e_0 (6 x 6) by Gauss-Jordan elimination with full pivoting
// (pivots chosen on values).
template <class S> bool solve6(S M[6][6], S w[6]) {
    S rhs[6];
    for (int k = 0; k < 6; ++k) rhs[k] = lift<S>(k == 0 ? 1.0 : 0.0);
    int colperm[6] = {0, 1, 2, 3, 4, 5};
    double big = 0;
    for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) big = std::max(big, std::fabs(val(M[r][c])));
    for (int k = 0; k < 6; ++k) {
        int pr = k, pc = k;
        for (int r = k; r < 6; ++r)
            for (int c = k; c < 6; ++c)
                if (std::fabs(val(M[r][c])) > std::fabs(val(M[pr][pc]))) pr = r, pc = c;
        if (std::fabs(val(M[pr][pc])) < 1e-10 * big) return false;
        if (pr != k) {
            for (int c = 0; c < 6; ++c) std::swap(M[k][c], M[pr][c]);
            std::swap(rhs[k], rhs[pr]);
        }
        if (pc != k) {
            for (int r = 0; r < 6; ++r) std::swap(M[r][k], M[r][pc]);
            std::swap(colperm[k], colperm[pc]);
        }
        const S inv = lift<S>(1.0) / M[k][k];
        for (int c = k; c < 6; ++c) M[k][c] *= inv;
        rhs[k] *= inv;
        for (int r = 0; r < 6; ++r) {
            // (a zero factor changes nothing in values; derivatives still flow through it)
            if (r == k || (val(M[r][k]) == 0.0 && std::is_same<S, double>::value)) continue;
            const S f = M[r][k];
            for (int c = k; c < 6; ++c) M[r][c] -= f * M[k][c];
            rhs[r] -= f * rhs[k];
        }
    }
    for (int k = 0; k < 6; ++k) w[colperm[k]] = rhs[k];
    return true;
}

// Donors and weights of one triangle's stencil at (x, y): the quadratic of
// eq. (8) through the triangle's vertices and the vertices opposite its three
// edges in the neighbouring triangles (exact for quadratics); barycentric
// weights when linear is asked for, a neighbour is missing, or singular.
// Topology and pivoting come from the values; xy may carry derivatives.
template <class S>
int tri_stencil(const TriIndex& T, const S* xy, const int32_t* tri, int t, const S lam[3],
                double x, double y, bool linear, int* don, S* w, bool& fallback) {
    const int v0 = tri[3 * t], v1 = tri[3 * t + 1], v2 = tri[3 * t + 2];
    if (!linear) {
        auto opposite = [&](int a, int b) {
            for (int z = T.n2t_head[a]; z < T.n2t_head[a + 1]; ++z) {
                const int u = T.n2t[z];
                if (u == t) continue;
                int third = -1;
                bool hb = false;
                for (int r = 0; r < 3; ++r) {
                    const int q = tri[3 * u + r];
                    if (q == b) hb = true;
                    else if (q != a) third = q;
                }
                if (hb) return third;
            }
            return -1;
        };
        const int nodes[6] = {v0, v1, v2, opposite(v0, v1), opposite(v1, v2), opposite(v2, v0)};
        if (nodes[3] >= 0 && nodes[4] >= 0 && nodes[5] >= 0) {
            const S h = sqrt_(abs_(cross(V2T<S>{xy[2 * v1] - xy[2 * v0], xy[2 * v1 + 1] - xy[2 * v0 + 1]},
                                         V2T<S>{xy[2 * v2] - xy[2 * v0], xy[2 * v2 + 1] - xy[2 * v0 + 1]})));
            S M[6][6];
            for (int k = 0; k < 6; ++k) {
                const S a = (xy[2 * nodes[k]] - x) / h, b = (xy[2 * nodes[k] + 1] - y) / h;
                const S mono[6] = {lift<S>(1.0), a, b, a * a, a * b, b * b};
                for (int r = 0; r < 6; ++r) M[r][k] = mono[r];
            }
            S ww[6];
            if (solve6(M, ww)) {
                for (int k = 0; k < 6; ++k) don[k] = nodes[k], w[k] = ww[k];
                return 6;
            }
        }
        fallback = true;
    }
    don[0] = v0, don[1] = v1, don[2] = v2;
    w[0] = lam[0], w[1] = lam[1], w[2] = lam[2];
    return 3;
}

// Stencil of a structured interpolation node: a node it sits on; the stencil of
// the triangle containing it; the mean of the two stencils when it lies on the
// edge shared by two triangles.  Returns donor count or -1 (outside / ambiguous).
template <class S>
int mesh_stencil(const TriIndex& T, const S* xy, const int32_t* tri, double x, double y, bool linear,
                 int* don, S* w, bool& fallback) {
    fallback = false;
    const int bi = int(std::floor((x - T.x0) / T.h)), bj = int(std::floor((y - T.y0) / T.h));
    if (bi < 0 || bj < 0 || bi >= T.nbx || bj >= T.nby) return -1;
    const int b = bj * T.nbx + bi;
    int hits[8], nh = 0;
    S lams[8][3];
    for (int z = T.head[b]; z < T.head[b + 1] && nh < 8; ++z) {
        S l[3];
        bary(xy, tri, T.list[z], x, y, l);
        if (val(l[0]) >= -1e-12 && val(l[1]) >= -1e-12 && val(l[2]) >= -1e-12) {
            hits[nh] = T.list[z];
            std::copy(l, l + 3, lams[nh]);
            ++nh;
        }
    }
    if (nh == 0) return -1;
    for (int r = 0; r < 3; ++r)
        if (val(lams[0][r]) >= 1.0 - 1e-12) {
            don[0] = tri[3 * hits[0] + r];
            w[0] = lift<S>(1.0);
            return 1;
        }
    if (nh > 2) return -1;
    int n = 0;
    for (int a = 0; a < nh; ++a) {
        int d[6];
        S ww[6];
        const int nd = tri_stencil(T, xy, tri, hits[a], lams[a], x, y, linear, d, ww, fallback);
        for (int k = 0; k < nd; ++k) {
            int slot = -1;
            for (int s = 0; s < n; ++s)
                if (don[s] == d[k]) slot = s;
            if (slot < 0) {
                slot = n++;
                don[slot] = d[k];
                w[slot] = lift<S>(0.0);
            }
            w[slot] += ww[k] / double(nh);
        }
    }
    return n;
}

// Tensor-product weights of eq. (9) at (x, y) relative to the finest origin
// (unit spacing): quadratic Lagrange on the 3 x 3 block around the nearest
// node, or bilinear on the cell.  Returns the donor count.
template <class S> int lagrange9(S x, S y, bool linear, int* di, int* dj, S* w) {
    if (!linear) {
        const int ic = int(std::floor(val(x) + 0.5)), jc = int(std::floor(val(y) + 0.5));
        const S s1 = x - double(ic), t1 = y - double(jc);
        const S lx[3] = {0.5 * s1 * (s1 - 1.0), (1.0 - s1) * (s1 + 1.0), 0.5 * s1 * (s1 + 1.0)};
        const S ly[3] = {0.5 * t1 * (t1 - 1.0), (1.0 - t1) * (t1 + 1.0), 0.5 * t1 * (t1 + 1.0)};
        int nd = 0;
        for (int b = -1; b <= 1; ++b)
            for (int a = -1; a <= 1; ++a) {
                di[nd] = ic + a;
                dj[nd] = jc + b;
                w[nd] = lx[a + 1] * ly[b + 1];
                ++nd;
            }
        return nd;
    }
    const int ic = int(std::floor(val(x))), jc = int(std::floor(val(y)));
    const S s1 = x - double(ic), t1 = y - double(jc);
    di[0] = ic, dj[0] = jc, w[0] = (1.0 - s1) * (1.0 - t1);
    di[1] = ic + 1, dj[1] = jc, w[1] = s1 * (1.0 - t1);
    di[2] = ic, dj[2] = jc + 1, w[2] = (1.0 - s1) * t1;
    di[3] = ic + 1, dj[3] = jc + 1, w[3] = s1 * t1;
    return 4;
}

// Default FV sub-steps per launch on meshes with at most 8 neighbour slots per
// node: in FP32 the most (up to kMaxFuse) whose tiles fit, in FP64 two; else
// one.  Measured on MI355X, per sub-step: FP32 264k nodes 7.66 us with four and
// 8.0 with three (512-thread tiles), 8.35 with two (256-thread tiles), 13.9-14.8
// unfused; FP32
// 33k nodes 3.17 us with four, 3.41 with three, 3.63 with two, 4.94 unfused;
// FP64 22.5 against 29.8 us (264k) and 4.6 against 7.1 us (33k) with two, three
// and four being slower there.
constexpr int kFvFuse = 2;

// Fused-kernel tiles (plan nodes) and workgroup sizes.  A launch is fastest
// when all of its workgroups are resident at once: the kernel then takes about
// one workgroup lifetime, and a partial second wave of workgroups doubles it
// (measured on MI355X, 264k-node mesh, two FP32 sub-steps per launch: 787
// tiles of 336 nodes 30.8 us, 768 tiles of 344-368 nodes 22.8 us; 3 blocks of
// 256 threads per CU x 256 CUs = 768 resident).  FP32 tiles are therefore sized
// so that the tiles fill a whole number of such waves.  On meshes with at most
// 8 slots the FP32 workgroups have 512 threads, two per CU (126 VGPRs: four
// waves per SIMD), so that a tile with its rings for three or four sub-steps
// still gives each thread at most two nodes; 16-slot meshes keep 256 threads.
constexpr int kFvCUs = 256;                          // compute units of an MI355X
constexpr int kFvThreadsF32 = 256, kFvTileMinF32 = 192, kFvTileMaxF32 = 368;
constexpr int kFvThreadsWide = 512, kFvTileMaxWide = 1024;   // FP32, at most 8 slots (the kernel's launch bound)
// LDS per fused-FV workgroup: 64 KB, and 80 KB for the 512-thread FP32 tiles, of
// which two share a CU's 160 KB on gfx950 (hlbm_create checks the plan against the
// device's per-workgroup limit).  With 80 KB the bench mesh takes four sub-steps per
// launch: 7.66 against 8.0 us per sub-step with three.
constexpr size_t kFvLds = 65536, kFvLdsWide = 81920;
// FP64 (240 VGPRs, 2 waves per SIMD): tiles of 128 nodes on large meshes, down
// to 64 so that a small mesh still gives about two tiles per CU (measured at
// 33k nodes: 6.2 us per sub-step with 64, 7.6 with 128; at 264k nodes, two
// sub-steps per launch: 36.1 us with 128, 37.3 with 144, 37.7 with 160, 38.6
// with 192).
constexpr int kFvThreadsF64 = 128, kFvTileMinF64 = 64, kFvTileMaxF64 = 128;

// Tiles for the fused finite-volume kernel, which takes several Jacobi
// sub-steps per launch out of LDS.  Plan nodes are grouped into tiles of at
// most `tile` nodes grown breadth-first over the mesh graph (compact tiles,
// small halos); each tile then gets the rings 1..fuse of neighbours around
// it: sub-step j of a launch of k sub-steps updates the tile and rings
// 1..k-j, reading rings up to k-j+1.  Local order: tile, ring 1, ..., ring
// fuse, each ascending.  The edge table of a tile covers the nodes that are
// ever updated (tile .. ring fuse-1), slot-major, with local columns.
void build_fv_tiles(Plan& p, int tile, int fuse) {
    const int nn = p.nn, W = p.ft_width;
    std::vector<int> owner(nn, -1);
    std::vector<std::vector<int>> tiles;
    int next = 0;
    for (;;) {
        while (next < nn && owner[next] >= 0) ++next;
        if (next >= nn) break;
        const int id = int(tiles.size());
        std::vector<int> t;
        std::queue<int> q;
        int seed = next;
        while (int(t.size()) < tile) {
            if (q.empty()) {          // region exhausted: continue from the next free node
                while (seed < nn && owner[seed] >= 0) ++seed;
                if (seed >= nn) break;
                owner[seed] = id;
                t.push_back(seed);
                q.push(seed);
                continue;
            }
            const int a = q.front();
            q.pop();
            for (int z = p.rowptr[a] + 1; z < p.rowptr[a + 1] && int(t.size()) < tile; ++z) {
                const int b = p.col[z];
                if (owner[b] < 0) {
                    owner[b] = id;
                    t.push_back(b);
                    q.push(b);
                }
            }
        }
        tiles.push_back(std::move(t));
    }
    p.fv_fuse = fuse;
    p.fv_tile = tile;
    p.n_tiles = int(tiles.size());
    p.fv_maxl = 0;
    p.fv_maxw = 0;
    p.fv_maxs = 0;
    p.ft_meta.assign(size_t(p.n_tiles) * kTileMeta, 0);
    p.ft_node.clear();
    p.ft_star.clear();
    std::vector<int> sstamp(nn, -1), sslot(nn, -1);
    p.ft_col.clear();
    p.ft_src.clear();
    std::vector<int> stamp(nn, -1), loc(nn, -1);
    for (int t = 0; t < p.n_tiles; ++t) {
        std::vector<int> nodes = tiles[t];
        std::sort(nodes.begin(), nodes.end());
        for (int a : nodes) stamp[a] = t;
        int32_t* meta = p.ft_meta.data() + size_t(t) * kTileMeta;
        meta[3] = int(nodes.size());
        size_t lo = 0;
        for (int r = 1; r <= fuse; ++r) {
            const size_t hi = nodes.size();
            for (size_t i = lo; i < hi; ++i)
                for (int z = p.rowptr[nodes[i]] + 1; z < p.rowptr[nodes[i] + 1]; ++z) {
                    const int b = p.col[z];
                    if (stamp[b] != t) {
                        stamp[b] = t;
                        nodes.push_back(b);
                    }
                }
            std::sort(nodes.begin() + hi, nodes.end());
            meta[3 + r] = int(nodes.size());
            lo = hi;
        }
        for (int r = fuse + 1; r <= kMaxFuse; ++r) meta[3 + r] = meta[3 + fuse];
        for (size_t i = 0; i < nodes.size(); ++i) loc[nodes[i]] = int(i);
        const int width = meta[3 + fuse - 1];
        meta[0] = int(p.ft_node.size());
        meta[1] = int(p.ft_col.size());
        meta[2] = width;
        p.ft_node.insert(p.ft_node.end(), nodes.begin(), nodes.end());
        meta[8] = int(p.ft_star.size());
        int ns = 0;
        for (int z = 0; z < W; ++z)
            for (int i = 0; i < width; ++i) {
                const int P = nodes[i], zz = p.rowptr[P] + z;
                const bool used = zz < p.rowptr[P + 1];
                // an interpolation pivot reads f* (eqs. (5)-(7)) for its interpolation neighbours
                const bool star = used && P >= p.n_core && p.col[zz] >= p.n_core;
                int32_t c = used ? loc[p.col[zz]] : -1;
                if (star) {
                    const int b = p.col[zz];
                    if (sstamp[b] != t) {
                        sstamp[b] = t;
                        sslot[b] = ns++;
                        p.ft_star.push_back(b - p.n_core);
                    }
                    c = sslot[b] | kFtStar;
                }
                p.ft_col.push_back(c);
                p.ft_src.push_back(used ? zz : -1);
            }
        meta[9] = ns;
        p.fv_maxs = std::max(p.fv_maxs, ns);
        p.fv_maxl = std::max(p.fv_maxl, int(nodes.size()));
        p.fv_maxw = std::max(p.fv_maxw, width);
    }
}

// Resident fused-FV workgroups per CU in FP32: two (of 512 threads at 8 slots,
// of 256 at 16).
constexpr int kFvBlocksPerCuF32 = 2;

void choose_fv_tiles(Plan& p, int fuse) {
    if (p.elem == 8) {
        const int tile = std::max(kFvTileMinF64, std::min(kFvTileMaxF64, p.nn / (2 * kFvCUs) / 8 * 8));
        build_fv_tiles(p, tile, fuse);
        return;
    }
    const int tmax = p.ell_width <= 8 ? kFvTileMaxWide : kFvTileMaxF32;
    const int64_t slots = int64_t(kFvCUs) * kFvBlocksPerCuF32;
    const int64_t waves = std::max<int64_t>(1, (p.nn + tmax * slots - 1) / (tmax * slots));
    int tile = int((p.nn + waves * slots - 1) / (waves * slots));
    tile = std::min(tmax, std::max(kFvTileMinF32, (tile + 7) / 8 * 8));
    build_fv_tiles(p, tile, fuse);
    // breadth-first tiles come out partly smaller than `tile`: grow until they fit
    while (p.n_tiles > waves * slots && tile + 8 <= tmax) {
        tile += 8;
        build_fv_tiles(p, tile, fuse);
    }
}

}  // namespace

int build_plan(const hlbm_grid* g, const hlbm_mesh* m, double Re, double tau, Plan& p, std::string& err) {
    if (!g) return fail(err, HLBM_E_ARG, "grid is null");
    p = Plan();
    p.has_grid = g->nx_cells > 0 && g->ny_cells > 0;
    p.has_mesh = m && m->n_nodes > 0;
    p.has_body = m && m->body_n > 0;
    if (!p.has_grid) return fail(err, HLBM_E_ARG, "a structured grid is required");
    if (g->n_refine < 0 || g->n_refine > 3) return fail(err, HLBM_E_ARG, "n_refine must be 0..3");
    if (g->precision != HLBM_FP64 && g->precision != HLBM_FP32_SHIFTED) return fail(err, HLBM_E_ARG, "bad precision");
    if (g->interp != HLBM_INTERP_QUADRATIC && g->interp != HLBM_INTERP_LINEAR) return fail(err, HLBM_E_ARG, "bad interp");
    if (g->bc != HLBM_BC_FARFIELD && g->bc != HLBM_BC_PERIODIC) return fail(err, HLBM_E_ARG, "bad bc");
    if (!(g->rho0 > 0)) return fail(err, HLBM_E_PARAM, "rho0 must be positive");
    p.L = g->n_refine;
    p.nlev = p.L + 1;
    p.precision = g->precision;
    p.elem = g->precision == HLBM_FP64 ? 8 : 4;
    p.interp = g->interp;
    p.periodic = g->bc == HLBM_BC_PERIODIC;
    p.wall_bc = g->wall_bc != 0;
    p.u_inf = g->u_inf;
    p.aoa = g->aoa_rad;
    p.rho0 = g->rho0;
    p.chord = p.has_mesh || p.has_body ? m->chord : 1.0;
    p.check_every = std::max(0, g->check_every);
    if (g->f2c_filter != 0 && g->f2c_filter != 1) return fail(err, HLBM_E_ARG, "f2c_filter must be 0 or 1");
    p.f2c_filter = g->f2c_filter;
    if (p.f2c_filter)
        for (int l = 0; l < g->n_refine && l < 3; ++l)
            if (g->patch_nx[l] < 8 || g->patch_ny[l] < 8)
                return fail(err, HLBM_E_ARG, "f2c_filter needs boxes of at least 8 x 8 cells");
    p.hist_len = g->history_len > 0 ? g->history_len : 65536;
    // relaxation time of the finest level (nu = c_s^2 (tau - 1/2), Sec. 2)
    if (tau > 0.5) {
        p.tau_s = tau;
        if (Re > 0) {
            const double t2 = 0.5 + 3.0 * g->u_inf * p.chord / Re;
            if (std::fabs(t2 - tau) > 1e-12 * tau) return fail(err, HLBM_E_PARAM, "Re and tau disagree");
        }
    } else if (Re > 0) {
        p.tau_s = 0.5 + 3.0 * g->u_inf * p.chord / Re;
    } else {
        return fail(err, HLBM_E_PARAM, "need tau > 1/2 or Re > 0");
    }
    if (!(p.tau_s > 0.5)) return fail(err, HLBM_E_PARAM, "tau must exceed 1/2");
    p.tau_u = p.tau_s - 0.5;
    p.n_sub = g->n_sub > 0 ? g->n_sub : std::max(10, int(std::ceil(1.0 / p.tau_u)));
    p.dt_u = 1.0 / p.n_sub;

    // ---- levels
    {
        LevelPlan& b = p.lev[0];
        b.nx = g->nx_cells + (p.periodic ? 0 : 1);
        b.ny = g->ny_cells + (p.periodic ? 0 : 1);
        b.sp = 1 << p.L;
        b.farfield = !p.periodic;
        b.periodic = p.periodic;
        if (b.nx < 4 || b.ny < 4) return fail(err, HLBM_E_ARG, "grid too small");
    }
    for (int l = 1; l <= p.L; ++l) {
        LevelPlan& c = p.lev[l];
        LevelPlan& a = p.lev[l - 1];
        const int px = g->patch_nx[l - 1], py = g->patch_ny[l - 1];
        if (px <= 0 || py <= 0 || px % 2 || py % 2) return fail(err, HLBM_E_GEOMETRY, "box %d: sizes must be positive and even", l);
        c.nx = px + 1;
        c.ny = py + 1;
        c.i0 = g->patch_i0[l - 1];
        c.j0 = g->patch_j0[l - 1];
        c.sp = a.sp / 2;
        c.ox = a.ox + c.i0 * a.sp;
        c.oy = a.oy + c.j0 * a.sp;
        c.perim_inactive = true;
        a.has_child = true;
        a.ci0 = c.i0;
        a.cj0 = c.j0;
        a.ci1 = c.i0 + px / 2;
        a.cj1 = c.j0 + py / 2;
        const int lo = (a.perim_inactive ? 2 : 2);
        if (a.ci0 < lo || a.cj0 < lo || a.ci1 > a.nx - 1 - lo || a.cj1 > a.ny - 1 - lo)
            return fail(err, HLBM_E_GEOMETRY, "box %d does not fit inside its parent with a two-node margin", l);
        if (px / 2 < 4 || py / 2 < 4) return fail(err, HLBM_E_GEOMETRY, "box %d too small", l);
    }
    for (int l = 0; l <= p.L; ++l) {
        LevelPlan& v = p.lev[l];
        v.tau = 0.5 + (p.tau_s - 0.5) / double(1 << (p.L - l));
        if (!(v.tau > 0.5)) return fail(err, HLBM_E_PARAM, "tau <= 1/2 on level %d", l);
        const int al = p.elem == 8 ? 32 : 64;   // 256-byte rows
        v.pitch = (v.nx + al - 1) / al * al;
    }
    LevelPlan& fl = p.lev[p.L];
    // ---- inner ellipse, or a body resolved by bounce-back: inactive nodes of the
    // finest level (one span per row)
    const bool has_ein = p.has_mesh && m->inner_ellipse[2] > 0 && m->inner_ellipse[3] > 0;
    std::vector<uint8_t> inside;   // finest level, 1 = strictly inside the inner ellipse or the body
    if (p.has_body) {
        if (p.has_mesh || (m->inner_ellipse[2] > 0 && m->inner_ellipse[3] > 0))
            return fail(err, HLBM_E_ARG, "a body resolved by bounce-back excludes a mesh and an inner ellipse");
        if (m->body_n < 3 || !m->body_xy) return fail(err, HLBM_E_ARG, "the body needs at least 3 vertices");
    }
    if (has_ein || p.has_body) {
        inside.assign(size_t(fl.nx) * fl.ny, 0);
        int jmin = fl.ny, jmax = -1;
        for (int j = 0; j < fl.ny; ++j)
            for (int i = 0; i < fl.nx; ++i) {
                const double x = fl.ox + i * fl.sp, y = fl.oy + j * fl.sp;
                bool in;
                if (has_ein) {
                    const double dx = (x - m->inner_ellipse[0]) / m->inner_ellipse[2];
                    const double dy = (y - m->inner_ellipse[1]) / m->inner_ellipse[3];
                    in = dx * dx + dy * dy < 1.0;
                } else {
                    in = polygon_contains(m->body_n, m->body_xy, x, y);
                }
                if (in) {
                    inside[size_t(j) * fl.nx + i] = 1;
                    jmin = std::min(jmin, j);
                    jmax = std::max(jmax, j);
                }
            }
        if (p.has_body && jmax < 0) return fail(err, HLBM_E_GEOMETRY, "the body covers no node of the finest level");
        // the body keeps clear of the finest level's edge by 6 nodes: the refinement
        // transfers and the far-field conditions read there without bounce-back
        const int margin = p.has_body ? 6 : 2;
        if (jmax >= 0) {
            fl.sj0 = jmin;
            fl.sj1 = jmax + 1;
            for (int j = fl.sj0; j < fl.sj1; ++j) {
                int lo = -1, hi = -1;
                for (int i = 0; i < fl.nx; ++i)
                    if (inside[size_t(j) * fl.nx + i]) {
                        if (lo < 0) lo = i;
                        if (hi >= 0 && hi != i) return fail(err, HLBM_E_GEOMETRY, "inactive region not convex in row %d", j);
                        hi = i + 1;
                    }
                if (lo < 0) lo = hi = 0;
                if (lo < margin || hi > fl.nx - margin || j < margin || j > fl.ny - 1 - margin)
                    return fail(err, HLBM_E_GEOMETRY, p.has_body ? "the body is too close to the edge of the finest level"
                                                                 : "inner ellipse too close to the edge of the finest level");
                p.spans.push_back(lo);
                p.spans.push_back(hi);
            }
        }
    }
    auto collide_node = [&](int l, int i, int j) -> bool {   // is (i, j) a collide-stream node of level l
        const LevelPlan& v = p.lev[l];
        if (i < 0 || j < 0 || i >= v.nx || j >= v.ny) return false;
        if (v.perim_inactive && (i == 0 || j == 0 || i == v.nx - 1 || j == v.ny - 1)) return false;
        if (v.has_child && i > v.ci0 && i < v.ci1 && j > v.cj0 && j < v.cj1) return false;
        if (l == p.L && !inside.empty() && inside[size_t(j) * v.nx + i]) return false;
        return true;
    };
    if (p.has_body) {   // bounce-back links of the collide-stream nodes next to the body
        for (int j = std::max(1, fl.sj0 - 1); j <= std::min(fl.ny - 2, fl.sj1); ++j)
            for (int i = 1; i < fl.nx - 1; ++i) {
                if (!collide_node(p.L, i, j)) continue;
                int mask = 0;
                for (int q = 1; q < 9; ++q)
                    if (inside[size_t(j - kCy[q]) * fl.nx + (i - kCx[q])]) mask |= 1 << q;
                if (!mask) continue;
                p.bounce_node.push_back(i + fl.nx * j);
                p.bounce_mask.push_back(mask);
            }
        for (uint8_t v : inside) p.n_solid += v;
    }
    for (int l = 0; l <= p.L; ++l) {
        const LevelPlan& v = p.lev[l];
        int64_t n = int64_t(v.nx) * v.ny;
        if (v.perim_inactive) n -= 2 * int64_t(v.nx + v.ny) - 4;
        if (v.has_child) n -= int64_t(v.ci1 - v.ci0 - 1) * (v.cj1 - v.cj0 - 1);
        if (l == p.L)
            for (size_t a = 0; a < p.spans.size(); a += 2) n -= p.spans[a + 1] - p.spans[a];
        p.lev[l].active = n;
    }

    // ---- mesh
    if (p.has_mesh) {
        if (!m->xy || !m->tri || !m->kind || m->n_tris <= 0) return fail(err, HLBM_E_ARG, "mesh arrays missing");
        const int nn = m->n_nodes, nt = m->n_tris;
        p.nn = nn;
        p.nt = nt;
        for (int a = 0; a < nn; ++a)
            if (m->kind[a] > 2) return fail(err, HLBM_E_ARG, "node kind must be 0, 1 or 2");
        std::vector<Entry> ent;
        std::vector<double> area;
        std::vector<std::array<int, 2>> bnd;
        int rc = median_dual(nn, nt, m->xy, m->tri, ent, area, bnd, err);
        if (rc) return rc;
        p.mxy.assign(m->xy, m->xy + 2 * size_t(nn));
        p.mtri.assign(m->tri, m->tri + 3 * size_t(nt));
        if (m->n_shape < 0 || (m->n_shape > 0 && !m->dxy_dshape))
            return fail(err, HLBM_E_ARG, "n_shape must be >= 0, with dxy_dshape given when it is positive");
        p.n_shape = m->n_shape;
        if (p.n_shape > 0) p.dshape.assign(m->dxy_dshape, m->dxy_dshape + size_t(p.n_shape) * 2 * nn);
        p.mbnd = bnd;
        std::vector<int> rp(nn + 1, 0), cl(ent.size());
        for (const Entry& e : ent) rp[e.p + 1]++;
        for (int a = 0; a < nn; ++a) rp[a + 1] += rp[a];
        for (size_t z = 0; z < ent.size(); ++z) cl[z] = ent[z].k;
        // node order: RCM, then stable partition [wall | interior | interpolation]
        const std::vector<int> rcm = rcm_order(nn, rp, cl, m->kind);
        p.perm.clear();
        for (int kindsel : {1, 0, 2})
            for (int a : rcm)
                if (m->kind[a] == kindsel) p.perm.push_back(a);
        std::vector<int> inv(nn);
        for (int a = 0; a < nn; ++a) inv[p.perm[a]] = a;
        p.n_wall = 0;
        p.n_int = 0;
        for (int a = 0; a < nn; ++a) p.n_wall += m->kind[a] == 1, p.n_int += m->kind[a] == 2;
        p.n_core = nn - p.n_int;
        // CSR in plan order: self entry first, then neighbours by plan index
        p.rowptr.assign(nn + 1, 0);
        p.col.clear();
        p.gx.clear();
        p.gy.clear();
        p.cc.clear();
        for (int P = 0; P < nn; ++P) {
            const int o = p.perm[P];
            std::vector<std::pair<int, int>> row;   // (new col, entry index)
            for (int z = rp[o]; z < rp[o + 1]; ++z) row.emplace_back(inv[cl[z]], z);
            std::sort(row.begin(), row.end(), [&](const std::pair<int, int>& a, const std::pair<int, int>& b) {
                const bool sa = a.first == P, sb = b.first == P;
                if (sa != sb) return sa;
                return a.first < b.first;
            });
            for (auto& pr : row) {
                p.col.push_back(pr.first);
                p.gx.push_back(ent[pr.second].gx);
                p.gy.push_back(ent[pr.second].gy);
                p.cc.push_back(ent[pr.second].c);
            }
            p.rowptr[P + 1] = int(p.col.size());
        }
        int maxrow = 0;
        for (int P = 0; P < nn; ++P) maxrow = std::max(maxrow, p.rowptr[P + 1] - p.rowptr[P]);
        if (maxrow > 16) return fail(err, HLBM_E_GEOMETRY, "a mesh node has %d neighbours (at most 15 supported)", maxrow - 1);
        p.ell_width = maxrow <= 8 ? 8 : 16;
        // tile tables drop the eighth slot when no node has seven neighbours
        p.ft_width = maxrow <= 7 ? 7 : p.ell_width;
        // wall edges: boundary edges with both ends on the wall
        for (const auto& be : bnd)
            if (m->kind[be[0]] == 1 && m->kind[be[1]] == 1) {
                p.wedge.push_back(inv[be[0]]);
                p.wedge.push_back(inv[be[1]]);
                const double dx = m->xy[2 * be[1]] - m->xy[2 * be[0]], dy = m->xy[2 * be[1] + 1] - m->xy[2 * be[0] + 1];
                p.wnorm.push_back(dy);
                p.wnorm.push_back(-dx);
            }
        // fused FV sub-steps: fv_fuse per launch when a tile with its rings fits
        // in the LDS of a workgroup (kFvLds, kFvLdsWide) and a workgroup of at
        // most 256 threads (512 for the FP32 8-slot tiles) covers the nodes of
        // sub-step 1 with kFvStage nodes per thread, else fewer (one kernel per
        // sub-step when not even two fit)
        if (g->fv_fuse < 0 || g->fv_fuse > kMaxFuse) return fail(err, HLBM_E_ARG, "fv_fuse must be 0..%d", kMaxFuse);
        const bool wide = p.elem == 4 && p.ell_width <= 8;   // 512-thread FP32 workgroups
        const int fuse = g->fv_fuse > 0 ? g->fv_fuse : (p.ell_width <= 8 ? (wide ? kMaxFuse : kFvFuse) : 1);
        // the largest count from the requested one down to two whose tiles fit
        p.fv_fuse = 1;
        for (int k = fuse; k > 1; --k) {
            choose_fv_tiles(p, k);
            const int need = (p.fv_maxw + kFvStage - 1) / kFvStage;
            p.fv_threads = wide ? kFvThreadsWide
                                : std::max(p.elem == 8 ? kFvThreadsF64 : kFvThreadsF32, (need + 63) / 64 * 64);
            const int cap = wide ? kFvThreadsWide : kFvThreadsF32;
            const size_t lds = fv_lds_bytes(p.fv_maxl, p.fv_maxs, k, p.elem);
            // at most kFvStage updated nodes and one staged f* node per thread
            if (lds <= (wide ? kFvLdsWide : kFvLds) && need <= p.fv_threads && p.fv_threads <= cap &&
                p.fv_maxs <= p.fv_threads)
                break;
            p.fv_fuse = 1;
            p.n_tiles = 0;
            p.ft_meta.clear();
            p.ft_node.clear();
            p.ft_col.clear();
            p.ft_src.clear();
            p.ft_star.clear();
        }
        // wall statistics: unit normal into the fluid at each wall node (opposite
        // to half the sum of its wall-edge normals) and its output slot
        p.wall_nrm.assign(2 * size_t(p.n_wall), 0.0);
        for (size_t e = 0; e < p.wedge.size() / 2; ++e)
            for (int end = 0; end < 2; ++end) {
                const int P = p.wedge[2 * e + end];
                p.wall_nrm[2 * P] += 0.5 * p.wnorm[2 * e];
                p.wall_nrm[2 * P + 1] += 0.5 * p.wnorm[2 * e + 1];
            }
        for (int P = 0; P < p.n_wall; ++P) {
            const double vx = p.wall_nrm[2 * P], vy = p.wall_nrm[2 * P + 1], len = std::sqrt(vx * vx + vy * vy);
            if (!(len > 0)) return fail(err, HLBM_E_GEOMETRY, "wall node %d has no wall edge", p.perm[P]);
            p.wall_nrm[2 * P] = -vx / len;
            p.wall_nrm[2 * P + 1] = -vy / len;
        }
        {
            std::vector<int> order(p.n_wall);
            for (int P = 0; P < p.n_wall; ++P) order[P] = P;
            std::sort(order.begin(), order.end(), [&](int a, int b) { return p.perm[a] < p.perm[b]; });
            p.wall_slot.assign(p.n_wall, 0);
            for (int r = 0; r < p.n_wall; ++r) p.wall_slot[order[r]] = r;
        }
        // ---- coupling stencils
        const bool linear = p.interp == HLBM_INTERP_LINEAR;
        if (has_ein) {
            TriIndex T;
            build_tri_index(nn, nt, m->xy, m->tri, T);
            for (int j = fl.sj0; j < fl.sj1; ++j) {
                const int lo = p.spans[2 * (j - fl.sj0)], hi = p.spans[2 * (j - fl.sj0) + 1];
                for (int i = lo; i < hi; ++i) {
                    bool edge = false;
                    for (int q = 1; q < 9 && !edge; ++q) edge = collide_node(p.L, i + kCx[q], j + kCy[q]);
                    if (!edge) continue;
                    const double x = fl.ox + i * fl.sp, y = fl.oy + j * fl.sp;
                    int don[kSDon];
                    double w[kSDon];
                    bool fb = false;
                    const int nd = mesh_stencil(T, m->xy, m->tri, x, y, linear, don, w, fb);
                    if (nd < 0) return fail(err, HLBM_E_GEOMETRY, "structured interpolation node (%d,%d) is outside the mesh", i, j);
                    p.n_fallback += fb;
                    p.sint_node.push_back(i + fl.nx * j);
                    for (int d = 0; d < kSDon; ++d) {
                        p.sint_don.push_back(d < nd ? inv[don[d]] : -1);
                        p.sint_w.push_back(d < nd ? w[d] : 0.0);
                    }
                }
            }
        }
        for (int s = 0; s < p.n_int; ++s) {
            const int o = p.perm[p.n_core + s];
            const double x = m->xy[2 * o] - fl.ox, y = m->xy[2 * o + 1] - fl.oy;   // finest spacing is 1
            int di[9], dj[9];
            double w[9];
            const int nd = lagrange9<double>(x, y, linear, di, dj, w);
            for (int d = 0; d < kUDon; ++d) {
                if (d < nd) {
                    const bool interior = di[d] >= 1 && dj[d] >= 1 && di[d] <= fl.nx - 2 && dj[d] <= fl.ny - 2;
                    if (!interior || !collide_node(p.L, di[d], dj[d]))
                        return fail(err, HLBM_E_GEOMETRY,
                                    "mesh interpolation node %d: donor (%d,%d) is not a collide-stream node of the finest level", o, di[d], dj[d]);
                    p.uint_don.push_back(di[d] + fl.nx * dj[d]);
                    p.uint_w.push_back(w[d]);
                } else {
                    p.uint_don.push_back(-1);
                    p.uint_w.push_back(0.0);
                }
            }
        }
    } else if (has_ein) {
        return fail(err, HLBM_E_GEOMETRY, "an inactive region needs a mesh");
    }

    // ---- workspace layout
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + std::max<size_t>(bytes, 1));
        return o;
    };
    const size_t E = p.elem;
    for (int l = 0; l <= p.L; ++l) {
        const size_t lb = size_t(kQ) * p.lev[l].ny * p.lev[l].pitch * E;
        p.off.lev[l][0] = take(lb);
        p.off.lev[l][1] = take(lb);
    }
    for (int l = 0; l < p.L; ++l) {
        const LevelPlan& v = p.lev[l];
        const size_t nb = 2 * size_t((v.ci1 - v.ci0) + (v.cj1 - v.cj0));
        p.off.side[l][0] = take(nb * kMacro * E);
        p.off.side[l][1] = take(nb * kMacro * E);
    }
    p.off.spans = take(p.spans.size() * 4);
    p.off.bounce_node = take(p.bounce_node.size() * 4);
    p.off.bounce_mask = take(p.bounce_mask.size() * 4);
    const size_t ns = p.sint_node.size();
    p.off.sint_node = take(ns * 4);
    p.off.sint_don = take(ns * kSDon * 4);
    p.off.sint_w = take(ns * kSDon * E);
    const size_t nnp = size_t(std::max(p.nn, 1));
    p.off.mesh[0] = take(kRec * nnp * E);
    p.off.mesh[1] = take(kRec * nnp * E);
    p.off.rowptr = take((nnp + 1) * 4);
    p.off.edges = take(size_t(p.ell_width) * nnp * (E == 8 ? 32 : 16));
    p.off.wedge = take(p.wedge.size() * 4);
    p.off.wnorm = take(p.wnorm.size() * 8);
    p.off.prep[0] = take(size_t(std::max(p.n_int, 1)) * kMacro * E);
    p.off.prep[1] = take(size_t(std::max(p.n_int, 1)) * kMacro * E);
    p.off.uint_don = take(p.uint_don.size() * 4);
    p.off.uint_w = take(p.uint_w.size() * E);
    p.off.hist = take(size_t(p.hist_len) * 2 * 8);
    p.off.wall_nrm = take(size_t(p.n_wall) * 2 * 8);
    p.off.wall_slot = take(size_t(p.n_wall) * 4);
    p.off.wsum = take(size_t(p.n_wall) * 3 * 8);
    p.off.wout = take(size_t(p.n_wall) * 3 * 8);
    p.off.ft_meta = take(p.ft_meta.size() * 4);
    p.off.ft_node = take(p.ft_node.size() * 4);
    p.off.ft_edges = take(p.ft_col.size() * (E == 8 ? 32 : 16));
    p.off.ft_star = take(p.ft_star.size() * 4);
    size_t maxrow = 0;
    for (int l = 0; l <= p.L; ++l) maxrow = std::max(maxrow, size_t(p.lev[l].nx));
    p.stage_bytes = std::max(size_t(kQ) * maxrow * 8 * 8, std::min(size_t(32) << 20, size_t(kQ) * maxrow * 8 * 4096));
    p.stage_bytes = std::max(p.stage_bytes, size_t(kQ) * nnp * 8);
    p.off.stage = take(p.stage_bytes);
    p.off.total = off;
    return HLBM_OK;
}

int mesh_geometry_adjoint(const Plan& p, const double* gbar, const double* vbar, const double* w5bar,
                          const double* w6bar, double* grad, std::string& err) {
    const int nn = p.nn, nt = p.nt;
    const double* xy = p.mxy.data();
    const int32_t* tri = p.mtri.data();
    auto P_of = [&](int v) { return V2{xy[2 * v], xy[2 * v + 1]}; };
    // control-volume areas, as in the forward
    std::vector<double> area(nn, 0.0);
    for (int t = 0; t < nt; ++t) {
        const int v[3] = {tri[3 * t], tri[3 * t + 1], tri[3 * t + 2]};
        const double at = 0.5 * cross(P_of(v[1]) - P_of(v[0]), P_of(v[2]) - P_of(v[0]));
        for (int r = 0; r < 3; ++r) area[v[r]] += at / 3.0;
    }
    // adjoints of the raw (undivided) row entries and of the areas, keyed by caller ids
    std::vector<std::vector<std::pair<int, std::array<double, 3>>>> rowbar(nn);
    std::vector<double> abar(nn, 0.0);
    for (int P = 0; P < nn; ++P) {
        const int o = p.perm[P];
        for (int zz = p.rowptr[P]; zz < p.rowptr[P + 1]; ++zz) {
            const int z = zz - p.rowptr[P];
            const double* g = gbar + (size_t(z) * nn + P) * 3;
            rowbar[o].push_back({p.perm[p.col[zz]], {g[0] / area[o], g[1] / area[o], g[2] / area[o]}});
            abar[o] -= (g[0] * p.gx[zz] + g[1] * p.gy[zz] + g[2] * p.cc[zz]) / area[o];
        }
    }
    auto rb = [&](int o, int k) -> const std::array<double, 3>& {
        for (const auto& e : rowbar[o])
            if (e.first == k) return e.second;
        static const std::array<double, 3> zero{0.0, 0.0, 0.0};
        return zero;
    };
    // triangle corners: local forward mode over the six vertex coordinates
    for (int t = 0; t < nt; ++t) {
        const int v[3] = {tri[3 * t], tri[3 * t + 1], tri[3 * t + 2]};
        for (int c = 0; c < 6; ++c) {
            V2T<Dual> X[3];
            for (int a = 0; a < 3; ++a)
                X[a] = {Dual{xy[2 * v[a]], c == 2 * a ? 1.0 : 0.0}, Dual{xy[2 * v[a] + 1], c == 2 * a + 1 ? 1.0 : 0.0}};
            const Dual at = 0.5 * cross(X[1] - X[0], X[2] - X[0]);
            double d = 0.0;
            for (int r = 0; r < 3; ++r) {
                const int P = v[r], A = v[(r + 1) % 3], B = v[(r + 2) % 3];
                Dual o[9];
                corner_terms<Dual>(X[r], X[(r + 1) % 3], X[(r + 2) % 3], at, o);
                const auto &bP = rb(P, P), &bA = rb(P, A), &bB = rb(P, B);
                d += o[0].d * bP[0] + o[1].d * bP[1] + o[6].d * bP[2];
                d += o[2].d * bA[0] + o[3].d * bA[1] + o[7].d * bA[2];
                d += o[4].d * bB[0] + o[5].d * bB[1] + o[8].d * bB[2];
                d += (at.d / 3.0) * abar[P];
            }
            grad[2 * v[c / 2] + c % 2] += d;
        }
    }
    // half boundary edges: (P,P) and (Q,Q) get -3/4 nh, (P,Q) and (Q,P) -1/4 nh,
    // nh = (y_Q - y_P, -(x_Q - x_P)) / 2
    for (const auto& be : p.mbnd) {
        const int P = be[0], Q = be[1];
        double nb[2];
        for (int a = 0; a < 2; ++a)
            nb[a] = -0.75 * rb(P, P)[a] - 0.25 * rb(P, Q)[a] - 0.75 * rb(Q, Q)[a] - 0.25 * rb(Q, P)[a];
        grad[2 * Q + 1] += 0.5 * nb[0];
        grad[2 * P + 1] -= 0.5 * nb[0];
        grad[2 * Q] -= 0.5 * nb[1];
        grad[2 * P] += 0.5 * nb[1];
    }
    // wall normals N_e = (y_b - y_a, -(x_b - x_a)); V_P = sum of N_e / 2 over P's wall edges
    for (size_t e = 0; e < p.wedge.size() / 2; ++e) {
        const int a = p.wedge[2 * e], b = p.wedge[2 * e + 1];
        const double nx = 0.5 * (vbar[2 * a] + vbar[2 * b]), ny = 0.5 * (vbar[2 * a + 1] + vbar[2 * b + 1]);
        const int ao = p.perm[a], bo = p.perm[b];
        grad[2 * bo + 1] += nx;
        grad[2 * ao + 1] -= nx;
        grad[2 * bo] -= ny;
        grad[2 * ao] += ny;
    }
    const bool linear = p.interp == HLBM_INTERP_LINEAR;
    const LevelPlan& fl = p.lev[p.L];
    // eq. (4) weights: forward mode per donor coordinate through the same stencil code
    if (!p.sint_node.empty()) {
        TriIndex T;
        build_tri_index(nn, nt, xy, tri, T);
        std::vector<Dual> xyd(2 * size_t(nn));
        for (size_t a = 0; a < xyd.size(); ++a) xyd[a] = {xy[a], 0.0};
        for (size_t s = 0; s < p.sint_node.size(); ++s) {
            const int id = p.sint_node[s], i = id % fl.nx, j = id / fl.nx;
            const double x = fl.ox + i * fl.sp, y = fl.oy + j * fl.sp;
            int don0[kSDon], nd0 = 0;
            for (int d = 0; d < kSDon; ++d) {
                const int k = p.sint_don[s * kSDon + d];
                if (k < 0) break;
                don0[nd0++] = p.perm[k];
            }
            for (int a = 0; a < nd0; ++a)
                for (int c = 0; c < 2; ++c) {
                    Dual& seed = xyd[2 * size_t(don0[a]) + c];
                    seed.d = 1.0;
                    int don[kSDon];
                    Dual w[kSDon];
                    bool fb = false;
                    const int nd = mesh_stencil<Dual>(T, xyd.data(), tri, x, y, linear, don, w, fb);
                    seed.d = 0.0;
                    if (nd != nd0) return fail(err, HLBM_E_STATE, "eq. (4) stencil %zu changed in the shape adjoint", s);
                    double g = 0.0;
                    for (int d = 0; d < nd; ++d) {
                        if (don[d] != don0[d]) return fail(err, HLBM_E_STATE, "eq. (4) stencil %zu changed in the shape adjoint", s);
                        g += w5bar[s * kSDon + d] * w[d].d;
                    }
                    grad[2 * size_t(don0[a]) + c] += g;
                }
        }
    }
    // eq. (9) weights: each depends on its own mesh node's coordinates only
    for (int s = 0; s < p.n_int; ++s) {
        const int o = p.perm[p.n_core + s];
        for (int c = 0; c < 2; ++c) {
            const Dual x{xy[2 * o] - fl.ox, c == 0 ? 1.0 : 0.0}, y{xy[2 * o + 1] - fl.oy, c == 1 ? 1.0 : 0.0};
            int di[9], dj[9];
            Dual w[9];
            const int nd = lagrange9<Dual>(x, y, linear, di, dj, w);
            double g = 0.0;
            for (int d = 0; d < nd; ++d) g += w6bar[size_t(s) * kUDon + d] * w[d].d;
            grad[2 * o + c] += g;
        }
    }
    return HLBM_OK;
}

}  // namespace hlbm
