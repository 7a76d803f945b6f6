// kernels.hip -- HIP kernels of the HLBM step for gfx950 (MI355X).
//
// Storage: structure-of-arrays populations [9][ny][pitch] per level with
// 256-byte rows, double-buffered; the buffer holds post-collision values and
// the collide-stream kernel pulls f_i(x - c_i) from it (eq. (1)), collides and
// writes the next post-collision state.  Two instantiations:
//   <double, false>  FP64 populations f_i;
//   <float,  true>   FP32 populations stored as the shift f_i - w_i rho0
//                    (forces are still accumulated in FP64).
// Everything on this path is bandwidth bound (a few flops per byte), so there
// is no matrix-core (MFMA) work: the kernels are plain coalesced streams.
#include <hip/hip_runtime.h>

#include <mutex>

#include "hlbm_internal.h"

namespace hlbm {
namespace {

constexpr int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

template <typename T>
__device__ __forceinline__ T wgt(int q) {
    return q == 0 ? T(4.0 / 9.0) : (q < 5 ? T(1.0 / 9.0) : T(1.0 / 36.0));
}

// Macroscopic state of stored populations: rho (full), drho = rho - rho0
// (shifted storage only), velocity.
// First moments sum_i c_i g_i with the velocity components written out (c has
// entries -1, 0, 1), in the order of increasing i.
template <typename T>
__device__ __forceinline__ T moment_x(const T (&g)[9]) {
    return ((((g[1] - g[3]) + g[5]) - g[6]) - g[7]) + g[8];
}
template <typename T>
__device__ __forceinline__ T moment_y(const T (&g)[9]) {
    return ((((g[2] - g[4]) + g[5]) + g[6]) - g[7]) - g[8];
}

template <typename T, bool SHIFT>
__device__ __forceinline__ void macro(const T (&f)[9], T rho0, T& rho, T& drho, T& ux, T& uy) {
    T s = 0;
#pragma unroll
    for (int q = 0; q < 9; ++q) s += f[q];
    const T mx = moment_x(f), my = moment_y(f);
    if (SHIFT) {
        drho = s;
        rho = rho0 + s;
    } else {
        rho = s;
        drho = s - rho0;
    }
    if constexpr (sizeof(T) == 4) {
        // one reciprocal for both components: the hardware estimate refined by
        // one Newton step (within one unit in the last place of the quotient)
        float r = __builtin_amdgcn_rcpf(rho);
        r = __builtin_fmaf(__builtin_fmaf(-rho, r, 1.0f), r, r);
        ux = mx * r;
        uy = my * r;
    } else {
        ux = mx / rho;
        uy = my / rho;
    }
}

// w_i x in FP32 without a common bias.  Rounded to FP32, 4/9, 1/9 and 1/36
// share one mantissa and so one relative error (+7.5e-9): their sum is not 1
// and their second moment not c_s^2, so every collision would scale the
// momentum by 1 + 7.5e-9 / tau, a body force along the flow that sets up a
// streamwise pressure gradient.  Here w_i = W_i / 36 with W_i in {16, 4, 1}
// (exact) and x / 36 formed with a two-term 1/36, so the only error left is
// the final rounding, of either sign.
// The exact factor W_i (a power of two) is folded into both parts of 1/36.
__device__ __forceinline__ float weighted_f32(int q, float x) {
    constexpr float k_hi = float(1.0 / 36.0);
    constexpr float k_lo = float(1.0 / 36.0 - double(float(1.0 / 36.0)));
    const float w36 = q == 0 ? 16.0f : (q < 5 ? 4.0f : 1.0f);
    return __builtin_fmaf(x, w36 * k_hi, x * (w36 * k_lo));
}


// FP32 conservation repair.  o are post-collision populations of a node whose
// pre-collision ones are g (for a pure collision term pass g = 0).  In exact
// arithmetic the BGK and FV collision terms conserve mass and momentum; in
// FP32 each node leaves a rounding residual, and in near-uniform regions all
// nodes round the same values the same way, so the residuals add up instead
// of cancelling.  The residual of the rounded outputs is moved onto the rest
// population (mass) and the two diagonal pairs (momentum: (5, 7) carries
// x + y, (8, 6) carries x - y), whose stored values are among the smallest.
// Measured: FP32-shifted C_L at Re 1000, 5 deg within 8.3e-5 of FP64 (2.2e-4
// without), C_D at Re 100 within 1e-8 (6e-6).
__device__ __forceinline__ void conserve_f32(const float (&g)[9], float (&o)[9]) {
    float d[9], dm = 0.f;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        d[q] = o[q] - g[q];
        dm += d[q];
    }
    const float dx = moment_x(d), dy = moment_y(d);
    const float ax = 0.25f * dx, ay = 0.25f * dy;
    o[5] -= ax + ay;
    o[7] += ax + ay;
    o[8] -= ax - ay;
    o[6] += ax - ay;
    o[0] -= dm;
}

// Second-order equilibrium of eq. (2) in stored form:
//   FP64:    w_i rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u^2)
//   shifted: w_i (rho - rho0) + w_i rho (3 c.u + 9/2 (c.u)^2 - 3/2 u^2)
// c_i . (x, y) with the components of c_i written out.
template <typename T>
__device__ __forceinline__ T cdot(int q, T x, T y) {
    switch (q) {
    case 1: return x;
    case 2: return y;
    case 3: return -x;
    case 4: return -y;
    case 5: return x + y;
    case 6: return y - x;
    case 7: return -(x + y);
    case 8: return x - y;
    default: return T(0);
    }
}

template <typename T, bool SHIFT>
__device__ __forceinline__ void equilibrium(T rho, T drho, T ux, T uy, T (&feq)[9]) {
    const T uu = ux * ux + uy * uy;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const T cu = cdot(q, ux, uy);
        const T poly = T(3) * cu + T(4.5) * cu * cu - T(1.5) * uu;
        if constexpr (SHIFT && sizeof(T) == 4) feq[q] = weighted_f32(q, drho + rho * poly);
        else if constexpr (SHIFT) feq[q] = wgt<T>(q) * (drho + rho * poly);
        else feq[q] = wgt<T>(q) * rho * (T(1) + poly);
    }
}

template <typename T, bool SHIFT>
__device__ __forceinline__ void macro_neq(const T (&f)[9], T rho0, T& r, T& dr, T& ux, T& uy, T (&neq)[9]) {
    T feq[9];
    macro<T, SHIFT>(f, rho0, r, dr, ux, uy);
    equilibrium<T, SHIFT>(r, dr, ux, uy, feq);
#pragma unroll
    for (int q = 0; q < 9; ++q) neq[q] = f[q] - feq[q];
}

// stored <-> physical population
template <typename T, bool SHIFT>
__device__ __forceinline__ double to_phys(T v, int q, double rho0) {
    return SHIFT ? double(v) + wgt<double>(q) * rho0 : double(v);
}
template <typename T, bool SHIFT>
__device__ __forceinline__ T to_store(double v, int q, double rho0) {
    return SHIFT ? T(v - wgt<double>(q) * rho0) : T(v);
}

__device__ __forceinline__ size_t lidx(const KLevel& L, int q, int i, int j) {
    return size_t(j) * size_t(L.rs) + size_t(q) * L.pitch + i;
}

// Is (i, j) a collide-stream node: not on a refined level's perimeter, not
// strictly inside the child box, not inside the inner ellipse.
__device__ __forceinline__ bool is_active(const KLevel& L, int i, int j) {
    if (L.perim_inactive && (i == 0 || j == 0 || i == L.nx - 1 || j == L.ny - 1)) return false;
    if (i > L.ci0 && i < L.ci1 && j > L.cj0 && j < L.cj1) return false;
    if (L.spans && j >= L.sj0 && j < L.sj1) {
        const int lo = L.spans[2 * (j - L.sj0)], hi = L.spans[2 * (j - L.sj0) + 1];
        if (i >= lo && i < hi) return false;
    }
    return true;
}

// f_i(x, t+1) = f~_i(x - c_i, t): pull of the nine populations of node (i, j)
template <typename T>
__device__ __forceinline__ void pull(const KLevel& L, const T* __restrict__ A, int i, int j, T (&f)[9]) {
    if (L.periodic) {
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            int a = i - CX[q], b = j - CY[q];
            a = a < 0 ? a + L.nx : (a >= L.nx ? a - L.nx : a);
            b = b < 0 ? b + L.ny : (b >= L.ny ? b - L.ny : b);
            f[q] = A[lidx(L, q, a, b)];
        }
    } else {
        const size_t base = size_t(j) * size_t(L.rs) + i;
#pragma unroll
        for (int q = 0; q < 9; ++q)
            f[q] = A[size_t(q) * L.pitch + base - ptrdiff_t(CY[q]) * L.rs - CX[q]];
    }
}

// Streamed (pre-collision) populations of node (i, j), with the far-field
// conditions of the base level (Sec. 4): top and bottom copy the inner
// neighbour; inlet and outlet use non-equilibrium extrapolation with u, resp.
// rho, prescribed; corners belong to the inlet and outlet columns.
template <typename T, bool SHIFT>
__device__ __forceinline__ void streamed(const KLevel& L, const T* __restrict__ A, int i, int j, T (&f)[9]) {
    const bool edge = L.farfield && (i == 0 || j == 0 || i == L.nx - 1 || j == L.ny - 1);
    if (!edge) {
        pull(L, A, i, j, f);
        return;
    }
    const int jc = j < 1 ? 1 : (j > L.ny - 2 ? L.ny - 2 : j);
    if (i != 0 && i != L.nx - 1) {
        pull(L, A, i, jc, f);
        return;
    }
    T g[9];
    pull(L, A, i == 0 ? 1 : L.nx - 2, jc, g);
    const T rho0 = T(L.rho0);
    T r, dr, ux, uy, feq_nb[9], feq_b[9];
    macro<T, SHIFT>(g, rho0, r, dr, ux, uy);
    equilibrium<T, SHIFT>(r, dr, ux, uy, feq_nb);
    if (i == 0) equilibrium<T, SHIFT>(r, dr, T(L.u_in_x), T(L.u_in_y), feq_b);
    else equilibrium<T, SHIFT>(rho0, T(0), ux, uy, feq_b);
#pragma unroll
    for (int q = 0; q < 9; ++q) f[q] = feq_b[q] + (g[q] - feq_nb[q]);
}

// One fused pull-stream + BGK collision (eq. (1)) of every collide-stream
// node of a level that is not a far-field edge node: B = collide(stream(A)).
// Layout [ny][9][pitch]: the nine planes of a row are adjacent, so the three
// rows a node pulls from and the row it writes are close in memory.  One
// thread per node, one row per block (FP64 and periodic levels).  The output
// is written with non-temporal stores: it is not read again before the next
// step.  Edge nodes of the base level are done by k_edges, so this kernel
// keeps the register footprint of the plain pull.
template <typename T, bool SHIFT>
__global__ __launch_bounds__(256) void k_stream_collide(const KLevel L, const T* __restrict__ A, T* __restrict__ B) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= L.nx) return;
    if (L.farfield && (i == 0 || j == 0 || i == L.nx - 1 || j == L.ny - 1)) return;
    if (!is_active(L, i, j)) return;
    const T omega = T(L.omega), rho0 = T(L.rho0);
    T f[9], feq[9], rho, dr, ux, uy;
    pull(L, A, i, j, f);
    macro<T, SHIFT>(f, rho0, rho, dr, ux, uy);
    equilibrium<T, SHIFT>(rho, dr, ux, uy, feq);
    const size_t base = size_t(j) * size_t(L.rs) + i;
    T o[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) o[q] = f[q] - (f[q] - feq[q]) * omega;
    if constexpr (SHIFT && sizeof(T) == 4) conserve_f32(f, o);
#pragma unroll
    for (int q = 0; q < 9; ++q)
        __builtin_nontemporal_store(o[q], B + size_t(q) * L.pitch + base);
}

// Non-periodic FP32 levels: V consecutive nodes per thread, one V-wide load per
// population plane and row and one non-temporal store per plane.  The
// populations that stream along x are taken from the neighbouring lane (one
// lane shift); only the first and last lane of a wavefront load the element
// beyond the wavefront.  Measured on MI355X: two nodes per thread took 5.98
// against 5.38 TB/s for one.  Large levels (far beyond the 256 MB cache) take
// four nodes per thread with 16-byte non-temporal loads, as every stored value
// is read once per step: 413 against 420 us on the 33.6M-node base level of
// the bench workload.  Small levels stay at two with cached loads: their grids
// stay in the cache from step to step, and four nodes per thread with
// non-temporal loads made the Re 1000 grids 11% slower.  FP64 with two nodes
// per thread was 1% slower than one and keeps k_stream_collide.
template <typename T, int V> struct Vec16;
template <> struct Vec16<float, 2> { typedef float type __attribute__((ext_vector_type(2))); };
template <> struct Vec16<float, 4> { typedef float type __attribute__((ext_vector_type(4))); };

// levels of at least this many nodes take four nodes per thread
constexpr size_t kWideLevelNodes = size_t(8) << 20;

template <typename T, bool SHIFT, int V>
__global__ __launch_bounds__(256) void k_stream_collide_vec(const KLevel L, const T* __restrict__ A,
                                                            T* __restrict__ B) {
    typedef typename Vec16<T, V>::type VT;
    const int lane = threadIdx.x & 63;
    const int i0 = V * (blockIdx.x * blockDim.x + threadIdx.x);
    const int j = blockIdx.y;
    if (j == 0 || j == L.ny - 1) return;   // far-field edge rows or box perimeter rows: no pulling node
    bool act[V], any = false;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const int i = i0 + v;
        act[v] = i < L.nx && !(L.farfield && (i == 0 || i == L.nx - 1)) && is_active(L, i, j);
        any = any || act[v];
    }
    // a wave with no active node (inside a child box or the inner ellipse)
    // loads nothing; the others keep every lane for the neighbour shuffles
    if (__ballot(any) == 0) return;
    const bool in_row = i0 < L.pitch;
    T f[V][9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const size_t rowb = size_t(j - CY[q]) * size_t(L.rs) + size_t(q) * L.pitch;
        T a[V];
#pragma unroll
        for (int v = 0; v < V; ++v) a[v] = T(0);
        if (in_row) {
            const VT* src = reinterpret_cast<const VT*>(A + rowb + i0);
            const VT x = V == 4 ? __builtin_nontemporal_load(src) : *src;
#pragma unroll
            for (int v = 0; v < V; ++v) a[v] = x[v];
        }
        if (CX[q] == 0) {
#pragma unroll
            for (int v = 0; v < V; ++v) f[v][q] = a[v];
        } else if (CX[q] == 1) {        // node i pulls from i - 1
            T left = __shfl_up(a[V - 1], 1, 64);
            if (lane == 0) left = (in_row && i0 > 0) ? A[rowb + i0 - 1] : T(0);
            f[0][q] = left;
#pragma unroll
            for (int v = 1; v < V; ++v) f[v][q] = a[v - 1];
        } else {                        // node i pulls from i + 1
            T right = __shfl_down(a[0], 1, 64);
            if (lane == 63) right = (i0 + V < L.pitch) ? A[rowb + i0 + V] : T(0);
#pragma unroll
            for (int v = 0; v < V - 1; ++v) f[v][q] = a[v + 1];
            f[V - 1][q] = right;
        }
    }
    if (!any) return;
    const T omega = T(L.omega), rho0 = T(L.rho0);
    T out[9][V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        T g[9], feq[9], rho, dr, ux, uy, o[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) g[q] = f[v][q];
        macro<T, SHIFT>(g, rho0, rho, dr, ux, uy);
        equilibrium<T, SHIFT>(rho, dr, ux, uy, feq);
#pragma unroll
        for (int q = 0; q < 9; ++q) o[q] = g[q] - (g[q] - feq[q]) * omega;
        if constexpr (SHIFT && sizeof(T) == 4) conserve_f32(g, o);
#pragma unroll
        for (int q = 0; q < 9; ++q) out[q][v] = o[q];
    }
    const size_t base = size_t(j) * size_t(L.rs) + i0;
    bool all = true;
#pragma unroll
    for (int v = 0; v < V; ++v) all = all && act[v];
    if (all) {
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            VT o;
#pragma unroll
            for (int v = 0; v < V; ++v) o[v] = out[q][v];
            __builtin_nontemporal_store(o, reinterpret_cast<VT*>(B + size_t(q) * L.pitch + base));
        }
    } else {
#pragma unroll
        for (int q = 0; q < 9; ++q)
#pragma unroll
            for (int v = 0; v < V; ++v)
                if (act[v]) __builtin_nontemporal_store(out[q][v], B + size_t(q) * L.pitch + base + v);
    }
}

// Far-field edge nodes of the base level (Sec. 4 boundary conditions, see
// streamed()), collided like every other node.  Thread k walks the bottom
// row, the top row, then the left and right columns.
template <typename T, bool SHIFT>
__global__ __launch_bounds__(256) void k_edges(const KLevel L, const T* __restrict__ A, T* __restrict__ B) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int nx = L.nx, ny = L.ny;
    if (k >= 2 * nx + 2 * (ny - 2)) return;
    int i, j;
    if (k < nx) i = k, j = 0;
    else if (k < 2 * nx) i = k - nx, j = ny - 1;
    else if (k < 2 * nx + ny - 2) i = 0, j = k - 2 * nx + 1;
    else i = nx - 1, j = k - 2 * nx - (ny - 2) + 1;
    const T omega = T(L.omega), rho0 = T(L.rho0);
    T f[9], feq[9], rho, dr, ux, uy;
    streamed<T, SHIFT>(L, A, i, j, f);
    macro<T, SHIFT>(f, rho0, rho, dr, ux, uy);
    equilibrium<T, SHIFT>(rho, dr, ux, uy, feq);
    const size_t base = size_t(j) * size_t(L.rs) + i;
    T o[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) o[q] = f[q] - (f[q] - feq[q]) * omega;
    if constexpr (SHIFT && sizeof(T) == 4) conserve_f32(f, o);
#pragma unroll
    for (int q = 0; q < 9; ++q) B[size_t(q) * L.pitch + base] = o[q];
}

// Uniform f^eq(rho, u) in every node of a buffer (stored form).
template <typename T, bool SHIFT>
__global__ void k_fill_uniform(const KLevel L, T* __restrict__ A, double rho, double ux, double uy) {
    const size_t n = size_t(L.ny) * size_t(L.rs);
    const size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int q = int((e / size_t(L.pitch)) % 9);
    const double cu = CX[q] * ux + CY[q] * uy, uu = ux * ux + uy * uy;
    const double fe = wgt<double>(q) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    A[e] = to_store<T, SHIFT>(fe, q, L.rho0);
}

// Canonical export: streamed populations of rows [j0, j1) in FP64, zero at
// nodes that are not collide-stream nodes.  out = [9][j1 - j0][nx].
template <typename T, bool SHIFT>
__global__ void k_export_level(const KLevel L, const T* __restrict__ A, double* __restrict__ out, int j0, int j1) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = j0 + blockIdx.y;
    if (i >= L.nx || j >= j1) return;
    const size_t rows = size_t(j1 - j0), o = size_t(j - j0) * L.nx + i;
    if (!is_active(L, i, j)) {
        for (int q = 0; q < 9; ++q) out[q * rows * L.nx + o] = 0.0;
        return;
    }
    T f[9];
    streamed<T, SHIFT>(L, A, i, j, f);
    for (int q = 0; q < 9; ++q) out[q * rows * L.nx + o] = to_phys<T, SHIFT>(f[q], q, L.rho0);
}

// Canonical import of rows [j0, j1): scatter f_i(x) to A(x - c_i) so that the
// next pull of A returns the imported pre-collision populations.  Far-field
// edge nodes are skipped: their values follow from the boundary conditions.
template <typename T, bool SHIFT>
__global__ void k_import_level(const KLevel L, T* __restrict__ A, const double* __restrict__ in, int j0, int j1) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = j0 + blockIdx.y;
    if (i >= L.nx || j >= j1) return;
    if (!is_active(L, i, j)) return;
    if (L.farfield && (i == 0 || j == 0 || i == L.nx - 1 || j == L.ny - 1)) return;
    const size_t rows = size_t(j1 - j0), o = size_t(j - j0) * L.nx + i;
    for (int q = 0; q < 9; ++q) {
        int a = i - CX[q], b = j - CY[q];
        if (L.periodic) {
            a = (a + L.nx) % L.nx;
            b = (b + L.ny) % L.ny;
        }
        A[lidx(L, q, a, b)] = to_store<T, SHIFT>(in[q * rows * L.nx + o], q, L.rho0);
    }
}

// Position k along the boundary of the child box (in parent nodes):
// bottom row, top row, left column, right column.
__device__ __forceinline__ void box_node(int k, int nxc, int nyc, int& a, int& b) {
    if (k <= nxc) { a = k; b = 0; return; }
    k -= nxc + 1;
    if (k <= nxc) { a = k; b = nyc; return; }
    k -= nxc + 1;
    if (k < nyc - 1) { a = 0; b = k + 1; return; }
    k -= nyc - 1;
    a = nxc;
    b = k + 1;
}
__device__ __forceinline__ int box_index(int a, int b, int nxc, int nyc) {
    if (b == 0) return a;
    if (b == nyc) return nxc + 1 + a;
    if (a == 0) return 2 * (nxc + 1) + b - 1;
    return 2 * (nxc + 1) + (nyc - 1) + b - 1;
}

template <typename T, bool SHIFT>
__device__ __forceinline__ void store_macro(T* dst, const T (&f)[9], T rho0) {
    T r, dr, ux, uy, neq[9];
    macro_neq<T, SHIFT>(f, rho0, r, dr, ux, uy, neq);
    dst[0] = SHIFT ? dr : r;
    dst[1] = ux;
    dst[2] = uy;
#pragma unroll
    for (int q = 0; q < 9; ++q) dst[3 + q] = neq[q];
}

// (rho, u, f^neq) of the parent's streamed populations on the box boundary.
template <typename T, bool SHIFT>
__global__ void k_side_init(const KLevel P, int ci0, int cj0, int nxc, int nyc, const T* __restrict__ A, T* __restrict__ side) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 2 * (nxc + nyc)) return;
    int a, b;
    box_node(k, nxc, nyc, a, b);
    T f[9];
    pull(P, A, ci0 + a, cj0 + b, f);
    store_macro<T, SHIFT>(side + size_t(k) * kMacro, f, T(P.rho0));
}

// Coarse -> fine transfer (Sec. 4, Filippova-Haenel) onto the child perimeter:
// (rho, u, f^neq) of the parent, linear in time at theta and linear in space
// at odd fine nodes; f^neq rescaled by tau_f / (2 tau_c) to a fine
// pre-collision value, collided at tau_f.  With compute_side (theta = 0) the
// threads on even nodes also record the parent's (rho, u, f^neq) at t + 1.
template <typename T, bool SHIFT>
__global__ void k_coarse_to_fine(const KLevel P, const KLevel C, int ci0, int cj0, const T* __restrict__ pA,
                                 T* __restrict__ cA, T* __restrict__ side_cur, const T* __restrict__ side_prev,
                                 T theta, int compute_side, T scale, T omega_f) {
    const int cnx = C.nx - 1, cny = C.ny - 1, nxc = cnx / 2, nyc = cny / 2;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 2 * (cnx + cny)) return;
    int ic, jc;
    box_node(k, cnx, cny, ic, jc);
    const T rho0 = T(P.rho0);
    if (compute_side && !(ic & 1) && !(jc & 1)) {
        T f[9];
        pull(P, pA, ci0 + ic / 2, cj0 + jc / 2, f);
        store_macro<T, SHIFT>(side_cur + size_t(box_index(ic / 2, jc / 2, nxc, nyc)) * kMacro, f, rho0);
    }
    int ka, kb = -1;
    if (!(ic & 1) && !(jc & 1)) ka = box_index(ic / 2, jc / 2, nxc, nyc);
    else if (ic & 1) ka = box_index((ic - 1) / 2, jc / 2, nxc, nyc), kb = box_index((ic + 1) / 2, jc / 2, nxc, nyc);
    else ka = box_index(ic / 2, (jc - 1) / 2, nxc, nyc), kb = box_index(ic / 2, (jc + 1) / 2, nxc, nyc);
    T v[kMacro];
    const T wa = kb < 0 ? T(1) : T(0.5);
#pragma unroll
    for (int m = 0; m < kMacro; ++m) {
        T x = (T(1) - theta) * side_prev[size_t(ka) * kMacro + m];
        if (theta != T(0)) x += theta * side_cur[size_t(ka) * kMacro + m];
        x *= wa;
        if (kb >= 0) {
            T y = (T(1) - theta) * side_prev[size_t(kb) * kMacro + m];
            if (theta != T(0)) y += theta * side_cur[size_t(kb) * kMacro + m];
            x += wa * y;
        }
        v[m] = x;
    }
    const T rho = SHIFT ? rho0 + v[0] : v[0], dr = SHIFT ? v[0] : v[0] - rho0;
    T feq[9];
    equilibrium<T, SHIFT>(rho, dr, v[1], v[2], feq);
    const size_t base = size_t(jc) * size_t(C.rs) + ic;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const T pre = feq[q] + scale * v[3 + q];
        cA[size_t(q) * C.pitch + base] = pre - (pre - feq[q]) * omega_f;
    }
}

// Fine -> coarse transfer (Sec. 4): parent nodes on the first ring inside the
// box get the fine (rho, u) and f^neq rescaled by 2 tau_c / tau_f, collided at
// tau_c.  The fine streamed state is pulled from the child buffer.  With
// `filter` the f^neq is full-weighted over the 3 x 3 fine nodes around the
// coincident one (weights (2 - |di|)(2 - |dj|) / 16, exact in any precision),
// all interior nodes of the child, at least one cell inside its perimeter.
template <typename T, bool SHIFT>
__global__ void k_fine_to_coarse(const KLevel P, const KLevel C, int ci0, int cj0, int nxc, int nyc,
                                 const T* __restrict__ cprev, T* __restrict__ pdst, T scale, T omega_c, int filter) {
    const int rx = nxc - 2, ry = nyc - 2;          // ring box (ci0+1 .. ci0+nxc-1) has rx cells
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 2 * (rx + ry)) return;
    int a, b;
    box_node(k, rx, ry, a, b);
    const int pi = ci0 + 1 + a, pj = cj0 + 1 + b;
    const int fi = 2 * (pi - ci0), fj = 2 * (pj - cj0);
    T f[9], r, dr, ux, uy, neq[9], feq[9];
    pull(C, cprev, fi, fj, f);
    macro_neq<T, SHIFT>(f, T(P.rho0), r, dr, ux, uy, neq);
    if (filter) {
#pragma unroll
        for (int q = 0; q < 9; ++q) neq[q] = T(0);
        for (int dj = -1; dj <= 1; ++dj)
            for (int di = -1; di <= 1; ++di) {
                T g[9], r2, dr2, x2, y2, n2[9];
                const T w = T((2 - abs(di)) * (2 - abs(dj))) * T(0.0625);
                pull(C, cprev, fi + di, fj + dj, g);
                macro_neq<T, SHIFT>(g, T(P.rho0), r2, dr2, x2, y2, n2);
#pragma unroll
                for (int q = 0; q < 9; ++q) neq[q] += w * n2[q];
            }
    }
    equilibrium<T, SHIFT>(r, dr, ux, uy, feq);
    const size_t base = size_t(pj) * size_t(P.rs) + pi;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const T pre = feq[q] + scale * neq[q];
        pdst[size_t(q) * P.pitch + base] = pre - (pre - feq[q]) * omega_c;
    }
}

// Structured interpolation nodes, eq. (4): f~ = f^eq(rho, u) +
// 2 (tau_s - 1) / (2 tau_s - 1) f^neq with rho, u, f^neq interpolated from the
// mesh donors (eq. (8)).  Mesh nodes are records [f_0..f_8, rho (or
// rho - rho0), ux, uy].
template <typename T, bool SHIFT>
__global__ __launch_bounds__(64) void k_mesh_to_struct(const KLevel F, T* __restrict__ A, int n, const int32_t* __restrict__ node,
                                 const int32_t* __restrict__ don, const T* __restrict__ w,
                                 const T* __restrict__ mf, T factor) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const T rho0 = T(F.rho0);
    T acc[kMacro];
#pragma unroll
    for (int m = 0; m < kMacro; ++m) acc[m] = 0;
    // every donor index, then every donor record, in flight together (the list
    // is packed: the first unused slot ends it); then the sums in donor order
    int kd[kSDon];
#pragma unroll
    for (int d = 0; d < kSDon; ++d) kd[d] = don[size_t(s) * kSDon + d];
    T rd[kSDon][kRec];
#pragma unroll
    for (int d = 0; d < kSDon; ++d)
        if (kd[d] >= 0) {
#pragma unroll
            for (int q = 0; q < kRec; ++q) rd[d][q] = mf[size_t(kd[d]) * kRec + q];
        }
#pragma unroll
    for (int d = 0; d < kSDon; ++d) {
        if (kd[d] < 0) break;
        const T* rec = rd[d];
        T f[9], feq[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) f[q] = rec[q];
        const T m0 = rec[9], ux = rec[10], uy = rec[11];
        const T rho = SHIFT ? rho0 + m0 : m0, dr = SHIFT ? m0 : m0 - rho0;
        equilibrium<T, SHIFT>(rho, dr, ux, uy, feq);
        const T ww = w[size_t(s) * kSDon + d];
        acc[0] += ww * m0;
        acc[1] += ww * ux;
        acc[2] += ww * uy;
#pragma unroll
        for (int q = 0; q < 9; ++q) acc[3 + q] += ww * (f[q] - feq[q]);
    }
    const T rho = SHIFT ? rho0 + acc[0] : acc[0], dr = SHIFT ? acc[0] : acc[0] - rho0;
    T feq[9];
    equilibrium<T, SHIFT>(rho, dr, acc[1], acc[2], feq);
    const int id = node[s];
    const int i = id % F.nx, j = id / F.nx;
    const size_t base = size_t(j) * size_t(F.rs) + i;
#pragma unroll
    for (int q = 0; q < 9; ++q) A[size_t(q) * F.pitch + base] = feq[q] + factor * acc[3 + q];
}

// Mesh interpolation nodes <- finest level, eq. (9): (rho, u, f^neq) of the
// streamed populations of the 3 x 3 (or 2 x 2) donor block.
template <typename T, bool SHIFT>
__global__ __launch_bounds__(64) void k_struct_to_mesh(const KLevel F, const T* __restrict__ A, int n, const int32_t* __restrict__ don,
                                 const T* __restrict__ w, T* __restrict__ prep) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const T rho0 = T(F.rho0);
    T acc[kMacro];
#pragma unroll
    for (int m = 0; m < kMacro; ++m) acc[m] = 0;
    // every donor index, then every donor's pulled populations, in flight
    // together (the list is packed: the first unused slot ends it); then the
    // sums in donor order
    int idd[kUDon];
#pragma unroll
    for (int d = 0; d < kUDon; ++d) idd[d] = don[size_t(s) * kUDon + d];
    T fd[kUDon][9];
#pragma unroll
    for (int d = 0; d < kUDon; ++d)
        if (idd[d] >= 0) pull(F, A, idd[d] % F.nx, idd[d] / F.nx, fd[d]);
#pragma unroll
    for (int d = 0; d < kUDon; ++d) {
        const int id = idd[d];
        if (id < 0) break;
        T r, dr, ux, uy, neq[9];
        const T(&f)[9] = fd[d];
        macro_neq<T, SHIFT>(f, rho0, r, dr, ux, uy, neq);
        const T ww = w[size_t(s) * kUDon + d];
        acc[0] += ww * (SHIFT ? dr : r);
        acc[1] += ww * ux;
        acc[2] += ww * uy;
#pragma unroll
        for (int q = 0; q < 9; ++q) acc[3 + q] += ww * neq[q];
    }
#pragma unroll
    for (int m = 0; m < kMacro; ++m) prep[size_t(s) * kMacro + m] = acc[m];
}

// Time fractions theta of the sub-steps of one fused launch (computed on the host).
struct FvTheta {
    double v[kMaxFuse];
};

template <typename T> struct EdgeRec;
template <> struct alignas(32) EdgeRec<double> { int32_t col, pad; double gx, gy, c; };
template <> struct alignas(16) EdgeRec<float> { int32_t col; float gx, gy, c; };

// f* at a mesh interpolation node (eqs. (5)-(6)): the structured (rho, u,
// f^neq) blended linearly in time, f* = f^eq(rho, u) + (1 - 1/(2 tau_s)) f^neq;
// nstar = its non-equilibrium part.  Evaluated without floating-point
// contraction (the equilibrium written out here for that), so that every
// kernel that forms f* rounds it the same way whatever code surrounds the
// call: the fused and the one-sub-step finite-volume kernels give the same
// bits, and an adjoint segment that keeps its sub-step states agrees bit for
// bit with one that recomputes them.
template <typename T, bool SHIFT>
__device__ __forceinline__ void star_values(const T* __restrict__ p0, const T* __restrict__ p1, T theta, T cst,
                                            T rho0, T (&fs)[9], T (&ns)[9]) {
#pragma clang fp contract(off)
    T v[kMacro];
#pragma unroll
    for (int m = 0; m < kMacro; ++m) v[m] = (T(1) - theta) * p0[m] + theta * p1[m];
    const T rho = SHIFT ? rho0 + v[0] : v[0], dr = SHIFT ? v[0] : v[0] - rho0;
    const T ux = v[1], uy = v[2], uu = ux * ux + uy * uy;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const T cu = cdot(q, ux, uy);
        const T poly = T(3) * cu + T(4.5) * cu * cu - T(1.5) * uu;
        T feq;
        if constexpr (SHIFT && sizeof(T) == 4) feq = weighted_f32(q, dr + rho * poly);
        else if constexpr (SHIFT) feq = wgt<T>(q) * (dr + rho * poly);
        else feq = wgt<T>(q) * rho * (T(1) + poly);
        ns[q] = cst * v[3 + q];
        fs[q] = feq + ns[q];
    }
}

// Loads one mesh record [f_0..f_8, m0, ux, uy] with 16-byte vector loads.
template <typename T>
__device__ __forceinline__ void load_rec(const T* __restrict__ rec, T (&f)[9], T& m0, T& ux, T& uy) {
    if constexpr (sizeof(T) == 4) {
        const float4* v = reinterpret_cast<const float4*>(rec);
        const float4 a = v[0], b = v[1], c = v[2];
        f[0] = a.x; f[1] = a.y; f[2] = a.z; f[3] = a.w;
        f[4] = b.x; f[5] = b.y; f[6] = b.z; f[7] = b.w;
        f[8] = c.x; m0 = c.y; ux = c.z; uy = c.w;
    } else {
        const double2* v = reinterpret_cast<const double2*>(rec);
        const double2 a = v[0], b = v[1], c = v[2], d = v[3], e = v[4], g = v[5];
        f[0] = a.x; f[1] = a.y; f[2] = b.x; f[3] = b.y; f[4] = c.x; f[5] = c.y;
        f[6] = d.x; f[7] = d.y; f[8] = e.x; m0 = e.y; ux = g.x; uy = g.y;
    }
}

template <typename T>
__device__ __forceinline__ void store_rec(T* __restrict__ rec, const T (&f)[9], T m0, T ux, T uy) {
    if constexpr (sizeof(T) == 4) {
        float4* v = reinterpret_cast<float4*>(rec);
        v[0] = make_float4(f[0], f[1], f[2], f[3]);
        v[1] = make_float4(f[4], f[5], f[6], f[7]);
        v[2] = make_float4(f[8], m0, ux, uy);
    } else {
        double2* v = reinterpret_cast<double2*>(rec);
        v[0] = make_double2(f[0], f[1]); v[1] = make_double2(f[2], f[3]); v[2] = make_double2(f[4], f[5]);
        v[3] = make_double2(f[6], f[7]); v[4] = make_double2(f[8], m0); v[5] = make_double2(ux, uy);
    }
}

template <typename T>
__device__ __forceinline__ void store_wmom(double* w, const T (&pre)[3]) {
    w[0] = double(pre[0]), w[1] = double(pre[1]), w[2] = double(pre[2]);
}

// One finite-volume sub-step of eq. (3) at one mesh node (eq. (5) at the
// interpolation nodes), Jacobi style:
//   f_P <- f_P + dt sum_k (c_i . G_Pk) f_k - dt/tau_u sum_k C_Pk (f_k - f^eq_k)
// The streaming sum is evaluated as sum_{k != P} (c_i . G_Pk)(f_k - f_P),
// equal to the above because sum_k G_Pk = 0 on a closed control volume, and
// exact for a uniform state in any precision.  The collision sum is split as
// sum_k C_Pk f_k - sum_k C_Pk f^eq_k, and because f^eq_i is a quadratic form
// in (rho, rho u) the second part needs only the weighted moments
//   a0 = sum C (rho or rho - rho0),  a1 = sum C rho u,  a2 = sum C rho u u^T:
//   sum_k C_Pk f^eq_i(k) = w_i (a0 + 3 c_i.a1 + 9/2 c_i^T a2 c_i - 3/2 tr a2),
// the same value in a different rounding order, for 20 instead of ~100
// arithmetic instructions per neighbour (the kernel is bound by its vector
// ALU).  Interpolation pivots use f* for themselves and for interpolation
// neighbours (eqs. (5)-(7)), whose non-equilibrium part enters directly;
// wall nodes then get u -> 0 keeping rho and f^neq.  Each record carries the
// node's (rho, u), so neighbours do not recompute them.
template <typename T>
struct FvAcc {
    T base[9], ss[9], sf[9];
    T a0, a1x, a1y, axx, axy, ayy;
};

// Adds slot z (z = 0: the node itself) with populations f of neighbour k:
// regular neighbours give their stored moments (m0, ux, uy); interpolation
// neighbours of an interpolation pivot (star) give their f^neq in nq.
template <typename T, bool SHIFT>
__device__ __forceinline__ void fv_add(FvAcc<T>& A, int z, const T (&f)[9], bool star, const T (&nq)[9], T m0, T ux,
                                       T uy, T gx, T gy, T c, T rho0) {
    if (z == 0) {
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            A.base[q] = f[q];
            A.ss[q] = 0;
            A.sf[q] = 0;
        }
        A.a0 = A.a1x = A.a1y = A.axx = A.axy = A.ayy = 0;
    } else {
        const T gp = gx + gy, gm = gx - gy;
        const T s[9] = {T(0), gx, gy, -gx, -gy, gp, -gm, -gp, gm};   // c_i . G_Pk
#pragma unroll
        for (int q = 1; q < 9; ++q) A.ss[q] += s[q] * (f[q] - A.base[q]);
    }
    if (star) {
#pragma unroll
        for (int q = 0; q < 9; ++q) A.sf[q] += c * nq[q];
    } else {
#pragma unroll
        for (int q = 0; q < 9; ++q) A.sf[q] += c * f[q];
        const T rho = SHIFT ? rho0 + m0 : m0;
        const T cr = c * rho, crx = cr * ux, cry = cr * uy;
        A.a0 += c * m0;
        A.a1x += crx;
        A.a1y += cry;
        A.axx += crx * ux;
        A.axy += crx * uy;
        A.ayy += cry * uy;
    }
}

// New populations and moments of the node from its accumulators.
// pre: (rho, u_x, u_y) of the update before the no-slip reset (wall nodes).
template <typename T, bool SHIFT>
__device__ __forceinline__ void fv_finish(const KMesh& M, int P, const FvAcc<T>& A, T (&fn)[9], T& r, T& dr, T& ux,
                                          T& uy, T (&pre)[3]) {
    const T rho0 = T(M.rho0), dt = T(M.dt), dtt = T(M.dt_over_tau);
    // x_i = a0 + 3 c_i.a1 + 9/2 c_i^T a2 c_i - 3/2 tr a2, with the shared parts
    // b = a0 - 3/2 tr a2 and c_i^T a2 c_i in {0, a_xx, a_yy, tr a2 +- 2 a_xy}
    const T tr = A.axx + A.ayy;
    const T b = A.a0 - T(1.5) * tr;
    const T hxx = T(4.5) * A.axx, hyy = T(4.5) * A.ayy;
    const T hpp = T(4.5) * (tr + T(2) * A.axy), hpm = T(4.5) * (tr - T(2) * A.axy);
    const T sp = A.a1x + A.a1y, sm = A.a1y - A.a1x;
    const T xs[9] = {b,
                     (b + T(3) * A.a1x) + hxx, (b + T(3) * A.a1y) + hyy,
                     (b - T(3) * A.a1x) + hxx, (b - T(3) * A.a1y) + hyy,
                     (b + T(3) * sp) + hpp, (b + T(3) * sm) + hpm,
                     (b - T(3) * sp) + hpp, (b - T(3) * sm) + hpm};
    T col[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const T x = xs[q];
        T eqs;
        if constexpr (SHIFT && sizeof(T) == 4) eqs = weighted_f32(q, x);
        else eqs = wgt<T>(q) * x;
        col[q] = A.sf[q] - eqs;
    }
    if constexpr (SHIFT && sizeof(T) == 4) {
        T zero[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) zero[q] = 0;
        conserve_f32(zero, col);
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) fn[q] = A.base[q] + dt * A.ss[q] - dtt * col[q];
    macro<T, SHIFT>(fn, rho0, r, dr, ux, uy);
    pre[0] = r, pre[1] = ux, pre[2] = uy;
    if (M.wall_bc && P < M.n_wall) {
        T feq[9], feq0[9];
        equilibrium<T, SHIFT>(r, dr, ux, uy, feq);
        equilibrium<T, SHIFT>(r, dr, T(0), T(0), feq0);
#pragma unroll
        for (int q = 0; q < 9; ++q) fn[q] = feq0[q] + (fn[q] - feq[q]);
        macro<T, SHIFT>(fn, rho0, r, dr, ux, uy);
    }
}

// Workgroup -> node block such that each of the 8 dies (dealt workgroups
// round-robin, one L2 each) gets a contiguous range of nodes, whose
// neighbours then mostly sit in the same L2 (measured: -11% FP32, -13% FP64
// sub-step time on the 264k-node mesh).
// The order is reversed: the last node blocks hold the interpolation pivots,
// whose f* work makes them the slowest, and dispatching them first keeps them
// out of the kernel's tail (measured: -5.5% per FP32 sub-step on the
// 264k-node mesh).
__device__ __forceinline__ int die_block(int b, int nb) {
    b = nb - 1 - b;
    const int q = nb / 8, r = nb % 8, x = b % 8, slot = b / 8;
    return x < r ? x * (q + 1) + slot : r * (q + 1) + (x - r) * q + slot;
}

// Neighbour slots whose loads are issued together: all eight in FP32 (168
// VGPRs, 3 waves/SIMD), two in FP64 (188 VGPRs); measured fastest on MI355X
// among 2, 4 and 8 (FP64: 30.3 against 32.0 us per sub-step with four, on
// the 264k-node mesh).
template <typename T> struct FvGroup { static constexpr int value = sizeof(T) == 4 ? 8 : 2; };

template <typename T, bool SHIFT, int W>
__global__ __launch_bounds__(256) void k_fv_substep(const KMesh M, const T* __restrict__ fin, T* __restrict__ fout,
                                                    const T* __restrict__ prep0, const T* __restrict__ prep1, T theta) {
    const int blk = die_block(blockIdx.x, gridDim.x);
    const int P = blk * blockDim.x + threadIdx.x;
    if (P >= M.nn) return;
    const int nn = M.nn;
    const bool pivot_interp = P >= M.n_core;
    const T rho0 = T(M.rho0), cst = T(M.star_neq);
    const EdgeRec<T>* __restrict__ E = reinterpret_cast<const EdgeRec<T>*>(M.edges);
    constexpr int kFvGroup = FvGroup<T>::value;
    FvAcc<T> A;
#pragma unroll 1
    for (int g0 = 0; g0 < W; g0 += kFvGroup) {
        EdgeRec<T> e[kFvGroup];
        T fr[kFvGroup][9], mr[kFvGroup][3];
#pragma unroll
        for (int a = 0; a < kFvGroup; ++a) e[a] = E[size_t(g0 + a) * nn + P];
#pragma unroll
        for (int a = 0; a < kFvGroup; ++a) {
            const int k = e[a].col < 0 ? P : e[a].col;
            load_rec(fin + size_t(k) * kRec, fr[a], mr[a][0], mr[a][1], mr[a][2]);
        }
#pragma unroll
        for (int a = 0; a < kFvGroup; ++a) {
            const int k = e[a].col;
            if (k < 0) continue;
            const bool star = pivot_interp && k >= M.n_core;
            T fs[9], nq[9];
            if (star) {
                const size_t sl = size_t(k - M.n_core) * kMacro;
                star_values<T, SHIFT>(prep0 + sl, prep1 + sl, theta, cst, rho0, fs, nq);
            }
            fv_add<T, SHIFT>(A, g0 + a, star ? fs : fr[a], star, nq, mr[a][0], mr[a][1], mr[a][2], e[a].gx, e[a].gy,
                             e[a].c, rho0);
        }
    }
    T fn[9], r, dr, ux, uy, pre[3];
    fv_finish<T, SHIFT>(M, P, A, fn, r, dr, ux, uy, pre);
    store_rec(fout + size_t(P) * kRec, fn, SHIFT ? dr : r, ux, uy);
    if (M.wmom && P < M.n_wall) store_wmom(M.wmom + 3 * size_t(P), pre);
}

// The rest of a staged f* record [f*_0..f*_8, f^neq_0..f^neq_8, unused x 2]
// after its first twelve values (read like a node record): f^neq_3..f^neq_8.
template <typename T>
__device__ __forceinline__ void load_star_tail(const T* __restrict__ s, T (&nq)[9]) {
    if constexpr (sizeof(T) == 4) {
        const float4 a = reinterpret_cast<const float4*>(s)[3];
        const float2 b = reinterpret_cast<const float2*>(s)[8];
        nq[3] = a.x; nq[4] = a.y; nq[5] = a.z; nq[6] = a.w; nq[7] = b.x; nq[8] = b.y;
    } else {
        const double2* v = reinterpret_cast<const double2*>(s);
        const double2 a = v[6], b = v[7], c = v[8];
        nq[3] = a.x; nq[4] = a.y; nq[5] = b.x; nq[6] = b.y; nq[7] = c.x; nq[8] = c.y;
    }
}

// One node update of the fused kernel: local node i with its edge records e,
// reading the tile state in buf and, for neighbours that enter through f*
// (kFtStar in the edge record), the values staged in st for this sub-step;
// returns the node's plan index.
template <typename T, bool SHIFT, int W>
__device__ __forceinline__ int fv_tile_node(const KMesh& M, const T* __restrict__ buf, const int32_t* gid,
                                            const T* __restrict__ st, int i, const EdgeRec<T> (&e)[W], T (&fn)[9],
                                            T (&mv)[3], double* wmom = nullptr) {
    const T rho0 = T(M.rho0);
    const int P = gid[i];
    FvAcc<T> A;
#pragma unroll
    for (int z = 0; z < W; ++z) {
        const int32_t cz = e[z].col;
        if (cz < 0) continue;
        const bool star = (cz & kFtStar) != 0;
        const int lc = cz & kFtLocal;
        // both record kinds start with the nine populations: one vector read of the
        // first twelve values, then the rest of f^neq for an f* record
        const T* src = star ? st + size_t(lc) * kStarRec : buf + size_t(lc) * kRec;
        T f[9], nq[9], mk, uxk, uyk;
        load_rec(src, f, mk, uxk, uyk);
        if (star) {
            nq[0] = mk; nq[1] = uxk; nq[2] = uyk;
            load_star_tail(src, nq);
        }
        fv_add<T, SHIFT>(A, z, f, star, nq, mk, uxk, uyk, e[z].gx, e[z].gy, e[z].c, rho0);
    }
    T r, dr, pre[3];
    fv_finish<T, SHIFT>(M, P, A, fn, r, dr, mv[1], mv[2], pre);
    mv[0] = SHIFT ? dr : r;
    if (wmom && P < M.n_wall) store_wmom(wmom + 3 * size_t(P), pre);
    return P;
}

// Several FV sub-steps in one launch (temporal blocking).  One workgroup per
// tile of mesh nodes: it loads the records of the tile and of the rings of
// neighbours around it into LDS, takes sub-step j (j = 1..k) on the tile and
// rings 1..k-j, and writes only the tile's records after sub-step k.  Each
// thread updates nodes tid and tid + blockDim (the host sizes the workgroup
// so that these cover every updated node) and holds their new records in
// registers until all reads of the sub-step are done, then writes them back
// in place: one LDS buffer per tile, so that a 264k-node mesh fits the chip
// in a single wave of workgroups.  The rings are recomputed by every tile
// that borders them, so each sub-step is exactly the Jacobi update of
// k_fv_substep, in the same operation order, while HBM sees the records
// and edge coefficients once per k sub-steps.  Tile tables: see
// build_fv_tiles.  Two sub-steps per launch (the default) take a path of
// their own that reuses the edge records of node tid in the second sub-step
// (measured: 19.8 against 22.3 us per launch on the 264k-node mesh, FP32).
// With mid set, the state after each sub-step j < k is
// written too, each tile its own nodes, to mid + (j - 1) * mid_stride (the
// intermediate states that the discrete adjoint reads).
// Waves per SIMD the fused kernel is compiled for: three in FP32 with 8 slots
// (at most 168 VGPRs), so that three workgroups of 256 threads share a CU.
template <typename T, int W> struct FvFusedWaves { static constexpr int value = sizeof(T) == 4 && W <= 8 ? 3 : 1; };
// Largest workgroup of the fused kernel: 512 threads in FP32 (one node per thread
// on meshes with fewer tiles than compute units), 256 in FP64.
template <typename T> struct FvFusedBlock { static constexpr int value = sizeof(T) == 4 ? 512 : 256; };

template <typename T, bool SHIFT, int W>
__global__ __launch_bounds__(FvFusedBlock<T>::value) __attribute__((amdgpu_waves_per_eu(FvFusedWaves<T, W>::value))) void k_fv_fused(const KMesh M, const T* __restrict__ fin, T* __restrict__ fout,
                                                  const T* __restrict__ prep0, const T* __restrict__ prep1,
                                                  FvTheta th, int ksteps, T* __restrict__ mid, size_t mid_stride) {
    extern __shared__ __align__(16) unsigned char smem[];
    T* const buf = reinterpret_cast<T*>(smem);
    int32_t* const gid = reinterpret_cast<int32_t*>(buf + size_t(M.maxl) * kRec);
    // f* of the tile's interpolation nodes, sub-step j of the launch at stg + j * stj
    T* const stg = reinterpret_cast<T*>(smem + fv_stg_offset(M.maxl, sizeof(T)));
    const size_t stj = size_t(M.maxs) * kStarRec;
    const int t = die_block(blockIdx.x, gridDim.x);
    const int32_t* meta = M.ft_meta + size_t(t) * kTileMeta;
    const int noff = meta[0], eoff = meta[1], width = meta[2];
    const int nload = meta[3 + ksteps], ntile = meta[3];
    const EdgeRec<T>* __restrict__ E = reinterpret_cast<const EdgeRec<T>*>(M.ft_edges) + eoff;
    // structured values (t, t + 1) of this thread's interpolation node, if the tile
    // stages one for it (at most one per thread), loaded before the records
    const int soff = meta[8], ns = meta[9];
    const bool has_star = int(threadIdx.x) < ns;
    T sp0[kMacro], sp1[kMacro];
    if (has_star) {
        const size_t sl = size_t(M.ft_star[soff + threadIdx.x]) * kMacro;
#pragma unroll
        for (int m = 0; m < kMacro; ++m) sp0[m] = prep0[sl + m], sp1[m] = prep1[sl + m];
    }
    // records of the tile and its rings: all loads of a batch in flight together
    constexpr int kBatch = 3;
    for (int i0 = 0; i0 < nload; i0 += kBatch * int(blockDim.x)) {
        int P[kBatch];
        T f[kBatch][9], mm[kBatch][3];
#pragma unroll
        for (int r = 0; r < kBatch; ++r) {
            const int i = i0 + r * int(blockDim.x) + int(threadIdx.x);
            P[r] = i < nload ? M.ft_node[noff + i] : -1;
        }
#pragma unroll
        for (int r = 0; r < kBatch; ++r)
            if (P[r] >= 0) load_rec(fin + size_t(P[r]) * kRec, f[r], mm[r][0], mm[r][1], mm[r][2]);
#pragma unroll
        for (int r = 0; r < kBatch; ++r) {
            const int i = i0 + r * int(blockDim.x) + int(threadIdx.x);
            if (P[r] < 0) continue;
            gid[i] = P[r];
            store_rec(buf + size_t(i) * kRec, f[r], mm[r][0], mm[r][1], mm[r][2]);
        }
    }
    // f* (eqs. (5)-(7)) of each interpolation node that a pivot of the tile reads
    // through it, once per sub-step, shared by all its readers
    if (has_star) {
        const T rho0 = T(M.rho0), cst = T(M.star_neq);
        for (int j = 0; j < ksteps; ++j) {
            T fs[9], nq[9];
            star_values<T, SHIFT>(sp0, sp1, T(th.v[j]), cst, rho0, fs, nq);
            T* d = stg + j * stj + size_t(threadIdx.x) * kStarRec;
#pragma unroll
            for (int q = 0; q < 9; ++q) d[q] = fs[q], d[9 + q] = nq[q];
        }
    }
    __syncthreads();
    const int B = int(blockDim.x), tx = int(threadIdx.x);
    if (ksteps == 2) {
        // Sub-step 1 takes node tx + B first and node tx last, so that the edge
        // records of node tx (the same local node in both sub-steps) stay in
        // registers for sub-step 2, which takes node tx first.
        const int n1 = meta[4];
        const T* const st1 = stg;
        const T* const st2 = stg + stj;
        EdgeRec<T> e[W], e0[W];
        T r1[9], m1[3], r0[9], m0v[3];
        const bool has1 = tx + B < n1, has0 = tx < n1;
        if (has1) {
#pragma unroll
            for (int z = 0; z < W; ++z) e[z] = E[size_t(z) * width + tx + B];
            const int P = fv_tile_node<T, SHIFT, W>(M, buf, gid, st1, tx + B, e, r1, m1,
                                                    tx + B < ntile ? M.wmom : nullptr);
            if (mid && tx + B < ntile) store_rec(mid + size_t(P) * kRec, r1, m1[0], m1[1], m1[2]);
        }
        __builtin_amdgcn_sched_barrier(0);
        if (has0) {
#pragma unroll
            for (int z = 0; z < W; ++z) e0[z] = E[size_t(z) * width + tx];
            const int P = fv_tile_node<T, SHIFT, W>(M, buf, gid, st1, tx, e0, r0, m0v, tx < ntile ? M.wmom : nullptr);
            if (mid && tx < ntile) store_rec(mid + size_t(P) * kRec, r0, m0v[0], m0v[1], m0v[2]);
        }
        __syncthreads();   // every read of sub-step 1 is done
        if (has1) store_rec(buf + size_t(tx + B) * kRec, r1, m1[0], m1[1], m1[2]);
        if (has0) store_rec(buf + size_t(tx) * kRec, r0, m0v[0], m0v[1], m0v[2]);
        __syncthreads();
        if (tx < ntile) {
            const int P = fv_tile_node<T, SHIFT, W>(M, buf, gid, st2, tx, e0, r0, m0v,
                                                    M.wmom ? M.wmom + M.wmom_stride : nullptr);
            store_rec(fout + size_t(P) * kRec, r0, m0v[0], m0v[1], m0v[2]);
        }
        __builtin_amdgcn_sched_barrier(0);
        if (tx + B < ntile) {
#pragma unroll
            for (int z = 0; z < W; ++z) e[z] = E[size_t(z) * width + tx + B];
            const int P = fv_tile_node<T, SHIFT, W>(M, buf, gid, st2, tx + B, e, r1, m1,
                                                    M.wmom ? M.wmom + M.wmom_stride : nullptr);
            store_rec(fout + size_t(P) * kRec, r1, m1[0], m1[1], m1[2]);
        }
        return;
    }
    for (int j = 1; j <= ksteps; ++j) {
        const int ncomp = meta[3 + ksteps - j];
        const T* const stj_ = stg + (j - 1) * stj;
        const bool last = j == ksteps;
        T res[kFvStage][9], rm[kFvStage][3];
#pragma unroll
        for (int s2 = 0; s2 < kFvStage; ++s2) {
            const int i = tx + s2 * B;
            if (i >= ncomp) break;
            EdgeRec<T> e[W];
#pragma unroll
            for (int z = 0; z < W; ++z) e[z] = E[size_t(z) * width + i];
            const int P = fv_tile_node<T, SHIFT, W>(M, buf, gid, stj_, i, e, res[s2], rm[s2],
                                                    M.wmom && i < ntile ? M.wmom + (j - 1) * M.wmom_stride : nullptr);
            if (last) store_rec(fout + size_t(P) * kRec, res[s2], rm[s2][0], rm[s2][1], rm[s2][2]);
            else if (mid && i < ntile)
                store_rec(mid + size_t(j - 1) * mid_stride + size_t(P) * kRec, res[s2], rm[s2][0], rm[s2][1], rm[s2][2]);
            __builtin_amdgcn_sched_barrier(0);   // one node at a time: registers for occupancy
        }
        if (!last) {
            __syncthreads();   // every read of this sub-step is done
#pragma unroll
            for (int s2 = 0; s2 < kFvStage; ++s2) {
                const int i = tx + s2 * B;
                if (i < ncomp) store_rec(buf + size_t(i) * kRec, res[s2], rm[s2][0], rm[s2][1], rm[s2][2]);
            }
            __syncthreads();
        }
    }
}

// Threads of the single wall-force block: with 1024, each thread takes about
// two of the 2048 wall edges of the 264k-node mesh, so its chain of dependent
// loads (edge, then the two records) is short.
constexpr int kWallForceThreads = 1024;

// Drag and lift, eqs. (10)-(11), in FP64: momentum flux out of the fluid
// through the wall edges, sum_i c_i (c_i . N_e) (f_i(a) + f_i(b)) / 2, reduced
// by one block in a fixed order (deterministic).  Shifted storage drops the
// rest-state part rho0 c_s^2 N_e, which sums to zero over the closed wall.
template <typename T, bool SHIFT>
__global__ __launch_bounds__(kWallForceThreads) void k_wall_force(const T* __restrict__ f, int ne,
                                                                  const int32_t* __restrict__ wedge,
                                                                  const double* __restrict__ wn,
                                                                  double* __restrict__ out, double ca, double sa,
                                                                  double qn) {
    __shared__ double sx[kWallForceThreads], sy[kWallForceThreads];
    double ax = 0, ay = 0;
    for (int e = threadIdx.x; e < ne; e += kWallForceThreads) {
        const int a = wedge[2 * e], b = wedge[2 * e + 1];
        const double nx = wn[2 * e], ny = wn[2 * e + 1];
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            const double m = 0.5 * (double(f[size_t(a) * kRec + q]) + double(f[size_t(b) * kRec + q]));
            const double cn = CX[q] * nx + CY[q] * ny;
            ax += CX[q] * cn * m;
            ay += CY[q] * cn * m;
        }
    }
    sx[threadIdx.x] = ax;
    sy[threadIdx.x] = ay;
    __syncthreads();
    for (int h = kWallForceThreads / 2; h > 0; h >>= 1) {
        if (int(threadIdx.x) < h) {
            sx[threadIdx.x] += sx[threadIdx.x + h];
            sy[threadIdx.x] += sy[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = (sx[0] * ca + sy[0] * sa) / qn;
        out[1] = (-sx[0] * sa + sy[0] * ca) / qn;
    }
}

// ---- Body resolved by bounce-back (the standard LBM of eq. (14)) ----
// The collide-stream kernels pull every direction from x - c_q; at the nodes
// next to a solid body (a short list on the finest level) the directions whose
// source is solid are redone here: f_q(x, t+1) = f~_{-q}(x, t), the node's own
// post-collision population of the opposite direction (halfway bounce-back).

constexpr int kOpposite[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

// Streamed populations of bounce-back node b (interior of the level: the plan
// keeps the body 6 nodes from its edges, so no far-field or periodic source).
template <typename T>
__device__ __forceinline__ void bounce_pull(const KLevel& L, const T* __restrict__ A, int b, int& i, int& j,
                                            T (&f)[9]) {
    const int id = L.bounce_node[b], mask = L.bounce_mask[b];
    i = id % L.nx;
    j = id / L.nx;
    const size_t base = size_t(j) * size_t(L.rs) + i;
#pragma unroll
    for (int q = 0; q < 9; ++q)
        f[q] = (mask >> q) & 1 ? A[size_t(kOpposite[q]) * L.pitch + base]
                               : A[size_t(q) * L.pitch + base - ptrdiff_t(CY[q]) * L.rs - CX[q]];
}

// Collide-stream of the bounce-back nodes, after the level's kernel: B = collide(stream(A)).
template <typename T, bool SHIFT>
__global__ __launch_bounds__(256) void k_bounce(const KLevel L, const T* __restrict__ A, T* __restrict__ B) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= L.n_bounce) return;
    int i, j;
    T f[9], feq[9], rho, dr, ux, uy, o[9];
    bounce_pull(L, A, b, i, j, f);
    const T omega = T(L.omega), rho0 = T(L.rho0);
    macro<T, SHIFT>(f, rho0, rho, dr, ux, uy);
    equilibrium<T, SHIFT>(rho, dr, ux, uy, feq);
#pragma unroll
    for (int q = 0; q < 9; ++q) o[q] = f[q] - (f[q] - feq[q]) * omega;
    if constexpr (SHIFT && sizeof(T) == 4) conserve_f32(f, o);
    const size_t base = size_t(j) * size_t(L.rs) + i;
#pragma unroll
    for (int q = 0; q < 9; ++q) B[size_t(q) * L.pitch + base] = o[q];
}

// Canonical export of the bounce-back nodes in rows [j0, j1) (after k_export_level).
template <typename T, bool SHIFT>
__global__ void k_bounce_export(const KLevel L, const T* __restrict__ A, double* __restrict__ out, int j0, int j1) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= L.n_bounce) return;
    const int jb = L.bounce_node[b] / L.nx;
    if (jb < j0 || jb >= j1) return;
    int i, j;
    T f[9];
    bounce_pull(L, A, b, i, j, f);
    const size_t rows = size_t(j1 - j0), o = size_t(j - j0) * L.nx + i;
    for (int q = 0; q < 9; ++q) out[q * rows * L.nx + o] = to_phys<T, SHIFT>(f[q], q, L.rho0);
}

// Canonical import of the bounce-back nodes in rows [j0, j1) (after
// k_import_level): a bounced f_q(x) goes to the opposite direction at x itself,
// which no other node pulls (its source would be the solid node x - c_q).
template <typename T, bool SHIFT>
__global__ void k_bounce_import(const KLevel L, T* __restrict__ A, const double* __restrict__ in, int j0, int j1) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= L.n_bounce) return;
    const int id = L.bounce_node[b], mask = L.bounce_mask[b];
    const int i = id % L.nx, j = id / L.nx;
    if (j < j0 || j >= j1) return;
    const size_t rows = size_t(j1 - j0), o = size_t(j - j0) * L.nx + i;
    for (int q = 1; q < 9; ++q)
        if ((mask >> q) & 1)   // w_q = w_{-q}: the stored form is the same
            A[lidx(L, kOpposite[q], i, j)] = to_store<T, SHIFT>(in[q * rows * L.nx + o], q, L.rho0);
}

// The uniform start f^eq(rho, u) as the bounce-back nodes pull it (after k_fill_uniform).
template <typename T, bool SHIFT>
__global__ void k_bounce_uniform(const KLevel L, T* __restrict__ A, double rho, double ux, double uy) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= L.n_bounce) return;
    const int id = L.bounce_node[b], mask = L.bounce_mask[b];
    const int i = id % L.nx, j = id / L.nx;
    for (int q = 1; q < 9; ++q) {
        if (!((mask >> q) & 1)) continue;
        const double cu = CX[q] * ux + CY[q] * uy, uu = ux * ux + uy * uy;
        const double fe = wgt<double>(q) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
        A[lidx(L, kOpposite[q], i, j)] = to_store<T, SHIFT>(fe, q, L.rho0);
    }
}

// Force on the body by momentum exchange, in FP64, one block in a fixed order:
// each f~_p that left a bounce-back node towards the body (x + c_p solid)
// returns reversed and gives it 2 c_p f~_p.  Shifted storage drops the rest
// part 2 c_p w_p rho0, whose sum over the links of a closed body is zero (as
// many links leave the body in each direction as enter it).
template <typename T, bool SHIFT>
__global__ __launch_bounds__(kWallForceThreads) void k_body_force(const KLevel L, const T* __restrict__ A,
                                                                  double* __restrict__ out, double ca, double sa,
                                                                  double qn) {
    __shared__ double sx[kWallForceThreads], sy[kWallForceThreads];
    double ax = 0, ay = 0;
    for (int b = threadIdx.x; b < L.n_bounce; b += kWallForceThreads) {
        const int id = L.bounce_node[b], mask = L.bounce_mask[b];
        const size_t base = size_t(id / L.nx) * size_t(L.rs) + id % L.nx;
        for (int q = 1; q < 9; ++q) {
            if (!((mask >> q) & 1)) continue;
            const int p = kOpposite[q];
            const double v = double(A[size_t(p) * L.pitch + base]);
            ax += 2.0 * CX[p] * v;
            ay += 2.0 * CY[p] * v;
        }
    }
    sx[threadIdx.x] = ax;
    sy[threadIdx.x] = ay;
    __syncthreads();
    for (int h = kWallForceThreads / 2; h > 0; h >>= 1) {
        if (int(threadIdx.x) < h) {
            sx[threadIdx.x] += sx[threadIdx.x + h];
            sy[threadIdx.x] += sy[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = (sx[0] * ca + sy[0] * sa) / qn;
        out[1] = (-sx[0] * sa + sy[0] * ca) / qn;
    }
}

// [9][nn] FP64 populations -> mesh records (stored form plus moments)
template <typename T, bool SHIFT>
__global__ void k_mesh_convert(int nn, const double* __restrict__ in, T* __restrict__ out, double rho0) {
    const int P = blockIdx.x * blockDim.x + threadIdx.x;
    if (P >= nn) return;
    T f[9], r, dr, ux, uy;
#pragma unroll
    for (int q = 0; q < 9; ++q) f[q] = to_store<T, SHIFT>(in[size_t(q) * nn + P], q, rho0);
    macro<T, SHIFT>(f, T(rho0), r, dr, ux, uy);
    store_rec(out + size_t(P) * kRec, f, SHIFT ? dr : r, ux, uy);
}
// mesh records -> [9][nn] FP64 populations
template <typename T, bool SHIFT>
__global__ void k_mesh_export(int nn, const T* __restrict__ in, double* __restrict__ out, double rho0) {
    const int P = blockIdx.x * blockDim.x + threadIdx.x;
    if (P >= nn) return;
#pragma unroll
    for (int q = 0; q < 9; ++q) out[size_t(q) * nn + P] = to_phys<T, SHIFT>(in[size_t(P) * kRec + q], q, rho0);
}

unsigned blocks(size_t n, unsigned b = 256) { return unsigned((n + b - 1) / b); }

// Workgroup size of the one-sub-step FV kernel: 256 threads, or 64 when that
// leaves fewer than two workgroups per CU (small meshes are latency-bound, and
// more, smaller workgroups spread them over the chip).
unsigned fv_substep_block(int nn) { return nn < 2 * 256 * 256 ? 64u : 256u; }

// Workgroup size of the interface kernels (far-field edges, box transfers): a
// few thousand nodes, each a short chain of dependent loads; one-wave groups
// spread them over more CUs (measured on the 2048 x 1024 box: coarse -> fine
// 11.1 -> 9.4 us, fine -> coarse 10.3 -> 6.9 us against 256-thread groups).
constexpr unsigned kSmallBlock = 64;

}  // namespace

#define HLBM_DISPATCH(prec, CALL)        \
    do {                                 \
        if ((prec) == HLBM_FP64) {       \
            using T = double;            \
            constexpr bool S = false;    \
            CALL;                        \
        } else {                         \
            using T = float;             \
            constexpr bool S = true;     \
            CALL;                        \
        }                                \
    } while (0)

void launch_fill_uniform(int prec, void* buf, const KLevel& L, double rho, double ux, double uy, hipStream_t s) {
    HLBM_DISPATCH(prec, (k_fill_uniform<T, S><<<blocks(size_t(L.ny) * size_t(L.rs)), 256, 0, s>>>(L, (T*)buf, rho, ux, uy)));
    if (L.n_bounce > 0)
        HLBM_DISPATCH(prec, (k_bounce_uniform<T, S><<<blocks(L.n_bounce), 256, 0, s>>>(L, (T*)buf, rho, ux, uy)));
}

void launch_stream_collide(int prec, const KLevel& L, const void* A, void* B, hipStream_t s) {
    if (prec == HLBM_FP32_SHIFTED && !L.periodic) {
        if (size_t(L.nx) * size_t(L.ny) >= kWideLevelNodes) {
            dim3 grid(blocks(size_t(L.pitch / 4)), L.ny);
            k_stream_collide_vec<float, true, 4><<<grid, 256, 0, s>>>(L, (const float*)A, (float*)B);
        } else {
            dim3 grid(blocks(size_t(L.pitch / 2)), L.ny);
            k_stream_collide_vec<float, true, 2><<<grid, 256, 0, s>>>(L, (const float*)A, (float*)B);
        }
    } else {
        dim3 grid(blocks(L.nx), L.ny);
        HLBM_DISPATCH(prec, (k_stream_collide<T, S><<<grid, 256, 0, s>>>(L, (const T*)A, (T*)B)));
    }
    if (L.farfield)
        HLBM_DISPATCH(prec, (k_edges<T, S><<<blocks(2 * size_t(L.nx) + 2 * size_t(L.ny - 2), kSmallBlock), kSmallBlock, 0, s>>>(L, (const T*)A, (T*)B)));
    if (L.n_bounce > 0)
        HLBM_DISPATCH(prec, (k_bounce<T, S><<<blocks(L.n_bounce), 256, 0, s>>>(L, (const T*)A, (T*)B)));
}

void launch_body_force(int prec, const KLevel& L, const void* A, double* out, double ca, double sa, double qn,
                       hipStream_t s) {
    HLBM_DISPATCH(prec, (k_body_force<T, S><<<1, kWallForceThreads, 0, s>>>(L, (const T*)A, out, ca, sa, qn)));
}

void launch_export_level(int prec, const KLevel& L, const void* A, double* out, int j0, int j1, hipStream_t s) {
    dim3 grid(blocks(L.nx), j1 - j0);
    HLBM_DISPATCH(prec, (k_export_level<T, S><<<grid, 256, 0, s>>>(L, (const T*)A, out, j0, j1)));
    if (L.n_bounce > 0)
        HLBM_DISPATCH(prec, (k_bounce_export<T, S><<<blocks(L.n_bounce), 256, 0, s>>>(L, (const T*)A, out, j0, j1)));
}

void launch_import_level(int prec, const KLevel& L, void* A, const double* in, int j0, int j1, hipStream_t s) {
    dim3 grid(blocks(L.nx), j1 - j0);
    HLBM_DISPATCH(prec, (k_import_level<T, S><<<grid, 256, 0, s>>>(L, (T*)A, in, j0, j1)));
    if (L.n_bounce > 0)
        HLBM_DISPATCH(prec, (k_bounce_import<T, S><<<blocks(L.n_bounce), 256, 0, s>>>(L, (T*)A, in, j0, j1)));
}

void launch_side_init(int prec, const KLevel& P, int ci0, int cj0, int nxc, int nyc, const void* A, void* side, hipStream_t s) {
    HLBM_DISPATCH(prec, (k_side_init<T, S><<<blocks(2 * size_t(nxc + nyc)), 256, 0, s>>>(P, ci0, cj0, nxc, nyc, (const T*)A, (T*)side)));
}

void launch_coarse_to_fine(int prec, const KLevel& P, const KLevel& C, int ci0, int cj0, const void* pA, void* cA,
                           void* side_cur, const void* side_prev, double theta, int compute_side, double tau_c,
                           double tau_f, hipStream_t s) {
    const size_t n = 2 * size_t(C.nx - 1 + C.ny - 1);
    const double scale = tau_f / (2.0 * tau_c);
    HLBM_DISPATCH(prec, (k_coarse_to_fine<T, S><<<blocks(n, kSmallBlock), kSmallBlock, 0, s>>>(P, C, ci0, cj0, (const T*)pA, (T*)cA, (T*)side_cur,
                                                                          (const T*)side_prev, T(theta), compute_side,
                                                                          T(scale), T(1.0 / tau_f))));
}

void launch_fine_to_coarse(int prec, const KLevel& P, const KLevel& C, int ci0, int cj0, int nxc, int nyc,
                           const void* cprev, void* pdst, double tau_c, double tau_f, int filter, hipStream_t s) {
    const size_t n = 2 * size_t(nxc - 2 + nyc - 2);
    const double scale = 2.0 * tau_c / tau_f;
    HLBM_DISPATCH(prec, (k_fine_to_coarse<T, S><<<blocks(n, kSmallBlock), kSmallBlock, 0, s>>>(P, C, ci0, cj0, nxc, nyc, (const T*)cprev,
                                                                          (T*)pdst, T(scale), T(1.0 / tau_c), filter)));
}

void launch_mesh_to_struct(int prec, const KLevel& F, void* A, int n, const int32_t* node, const int32_t* don,
                           const void* w, const void* mf, int nn, double factor, hipStream_t s) {
    if (n <= 0) return;
    (void)nn;
    HLBM_DISPATCH(prec, (k_mesh_to_struct<T, S><<<blocks(n, 64), 64, 0, s>>>(F, (T*)A, n, node, don, (const T*)w,
                                                                             (const T*)mf, T(factor))));
}

void launch_struct_to_mesh(int prec, const KLevel& F, const void* A, int n, const int32_t* don, const void* w,
                           void* prep, hipStream_t s) {
    if (n <= 0) return;
    HLBM_DISPATCH(prec, (k_struct_to_mesh<T, S><<<blocks(n, 64), 64, 0, s>>>(F, (const T*)A, n, don, (const T*)w, (T*)prep)));
}

void launch_fv_substep(int prec, const KMesh& M, const void* fin, void* fout, const void* prep0, const void* prep1,
                       double theta, hipStream_t s) {
    const unsigned b = fv_substep_block(M.nn);
    if (M.ell_width <= 8) {
        HLBM_DISPATCH(prec, (k_fv_substep<T, S, 8><<<blocks(M.nn, b), b, 0, s>>>(M, (const T*)fin, (T*)fout, (const T*)prep0,
                                                                                (const T*)prep1, T(theta))));
    } else {
        HLBM_DISPATCH(prec, (k_fv_substep<T, S, 16><<<blocks(M.nn, b), b, 0, s>>>(M, (const T*)fin, (T*)fout, (const T*)prep0,
                                                                                 (const T*)prep1, T(theta))));
    }
}

void launch_fv_fused(int prec, const KMesh& M, const void* fin, void* fout, const void* prep0, const void* prep1,
                     int m0, int k, hipStream_t s, void* mid, size_t mid_stride_bytes) {
    if (M.n_tiles <= 0 || k < 1 || k > M.fuse) return;
    const size_t elem = prec == HLBM_FP64 ? 8 : 4;
    const size_t lds = fv_lds_bytes(M.maxl, M.maxs, k, elem);
    const unsigned threads = unsigned(M.threads);
    if (size_t(M.maxw) > size_t(kFvStage) * threads || threads > (prec == HLBM_FP64 ? 256u : 512u)) return;   // rejected by the plan
    FvTheta th;   // theta = m / n of sub-steps m0 .. m0 + k - 1, as the one-sub-step launches take it
    for (int j = 0; j < kMaxFuse; ++j) th.v[j] = double(m0 + j) / double(M.n_sub);
    if (M.ft_width == 7) {
        HLBM_DISPATCH(prec, (k_fv_fused<T, S, 7><<<M.n_tiles, threads, lds, s>>>(M, (const T*)fin, (T*)fout, (const T*)prep0,
                                                                                  (const T*)prep1, th, k, (T*)mid,
                                                                 mid_stride_bytes / sizeof(T))));
    } else if (M.ft_width == 8) {
        HLBM_DISPATCH(prec, (k_fv_fused<T, S, 8><<<M.n_tiles, threads, lds, s>>>(M, (const T*)fin, (T*)fout, (const T*)prep0,
                                                                                  (const T*)prep1, th, k, (T*)mid,
                                                                 mid_stride_bytes / sizeof(T))));
    } else {
        HLBM_DISPATCH(prec, (k_fv_fused<T, S, 16><<<M.n_tiles, threads, lds, s>>>(M, (const T*)fin, (T*)fout, (const T*)prep0,
                                                                                   (const T*)prep1, th, k, (T*)mid,
                                                                 mid_stride_bytes / sizeof(T))));
    }
}

void launch_wall_force(int prec, const void* f, int ne, const int32_t* wedge, const double* wn,
                       double* out, double ca, double sa, double qn, hipStream_t s) {
    HLBM_DISPATCH(prec, (k_wall_force<T, S><<<1, kWallForceThreads, 0, s>>>((const T*)f, ne, wedge, wn, out, ca, sa, qn)));
}

void launch_mesh_convert(int prec, int nn, const double* in, void* out, int to_storage, double rho0, hipStream_t s) {
    if (to_storage) {
        HLBM_DISPATCH(prec, (k_mesh_convert<T, S><<<blocks(nn), 256, 0, s>>>(nn, in, (T*)out, rho0)));
    } else {
        HLBM_DISPATCH(prec, (k_mesh_export<T, S><<<blocks(nn), 256, 0, s>>>(nn, (const T*)out, (double*)in, rho0)));
    }
}

}  // namespace hlbm

// ===========================================================================
// ---- Discrete adjoint kernels (reverse mode, FP64) ----
//
// Reverse mode of the forward kernels above, kernel by kernel: every forward
// scatter becomes a gather over a transposed table, so the adjoint is
// deterministic and uses no atomics.  Parameter derivatives (angle of attack,
// tau) are summed per block in a fixed tree order into `partial` slots and
// reduced by one block at the end of each step.
// ===========================================================================
namespace hlbm {
namespace {

using D9 = double[9];

// sum_q eb_q d feq_q(rho, u) / d(rho, u) for feq_q = w_q rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u^2)
__device__ __forceinline__ void feq_adj(double rho, double ux, double uy, const D9& eb, double& rb, double& uxb,
                                        double& uyb) {
    const double uu = ux * ux + uy * uy;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const double cu = CX[q] * ux + CY[q] * uy, w = wgt<double>(q);
        rb += eb[q] * w * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
        uxb += eb[q] * w * rho * (3.0 * CX[q] + 9.0 * cu * CX[q] - 3.0 * ux);
        uyb += eb[q] * w * rho * (3.0 * CY[q] + 9.0 * cu * CY[q] - 3.0 * uy);
    }
}

// fb += adjoint of (rho, u) = (sum f, sum c f / sum f) for adjoints (rb, uxb, uyb)
__device__ __forceinline__ void macro_adj(double rho, double ux, double uy, double rb, double uxb, double uyb, D9& fb) {
    const double jxb = uxb / rho, jyb = uyb / rho, r2 = rb - (uxb * ux + uyb * uy) / rho;
#pragma unroll
    for (int q = 0; q < 9; ++q) fb[q] += r2 + jxb * CX[q] + jyb * CY[q];
}

__device__ __forceinline__ void macro64(const D9& f, double& rho, double& ux, double& uy) {
    double s = 0, mx = 0, my = 0;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        s += f[q];
        mx += double(CX[q]) * f[q];
        my += double(CY[q]) * f[q];
    }
    rho = s;
    ux = mx / rho;
    uy = my / rho;
}

// fb += adjoint of the map f -> (rho, ux, uy, f - feq(rho, u)) for adjoint a[12]
__device__ __forceinline__ void macro_neq_adj(const D9& f, const double* a, D9& fb) {
    double rho, ux, uy;
    macro64(f, rho, ux, uy);
    double rb = a[0], uxb = a[1], uyb = a[2];
    D9 eb;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        fb[q] += a[3 + q];
        eb[q] = -a[3 + q];
    }
    feq_adj(rho, ux, uy, eb, rb, uxb, uyb);
    macro_adj(rho, ux, uy, rb, uxb, uyb, fb);
}

// fixed-order block sum of (a, b) written to partial[2 * (slot + blockIdx.x)],
// for blocks of B threads
template <int B = 256>
__device__ __forceinline__ void block_partial(double a, double b, double* partial, int slot) {
    __shared__ double sa[B], sb[B];
    sa[threadIdx.x] = a;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int h = B / 2; h > 0; h >>= 1) {
        if (int(threadIdx.x) < h) {
            sa[threadIdx.x] += sa[threadIdx.x + h];
            sb[threadIdx.x] += sb[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * (slot + blockIdx.x)] = sa[0];
        partial[2 * (slot + blockIdx.x) + 1] = sb[0];
    }
}

__global__ void k_zero(double* p, size_t n) {
    const size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e < n) p[e] = 0.0;
}

// Wall force, eqs. (10)-(11): d J / d f_q(P) = (c_q . j)(c_q . V_P), V_P = half the
// wall normals of the two wall edges at P, j = drag/lift weights / normaliser.
// With vbar set, also accumulates d J / d V_P = sum_q (c_q . j) c_q f_q(P) from the
// mesh state fst the force was taken on.
__global__ void k_adj_force(int n_wall, double* __restrict__ mbar, const double* __restrict__ V, double jx,
                            double jy, const double* __restrict__ fst, double* __restrict__ vbar) {
    const int P = blockIdx.x * blockDim.x + threadIdx.x;
    if (P >= n_wall) return;
#pragma unroll
    for (int q = 0; q < 9; ++q)
        mbar[size_t(P) * kAdjRec + q] += (CX[q] * jx + CY[q] * jy) * (CX[q] * V[2 * P] + CY[q] * V[2 * P + 1]);
    if (vbar) {
        double f[9], m0, ux, uy, ax = 0.0, ay = 0.0;
        load_rec(fst + size_t(P) * kRec, f, m0, ux, uy);
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            const double a = (CX[q] * jx + CY[q] * jy) * f[q];
            ax += CX[q] * a;
            ay += CY[q] * a;
        }
        vbar[2 * P] += ax;
        vbar[2 * P + 1] += ay;
    }
}

// star values of one interpolation slot at theta (FP64), with their inputs
__device__ __forceinline__ void star64(const double* p0, const double* p1, double theta, double cst, double (&v)[12],
                                       D9& fs, D9& ns) {
#pragma unroll
    for (int m = 0; m < 12; ++m) v[m] = (1.0 - theta) * p0[m] + theta * p1[m];
    double feq[9];
    equilibrium<double, false>(v[0], v[0], v[1], v[2], feq);
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        ns[q] = cst * v[3 + q];
        fs[q] = feq[q] + ns[q];
    }
}

// value f and non-equilibrium part nq of neighbour k as pivot P's update reads
// them: the star values of eqs. (5)-(7) between interpolation nodes, else the
// stored mesh value
__device__ __forceinline__ void fv_value(const KAdj& K, const double* fin, const double* prep0, const double* prep1,
                                         double theta, bool pivot_interp, int k, D9& f, D9& nq) {
    if (pivot_interp && k >= K.M.n_core) {
        double v[12];
        const size_t sl = size_t(k - K.M.n_core) * kMacro;
        star64(prep0 + sl, prep1 + sl, theta, K.cst, v, f, nq);
    } else {
        double m0, ux, uy, feq[9];
        load_rec(fin + size_t(k) * kRec, f, m0, ux, uy);
        equilibrium<double, false>(m0, m0, ux, uy, feq);
#pragma unroll
        for (int q = 0; q < 9; ++q) nq[q] = f[q] - feq[q];
    }
}

// Mesh adjoints are node records of kAdjRec doubles (9 used, 16-byte aligned),
// so a gather of a neighbour's nine values is five 16-byte loads.
__device__ __forceinline__ void load_adj(const double* __restrict__ p, D9& v) {
    const double2* r = reinterpret_cast<const double2*>(p);
    const double2 a = r[0], b = r[1], c = r[2], d = r[3], e = r[4];
    v[0] = a.x, v[1] = a.y, v[2] = b.x, v[3] = b.y, v[4] = c.x, v[5] = c.y, v[6] = d.x, v[7] = d.y, v[8] = e.x;
}
__device__ __forceinline__ void store_adj(double* __restrict__ p, const D9& v) {
    double2* r = reinterpret_cast<double2*>(p);
    r[0] = double2{v[0], v[1]};
    r[1] = double2{v[2], v[3]};
    r[2] = double2{v[4], v[5]};
    r[3] = double2{v[6], v[7]};
    r[4] = double2{v[8], 0.0};
}

// Adjoint of the no-slip reset at a wall node, out = f^eq(rho, 0) + fn - f^eq(rho, u):
// maps the adjoint yb of the reset output onto the pre-reset update fn,
// zb = R'(fn)^T yb, which depends on fn only through its (rho, u), recorded by
// the forward sub-step in w = (rho, u_x, u_y).
__device__ __forceinline__ void wall_reset_apply(const double* __restrict__ w, const D9& yb, D9& zb) {
    const double rho = w[0], ux = w[1], uy = w[2];
    double rb = 0.0, uxb = 0.0, uyb = 0.0, eb[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        zb[q] = yb[q];
        rb += yb[q] * wgt<double>(q);
        eb[q] = -yb[q];
    }
    feq_adj(rho, ux, uy, eb, rb, uxb, uyb);
    macro_adj(rho, ux, uy, rb, uxb, uyb, zb);
}

// No-slip reset adjoint of the last sub-step of a finest step (per wall pivot P):
// zwall_P (layout [9][n_wall]) from ybar_P.  Earlier sub-steps get theirs from
// k_adj_fv of the sub-step after them.
__global__ __launch_bounds__(256) void k_adj_fv_wall(const KAdj K, const double* __restrict__ wmom,
                                                     const double* __restrict__ ybar, double* __restrict__ zwall) {
    const KMesh& M = K.M;
    const int P = blockIdx.x * blockDim.x + threadIdx.x;
    if (P >= M.n_wall) return;
    double yb[9], zb[9];
    load_adj(ybar + size_t(P) * kAdjRec, yb);
    wall_reset_apply(wmom + 3 * size_t(P), yb, zb);
    store_adj(zwall + size_t(P) * kAdjRec, zb);
}

// FV sub-step adjoint (per node k): the adjoint of every value of k that the
// update of eqs. (3), (5) reads, gathered over the pivots P whose rows hold k
// (transposed table; slot 0 is k itself with its base and collision terms).
//   stored value M^m_k (read by pivots that are not both interpolation nodes)
//     -> mbar_k, through (rho, u, f^neq) of the record;
//   star value f*_k of an interpolation node (read by interpolation pivots)
//     -> the adjoints of the structured (rho, u, f^neq) at t and t + 1.
// The adjoint of each pivot's update is ybar_P, or zwall_P after the no-slip
// reset transpose at wall pivots.  tau enters through Delta t_u / tau_u and
// 1 - 1/(2 tau); with K.gbar set, the coefficient adjoints of the entries
// (P, k) are accumulated too, in the transposed slot of k (one writer per
// slot, so no conflicts; consecutive k are consecutive in memory): the
// neighbour part of G_Pk here, the pivot's base part once per pivot in gpivot.
// With wmom_prev set (the pre-reset (rho, u) of the wall nodes in the previous
// sub-step, recorded by the forward), wall nodes also take the no-slip reset
// transpose of that sub-step from the adjoint just computed, into zwall_prev,
// so the next launch needs no separate wall pass.
// Adjoint of the values of node k read through one class of pivots: the stored
// mesh value (STAR = false: every pivot unless both are interpolation nodes)
// or the star value of an interpolation node (STAR = true: interpolation
// pivots).  Accumulates into vb (adjoint of the value), nb (of its f^neq part)
// and, with K.gbar, the coefficient adjoints of the entries read.
template <int W, bool STAR, int G>
__device__ __forceinline__ void adj_fv_gather(const KAdj& K, int k, bool k_interp, const double* __restrict__ ybar,
                                              const double* __restrict__ zwall, const D9& val, const D9& nval, D9& vb,
                                              D9& nb, int z_begin = 0) {
    const KMesh& M = K.M;
    const int nn = M.nn;
    const int nwall = M.wall_bc ? M.n_wall : 0;
    const EdgeRec<double>* T = reinterpret_cast<const EdgeRec<double>*>(K.tedges);
    // slots in groups of G: the G table entries, then the G pivot adjoints are
    // loaded before the arithmetic
#pragma unroll 1
    for (int g0 = z_begin; g0 < z_begin + W; g0 += G) {
        EdgeRec<double> eg[G];
        double zg[G][9];
        // coefficient adjoints of the group's slots, read before the pivot gathers
        // (each entry has one writer per launch: the lane of its slot)
        double gold[G][3];
        if (K.gbar) {
#pragma unroll
            for (int a = 0; a < G; ++a) {
                const int z = g0 + a;
                if (z == 0) {
                    gold[a][0] = K.gpivot[2 * size_t(k)];
                    gold[a][1] = K.gpivot[2 * size_t(k) + 1];
                    gold[a][2] = K.gbar[size_t(k) * 3 + 2];
                } else {
                    const double* g = K.gbar + (size_t(z) * nn + k) * 3;
                    gold[a][0] = g[0], gold[a][1] = g[1], gold[a][2] = g[2];
                }
            }
        }
#pragma unroll
        for (int a = 0; a < G; ++a) eg[a] = T[size_t(g0 + a) * nn + k];
#pragma unroll
        for (int a = 0; a < G; ++a) {
            const int P = eg[a].col < 0 ? k : eg[a].col;
            load_adj((P < nwall ? zwall : ybar) + size_t(P) * kAdjRec, zg[a]);
        }
#pragma unroll
        for (int a = 0; a < G; ++a) {
            const EdgeRec<double>& e = eg[a];
            const int z = g0 + a;
            const int P = e.col;
            if (P < 0) continue;
            if ((k_interp && P >= M.n_core) != STAR) continue;
            const double(&zp)[9] = zg[a];
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const double sq = CX[q] * e.gx + CY[q] * e.gy;
                vb[q] += z == 0 ? zp[q] * (1.0 - K.dt * sq) : K.dt * sq * zp[q];
                nb[q] -= K.dtt * e.c * zp[q];
            }
            if (K.gbar) {
                double gx = 0.0, gy = 0.0, gc = 0.0;
#pragma unroll
                for (int q = 0; q < 9; ++q) {
                    gx += zp[q] * CX[q] * val[q];
                    gy += zp[q] * CY[q] * val[q];
                    gc += zp[q] * nval[q];
                }
                if (z == 0) {
                    K.gbar[size_t(k) * 3 + 2] = gold[a][2] - K.dtt * gc;
                    K.gpivot[2 * size_t(k)] = gold[a][0] + K.dt * gx;
                    K.gpivot[2 * size_t(k) + 1] = gold[a][1] + K.dt * gy;
                } else {   // transposed slot z of k (coalesced); mapped to the forward slot on download
                    double* g = K.gbar + (size_t(z) * nn + k) * 3;
                    g[0] = gold[a][0] + K.dt * gx;
                    g[1] = gold[a][1] + K.dt * gy;
                    g[2] = gold[a][2] - K.dtt * gc;
                }
            }
        }
    }
}

template <int W, int B, int G>
__global__ __launch_bounds__(B) void k_adj_fv(const KAdj K, const double* __restrict__ fin,
                                                const double* __restrict__ ybar, const double* __restrict__ zwall,
                                                double* __restrict__ mbar, const double* __restrict__ prep0,
                                                const double* __restrict__ prep1, double theta,
                                                double* __restrict__ p0bar, double* __restrict__ p1bar, int pslot,
                                                const double* __restrict__ wmom_prev, double* __restrict__ zwall_prev) {
    const KMesh& M = K.M;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    double dtau = 0.0;
    if (k < M.nn) {
        const bool k_interp = k >= M.n_core;
        const double rdt = K.ddtt_dtau / K.dtt;
        {   // the stored value M^m_k
            double f[9], m0, ux, uy, feq[9], nq[9], vb[9], nqb[9];
            load_rec(fin + size_t(k) * kRec, f, m0, ux, uy);
            equilibrium<double, false>(m0, m0, ux, uy, feq);
#pragma unroll
            for (int q = 0; q < 9; ++q) nq[q] = f[q] - feq[q], vb[q] = nqb[q] = 0.0;
            adj_fv_gather<W, false, G>(K, k, k_interp, ybar, zwall, f, nq, vb, nqb);
            double a12[12] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                dtau += rdt * nq[q] * nqb[q];
                a12[3 + q] = nqb[q];
            }
            macro_neq_adj(f, a12, vb);
            store_adj(mbar + size_t(k) * kAdjRec, vb);
            if (wmom_prev && k < (M.wall_bc ? M.n_wall : 0)) {
                double zb[9];
                wall_reset_apply(wmom_prev + 3 * size_t(k), vb, zb);
                store_adj(zwall_prev + size_t(k) * kAdjRec, zb);
            }
        }
        if (k_interp) {   // the star value f*_k read by interpolation pivots
            const size_t sl = size_t(k - M.n_core) * kMacro;
            double v[12], fs[9], ns[9], fsb[9], nsb[9];
            star64(prep0 + sl, prep1 + sl, theta, K.cst, v, fs, ns);
#pragma unroll
            for (int q = 0; q < 9; ++q) fsb[q] = nsb[q] = 0.0;
            adj_fv_gather<W, true, G>(K, k, true, ybar, zwall, fs, ns, fsb, nsb);
            // fs = feq(v0, v1, v2) + cst v[3..], ns = cst v[3..]
            double rb = 0.0, uxb = 0.0, uyb = 0.0, w12[12], dcst = 0.0;
            feq_adj(v[0], v[1], v[2], fsb, rb, uxb, uyb);
            w12[0] = rb, w12[1] = uxb, w12[2] = uyb;
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                w12[3 + q] = K.cst * (fsb[q] + nsb[q]);
                dcst += (fsb[q] + nsb[q]) * v[3 + q];
                dtau += rdt * ns[q] * nsb[q];
            }
            dtau += dcst * K.dcst_dtau;
#pragma unroll
            for (int m = 0; m < 12; ++m) {
                p0bar[sl + m] += (1.0 - theta) * w12[m];
                p1bar[sl + m] += theta * w12[m];
            }
        }
    }
    block_partial<B>(0.0, dtau, K.partial, pslot);
}

// Sum of a double over the two lanes of a pair (DPP quad_perm 1,0,3,2): both
// lanes get the same bits, the addition being commutative.  Both lanes of the
// pair must be active.
__device__ __forceinline__ double pair_sum(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    const int lo2 = __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xF, 0xF, false);
    const int hi2 = __builtin_amdgcn_mov_dpp(hi, 0xB1, 0xF, 0xF, false);
    return v + __hiloint2double(hi2, lo2);
}

// k_adj_fv on small 8-slot meshes, two lanes per node: lane h of node k
// gathers slots 4h..4h+3 (one round of four table entries, then four pivot
// adjoints), the two partial sums are added with pair_sum, and lane 0 finishes
// the node.  The same terms as k_adj_fv, with the slot sum split in two halves.
// Threads 2 nn .. 2 nn + 2 n_int - 1 take the star values of the interpolation
// nodes on lane pairs of their own, so that those gathers run beside the
// stored-value gathers instead of after them.
template <int B>
__global__ __launch_bounds__(B) void k_adj_fv2(const KAdj K, const double* __restrict__ fin,
                                                const double* __restrict__ ybar, const double* __restrict__ zwall,
                                                double* __restrict__ mbar, const double* __restrict__ prep0,
                                                const double* __restrict__ prep1, double theta,
                                                double* __restrict__ p0bar, double* __restrict__ p1bar, int pslot,
                                                const double* __restrict__ wmom_prev, double* __restrict__ zwall_prev) {
    const KMesh& M = K.M;
    const int gt = blockIdx.x * blockDim.x + threadIdx.x;
    const bool star_lane = gt >= 2 * M.nn;
    const int k = star_lane ? M.n_core + ((gt - 2 * M.nn) >> 1) : gt >> 1;
    const int h = gt & 1;   // lanes 2k, 2k + 1: slots 0-3, 4-7 of node k
    double dtau = 0.0;
    const double rdt = K.ddtt_dtau / K.dtt;
    if (!star_lane && k < M.nn) {
        const bool k_interp = k >= M.n_core;
        {   // the stored value M^m_k
            double f[9], m0, ux, uy, feq[9], nq[9], vb[9], nqb[9];
            load_rec(fin + size_t(k) * kRec, f, m0, ux, uy);
            equilibrium<double, false>(m0, m0, ux, uy, feq);
#pragma unroll
            for (int q = 0; q < 9; ++q) nq[q] = f[q] - feq[q], vb[q] = nqb[q] = 0.0;
            adj_fv_gather<4, false, 4>(K, k, k_interp, ybar, zwall, f, nq, vb, nqb, 4 * h);
#pragma unroll
            for (int q = 0; q < 9; ++q) vb[q] = pair_sum(vb[q]), nqb[q] = pair_sum(nqb[q]);
            if (h == 0) {
            double a12[12] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                dtau += rdt * nq[q] * nqb[q];
                a12[3 + q] = nqb[q];
            }
            macro_neq_adj(f, a12, vb);
            store_adj(mbar + size_t(k) * kAdjRec, vb);
            if (wmom_prev && k < (M.wall_bc ? M.n_wall : 0)) {
                double zb[9];
                wall_reset_apply(wmom_prev + 3 * size_t(k), vb, zb);
                store_adj(zwall_prev + size_t(k) * kAdjRec, zb);
            }
            }
        }
    } else if (star_lane && k < M.nn) {   // the star value f*_k read by interpolation pivots
            const size_t sl = size_t(k - M.n_core) * kMacro;
            double v[12], fs[9], ns[9], fsb[9], nsb[9];
            star64(prep0 + sl, prep1 + sl, theta, K.cst, v, fs, ns);
#pragma unroll
            for (int q = 0; q < 9; ++q) fsb[q] = nsb[q] = 0.0;
            adj_fv_gather<4, true, 4>(K, k, true, ybar, zwall, fs, ns, fsb, nsb, 4 * h);
#pragma unroll
            for (int q = 0; q < 9; ++q) fsb[q] = pair_sum(fsb[q]), nsb[q] = pair_sum(nsb[q]);
            if (h == 0) {
            // fs = feq(v0, v1, v2) + cst v[3..], ns = cst v[3..]
            double rb = 0.0, uxb = 0.0, uyb = 0.0, w12[12], dcst = 0.0;
            feq_adj(v[0], v[1], v[2], fsb, rb, uxb, uyb);
            w12[0] = rb, w12[1] = uxb, w12[2] = uyb;
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                w12[3 + q] = K.cst * (fsb[q] + nsb[q]);
                dcst += (fsb[q] + nsb[q]) * v[3 + q];
                dtau += rdt * ns[q] * nsb[q];
            }
            dtau += dcst * K.dcst_dtau;
#pragma unroll
            for (int m = 0; m < 12; ++m) {
                p0bar[sl + m] += (1.0 - theta) * w12[m];
                p1bar[sl + m] += theta * w12[m];
            }
            }
    }
    block_partial<B>(0.0, dtau, K.partial, pslot);
}

// Collision adjoint (per collide-stream node x, edges included): with
// g = streamed populations, B = g - omega (g - feq(g)):
// prebar = (1 - omega) Bbar + omega J_feq(g)^T Bbar; tau through omega.
__global__ __launch_bounds__(256) void k_adj_collide(const KAdj K, const double* __restrict__ A,
                                                     const double* __restrict__ bbar, double* __restrict__ prebar,
                                                     int pslot) {
    const KLevel& L = K.L;
    const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    double dtau = 0.0;
    if (i < L.nx && j < L.ny) {
        const size_t base = size_t(j) * size_t(L.rs) + i;
        if (!is_active(L, i, j)) {
#pragma unroll
            for (int q = 0; q < 9; ++q) prebar[size_t(q) * L.pitch + base] = 0.0;
        } else {
            double g[9], feq[9], rho, ux, uy, bb[9], fb[9], eb[9];
            streamed<double, false>(L, A, i, j, g);
            macro64(g, rho, ux, uy);
            equilibrium<double, false>(rho, rho, ux, uy, feq);
            double domega = 0.0;
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                bb[q] = bbar[size_t(q) * L.pitch + base];
                fb[q] = (1.0 - K.omega) * bb[q];
                eb[q] = K.omega * bb[q];
                domega -= bb[q] * (g[q] - feq[q]);
            }
            double rb = 0.0, uxb = 0.0, uyb = 0.0;
            feq_adj(rho, ux, uy, eb, rb, uxb, uyb);
            macro_adj(rho, ux, uy, rb, uxb, uyb, fb);
#pragma unroll
            for (int q = 0; q < 9; ++q) prebar[size_t(q) * L.pitch + base] = fb[q];
            dtau = domega * K.domega_dtau;
        }
    }
    block_partial(0.0, dtau, K.partial, pslot + blockIdx.y * gridDim.x);
}

// Adjoint of eq. (9): prebar(d) += J_(rho,u,neq)(g_d)^T sum_s w_sd pbar_s, per donor d.
__global__ void k_adj_s2m(const KAdj K, const double* __restrict__ A, int nd, const int32_t* __restrict__ node,
                          const int32_t* __restrict__ ptr, const int32_t* __restrict__ slot,
                          const double* __restrict__ w, const double* __restrict__ pbar, double* __restrict__ prebar) {
    const KLevel& L = K.L;
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= nd) return;
    double a[12];
#pragma unroll
    for (int m = 0; m < 12; ++m) a[m] = 0.0;
    for (int z = ptr[d]; z < ptr[d + 1]; ++z) {
        const double ww = w[z];
        const double* pb = pbar + size_t(slot[z]) * kMacro;
#pragma unroll
        for (int m = 0; m < 12; ++m) a[m] += ww * pb[m];
    }
    const int id = node[d], i = id % L.nx, j = id / L.nx;
    double g[9], fb[9];
    pull(L, A, i, j, g);
#pragma unroll
    for (int q = 0; q < 9; ++q) fb[q] = 0.0;
    macro_neq_adj(g, a, fb);
    const size_t base = size_t(j) * size_t(L.rs) + i;
#pragma unroll
    for (int q = 0; q < 9; ++q) prebar[size_t(q) * L.pitch + base] += fb[q];
    if (K.w6bar) {   // d J / d w_sd = pbar_s . (rho, u, f^neq)(g_d)
        double mac[12], feq[9];
        macro64(g, mac[0], mac[1], mac[2]);
        equilibrium<double, false>(mac[0], mac[0], mac[1], mac[2], feq);
#pragma unroll
        for (int q = 0; q < 9; ++q) mac[3 + q] = g[q] - feq[q];
        for (int z = ptr[d]; z < ptr[d + 1]; ++z) {
            const double* pb = pbar + size_t(slot[z]) * kMacro;
            double acc = 0.0;
#pragma unroll
            for (int m = 0; m < 12; ++m) acc += pb[m] * mac[m];
            K.w6bar[z] += acc;
        }
    }
}

// Far-field boundary adjoint for one edge node: moves prebar(edge) onto the
// neighbour whose streamed populations the boundary condition used (Sec. 4);
// returns the angle-of-attack derivative (inlet velocity).
__device__ __forceinline__ double bc_adj_node(const KAdj& K, const double* A, double* prebar, int i, int j) {
    const KLevel& L = K.L;
    const int jc = j < 1 ? 1 : (j > L.ny - 2 ? L.ny - 2 : j);
    const int ni = (i == 0) ? 1 : (i == L.nx - 1 ? L.nx - 2 : i);
    const int nj = (i == 0 || i == L.nx - 1) ? jc : (j == 0 ? 1 : L.ny - 2);
    const size_t be = size_t(j) * size_t(L.rs) + i, bn = size_t(nj) * size_t(L.rs) + ni;
    double fb[9], gb[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        fb[q] = prebar[size_t(q) * L.pitch + be];
        prebar[size_t(q) * L.pitch + be] = 0.0;
        gb[q] = fb[q];
    }
    double dalpha = 0.0;
    if (i == 0 || i == L.nx - 1) {
        double g[9], rho, ux, uy, eb[9];
        pull(L, A, ni, nj, g);
        macro64(g, rho, ux, uy);
        double rb = 0.0, uxb = 0.0, uyb = 0.0;
#pragma unroll
        for (int q = 0; q < 9; ++q) eb[q] = -fb[q];
        feq_adj(rho, ux, uy, eb, rb, uxb, uyb);   // - feq(rho_g, u_g)
        if (i == 0) {   // + feq(rho_g, u_in)
            double rb2 = 0.0, ub_x = 0.0, ub_y = 0.0;
            feq_adj(rho, L.u_in_x, L.u_in_y, fb, rb2, ub_x, ub_y);
            rb += rb2;
            dalpha = ub_x * K.duin_x + ub_y * K.duin_y;
        } else {        // + feq(rho0, u_g)
            double rb2 = 0.0;
            feq_adj(L.rho0, ux, uy, fb, rb2, uxb, uyb);
        }
        macro_adj(rho, ux, uy, rb, uxb, uyb, gb);
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) prebar[size_t(q) * L.pitch + bn] += gb[q];
    return dalpha;
}

// part 0: bottom and top rows (copies); part 1: inlet and outlet columns
// without corners; part 2: the four corners, one thread, in order.
__global__ __launch_bounds__(256) void k_adj_bc(const KAdj K, const double* __restrict__ A, double* __restrict__ prebar,
                                                int part, int pslot) {
    const KLevel& L = K.L;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    double dalpha = 0.0;
    if (part == 0) {
        if (t < 2 * (L.nx - 2)) {
            const int i = 1 + (t % (L.nx - 2)), j = t < L.nx - 2 ? 0 : L.ny - 1;
            dalpha = bc_adj_node(K, A, prebar, i, j);
        }
    } else if (part == 1) {
        if (t < 2 * (L.ny - 2)) {
            const int j = 1 + (t % (L.ny - 2)), i = t < L.ny - 2 ? 0 : L.nx - 1;
            dalpha = bc_adj_node(K, A, prebar, i, j);
        }
    } else if (t == 0) {
        dalpha += bc_adj_node(K, A, prebar, 0, 0);
        dalpha += bc_adj_node(K, A, prebar, 0, L.ny - 1);
        dalpha += bc_adj_node(K, A, prebar, L.nx - 1, 0);
        dalpha += bc_adj_node(K, A, prebar, L.nx - 1, L.ny - 1);
    }
    block_partial(dalpha, 0.0, K.partial, pslot);
}

// Transpose of the pull: Abar(y)_q = prebar(y + c_q)_q when y + c_q pulls
// (a collide-stream node that is not a far-field edge), else 0.
__global__ __launch_bounds__(256) void k_adj_push(const KAdj K, const double* __restrict__ prebar,
                                                  double* __restrict__ abar) {
    const KLevel& L = K.L;
    const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (i >= L.nx || j >= L.ny) return;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        int a = i + CX[q], b = j + CY[q];
        if (L.periodic) {
            a = (a + L.nx) % L.nx;
            b = (b + L.ny) % L.ny;
        }
        double v = 0.0;
        const bool inb = a >= 0 && b >= 0 && a < L.nx && b < L.ny;
        const bool edge = L.farfield && (a == 0 || b == 0 || a == L.nx - 1 || b == L.ny - 1);
        if (inb && !edge && is_active(L, a, b)) v = prebar[lidx(L, q, a, b)];
        abar[lidx(L, q, i, j)] = v;
    }
}

// Adjoint of eq. (4), phase 1 (per structured interpolation node s): reads and
// clears Abar at the node, records the adjoint of (rho, u, f^neq) of the
// interpolant in m5bar; tau through 2 (tau - 1)/(2 tau - 1).
__global__ __launch_bounds__(256) void k_adj_m2s_a(const KAdj K, const double* __restrict__ mf, int n,
                                                   const int32_t* __restrict__ node, const int32_t* __restrict__ don,
                                                   const double* __restrict__ w, double* __restrict__ abar,
                                                   double* __restrict__ m5bar, int pslot) {
    const KLevel& L = K.L;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    double dtau = 0.0;
    if (s < n) {
        double acc[12];
#pragma unroll
        for (int m = 0; m < 12; ++m) acc[m] = 0.0;
        for (int d = 0; d < kSDon; ++d) {
            const int k = don[size_t(s) * kSDon + d];
            if (k < 0) break;
            double f[9], m0, ux, uy, feq[9];
            load_rec(mf + size_t(k) * kRec, f, m0, ux, uy);
            equilibrium<double, false>(m0, m0, ux, uy, feq);
            const double ww = w[size_t(s) * kSDon + d];
            acc[0] += ww * m0;
            acc[1] += ww * ux;
            acc[2] += ww * uy;
#pragma unroll
            for (int q = 0; q < 9; ++q) acc[3 + q] += ww * (f[q] - feq[q]);
        }
        const int id = node[s], i = id % L.nx, j = id / L.nx;
        const size_t base = size_t(j) * size_t(L.rs) + i;
        double vb[9];
        double dphi = 0.0;
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            vb[q] = abar[size_t(q) * L.pitch + base];
            abar[size_t(q) * L.pitch + base] = 0.0;
            dphi += vb[q] * acc[3 + q];
        }
        double rb = 0.0, uxb = 0.0, uyb = 0.0;
        feq_adj(acc[0], acc[1], acc[2], vb, rb, uxb, uyb);
        double* o = m5bar + size_t(s) * kMacro;
        o[0] = rb, o[1] = uxb, o[2] = uyb;
#pragma unroll
        for (int q = 0; q < 9; ++q) o[3 + q] = K.phi * vb[q];
        dtau = dphi * K.dphi_dtau;
    }
    block_partial(0.0, dtau, K.partial, pslot);
}

// Adjoint of eq. (4), phase 2 (per mesh donor d): mbar(d) += J_(rho,u,neq)(M_d)^T
// sum_s w_sd m5bar_s.
__global__ void k_adj_m2s_b(const KAdj K, const double* __restrict__ mf, const int32_t* __restrict__ ptr,
                            const int32_t* __restrict__ slot, const double* __restrict__ w,
                            const double* __restrict__ m5bar, double* __restrict__ mbar) {
    const int nn = K.M.nn;
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= nn || ptr[d] == ptr[d + 1]) return;
    double a[12];
#pragma unroll
    for (int m = 0; m < 12; ++m) a[m] = 0.0;
    for (int z = ptr[d]; z < ptr[d + 1]; ++z) {
        const double ww = w[z];
        const double* mb = m5bar + size_t(slot[z]) * kMacro;
#pragma unroll
        for (int m = 0; m < 12; ++m) a[m] += ww * mb[m];
    }
    double f[9], m0, ux, uy, fb[9];
    load_rec(mf + size_t(d) * kRec, f, m0, ux, uy);
#pragma unroll
    for (int q = 0; q < 9; ++q) fb[q] = 0.0;
    macro_neq_adj(f, a, fb);
#pragma unroll
    for (int q = 0; q < 9; ++q) mbar[size_t(d) * kAdjRec + q] += fb[q];
    if (K.w5bar) {   // d J / d w_sd = m5bar_s . (rho, u, f^neq)(M_d)
        double mac[12], feq[9];
        mac[0] = m0, mac[1] = ux, mac[2] = uy;
        equilibrium<double, false>(m0, m0, ux, uy, feq);
#pragma unroll
        for (int q = 0; q < 9; ++q) mac[3 + q] = f[q] - feq[q];
        for (int z = ptr[d]; z < ptr[d + 1]; ++z) {
            const double* mb = m5bar + size_t(slot[z]) * kMacro;
            double acc = 0.0;
#pragma unroll
            for (int m = 0; m < 12; ++m) acc += mb[m] * mac[m];
            K.w5bar[z] += acc;
        }
    }
}

// Angle-of-attack derivative through the initial state: sum over the uniform
// structured fill and the non-wall mesh nodes of abar . d feq(rho0, u_inf)/d alpha.
__global__ __launch_bounds__(256) void k_adj_alpha_state(const KAdj K, const double* __restrict__ abar,
                                                         const double* __restrict__ mbar, const double* __restrict__ dfeq,
                                                         int nmesh, int pslot) {
    const KLevel& L = K.L;
    const size_t nlev = size_t(L.ny) * size_t(L.rs);
    const size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    double da = 0.0;
    if (e < nlev) {
        da = abar[e] * dfeq[(e / size_t(L.pitch)) % 9];
    } else if (e < nlev + size_t(nmesh)) {
        const size_t P = e - nlev;
        if (!(K.M.wall_bc && int(P) < K.M.n_wall)) {
#pragma unroll
            for (int q = 0; q < 9; ++q) da += mbar[P * kAdjRec + q] * dfeq[q];
        }
    }
    block_partial(da, 0.0, K.partial, pslot);
}

// ---- refinement transfer (Sec. 4, Filippova-Haenel), reverse mode ----

// Coarse -> fine adjoint, pass 1 (per fine perimeter node k): the perimeter
// value is post = f^eq(rho, u) + coef v_neq, coef = (1 - 1/tau_f) tau_f/(2 tau_c)
// = (tau_f - 1)/(2 tau_c), with v = (rho, u, f^neq) the side values blended at
// theta; reads and clears the adjoint of the fine perimeter node and writes
// vbar_k = d J / d v.
__global__ __launch_bounds__(256) void k_adj_c2f_a(const KLevel C, const double* __restrict__ side_prev,
                                                   const double* __restrict__ side_cur, double theta,
                                                   double* __restrict__ ybar, double* __restrict__ vbar, double coef,
                                                   double dcoef, double* partial, int pslot) {
    const int cnx = C.nx - 1, cny = C.ny - 1, nxc = cnx / 2, nyc = cny / 2;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    double dtau = 0.0;
    if (k < 2 * (cnx + cny)) {
        int ic, jc;
        box_node(k, cnx, cny, ic, jc);
        int ka, kb = -1;
        if (!(ic & 1) && !(jc & 1)) ka = box_index(ic / 2, jc / 2, nxc, nyc);
        else if (ic & 1) ka = box_index((ic - 1) / 2, jc / 2, nxc, nyc), kb = box_index((ic + 1) / 2, jc / 2, nxc, nyc);
        else ka = box_index(ic / 2, (jc - 1) / 2, nxc, nyc), kb = box_index(ic / 2, (jc + 1) / 2, nxc, nyc);
        const double wa = kb < 0 ? 1.0 : 0.5;
        double v[kMacro];
#pragma unroll
        for (int m = 0; m < kMacro; ++m) {
            double x = wa * ((1.0 - theta) * side_prev[size_t(ka) * kMacro + m] + theta * side_cur[size_t(ka) * kMacro + m]);
            if (kb >= 0)
                x += wa * ((1.0 - theta) * side_prev[size_t(kb) * kMacro + m] + theta * side_cur[size_t(kb) * kMacro + m]);
            v[m] = x;
        }
        const size_t base = size_t(jc) * size_t(C.rs) + ic;
        double pb[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            pb[q] = ybar[size_t(q) * C.pitch + base];
            ybar[size_t(q) * C.pitch + base] = 0.0;
        }
        double rb = 0.0, uxb = 0.0, uyb = 0.0;
        feq_adj(v[0], v[1], v[2], pb, rb, uxb, uyb);
        double* o = vbar + size_t(k) * kMacro;
        o[0] = rb, o[1] = uxb, o[2] = uyb;
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            o[3 + q] = coef * pb[q];
            dtau += dcoef * pb[q] * v[3 + q];
        }
    }
    block_partial(0.0, dtau, partial, pslot);
}

// Coarse -> fine adjoint, pass 2 (per box-boundary node kk of the parent):
// gathers vbar of the fine perimeter nodes that read side entry kk (the even
// node on it, weight 1, and its odd neighbours along the perimeter, weight 1/2)
// into the adjoints of the side values at the parent's two times.
__global__ void k_adj_c2f_b(int nxc, int nyc, const double* __restrict__ vbar, double theta,
                            double* __restrict__ sbar_prev, double* __restrict__ sbar_cur) {
    const int kk = blockIdx.x * blockDim.x + threadIdx.x;
    if (kk >= 2 * (nxc + nyc)) return;
    const int cnx = 2 * nxc, cny = 2 * nyc;
    int a, b;
    box_node(kk, nxc, nyc, a, b);
    double acc[kMacro];
    const double* v0 = vbar + size_t(box_index(2 * a, 2 * b, cnx, cny)) * kMacro;
#pragma unroll
    for (int m = 0; m < kMacro; ++m) acc[m] = v0[m];
    auto add_half = [&](int ic, int jc) {
        const double* vv = vbar + size_t(box_index(ic, jc, cnx, cny)) * kMacro;
#pragma unroll
        for (int m = 0; m < kMacro; ++m) acc[m] += 0.5 * vv[m];
    };
    if (b == 0 || b == nyc) {
        if (2 * a - 1 >= 0) add_half(2 * a - 1, 2 * b);
        if (2 * a + 1 <= cnx) add_half(2 * a + 1, 2 * b);
    }
    if (a == 0 || a == nxc) {
        if (2 * b - 1 >= 0) add_half(2 * a, 2 * b - 1);
        if (2 * b + 1 <= cny) add_half(2 * a, 2 * b + 1);
    }
#pragma unroll
    for (int m = 0; m < kMacro; ++m) {
        sbar_prev[size_t(kk) * kMacro + m] += (1.0 - theta) * acc[m];
        sbar_cur[size_t(kk) * kMacro + m] += theta * acc[m];
    }
}

// Fine -> coarse adjoint (per ring node of the parent): post = f^eq(rho, u) +
// coef f^neq of the fine pulled populations, coef = 2 (tau_c - 1)/tau_f; reads
// and clears the parent's adjoint at the ring node and adds the adjoint of the
// pulled fine values to the child's buffer adjoint at their sources (each
// source belongs to one ring node, so the scatter has no conflicts).
__global__ __launch_bounds__(256) void k_adj_f2c(const KLevel P, const KLevel C, int ci0, int cj0, int nxc, int nyc,
                                                 const double* __restrict__ cprev, double* __restrict__ xbar,
                                                 double* __restrict__ ybar, double coef, double dcoef,
                                                 double* partial, int pslot) {
    const int rx = nxc - 2, ry = nyc - 2;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    double dtau = 0.0;
    if (k < 2 * (rx + ry)) {
        int a, b;
        box_node(k, rx, ry, a, b);
        const int pi = ci0 + 1 + a, pj = cj0 + 1 + b;
        const int fi = 2 * (pi - ci0), fj = 2 * (pj - cj0);
        double f[9], rho, ux, uy, feq[9];
        pull(C, cprev, fi, fj, f);
        macro64(f, rho, ux, uy);
        equilibrium<double, false>(rho, rho, ux, uy, feq);
        const size_t base = size_t(pj) * size_t(P.rs) + pi;
        double xb[9], a12[12] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            xb[q] = xbar[size_t(q) * P.pitch + base];
            xbar[size_t(q) * P.pitch + base] = 0.0;
            a12[3 + q] = coef * xb[q];
            dtau += dcoef * xb[q] * (f[q] - feq[q]);
        }
        feq_adj(rho, ux, uy, xb, a12[0], a12[1], a12[2]);
        double fb[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) fb[q] = 0.0;
        macro_neq_adj(f, a12, fb);
#pragma unroll
        for (int q = 0; q < 9; ++q) ybar[lidx(C, q, fi - CX[q], fj - CY[q])] += fb[q];
    }
    block_partial(0.0, dtau, partial, pslot);
}

// Fine -> coarse^T with the filtered transfer (the f^neq of the coincident fine
// node full-weighted over its 3 x 3 fine nodes).  One thread per fine node of
// the band those stencils cover: the perimeters of the fine rectangles at
// offsets 1, 2 (the coincident nodes) and 3 from the child's edge.  Each band
// node gathers w * coef * xbar of the up to four ring nodes whose stencil holds
// it, adds the (rho, u) adjoint of its own ring node if it is a coincident one,
// and scatters the result onto the populations it pulls (a fine node's pull
// sources are its own, so the scatter has one writer per entry).  xbar of the
// ring nodes is cleared by k_adj_f2c_clear afterwards.
__device__ __forceinline__ bool f2c_ring_fine(int x, int y, int nxc, int nyc) {
    const int x1 = 2 * (nxc - 1), y1 = 2 * (nyc - 1);
    return x >= 2 && x <= x1 && y >= 2 && y <= y1 && (x == 2 || x == x1 || y == 2 || y == y1);
}
__global__ __launch_bounds__(256) void k_adj_f2c_filt(const KLevel P, const KLevel C, int ci0, int cj0, int nxc,
                                                      int nyc, const double* __restrict__ cprev,
                                                      const double* __restrict__ xbar, double* __restrict__ ybar,
                                                      double coef, double dcoef, double* partial, int pslot) {
    const int rx = nxc - 2, ry = nyc - 2;
    // band rectangles (cells): offset 1 has 2 rx + 2 by 2 ry + 2, offset 2 has 2 rx by 2 ry,
    // offset 3 has 2 rx - 2 by 2 ry - 2
    const int n1 = 2 * ((2 * rx + 2) + (2 * ry + 2)), n2 = 2 * (2 * rx + 2 * ry);
    const int n3 = rx > 1 && ry > 1 ? 2 * ((2 * rx - 2) + (2 * ry - 2)) : 0;
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    double dtau = 0.0;
    if (t < n1 + n2 + n3) {
        int off, cx, cy;
        if (t < n1) { off = 1; cx = 2 * rx + 2; cy = 2 * ry + 2; }
        else if (t < n1 + n2) { t -= n1; off = 2; cx = 2 * rx; cy = 2 * ry; }
        else { t -= n1 + n2; off = 3; cx = 2 * rx - 2; cy = 2 * ry - 2; }
        int a, b;
        box_node(t, cx, cy, a, b);
        const int x = off + a, y = off + b;
        double f[9], rho, ux, uy, feq[9], nb[9];
        pull(C, cprev, x, y, f);
        macro64(f, rho, ux, uy);
        equilibrium<double, false>(rho, rho, ux, uy, feq);
#pragma unroll
        for (int q = 0; q < 9; ++q) nb[q] = 0.0;
        double a12[12] = {0.0, 0.0, 0.0};
        const int xs0 = (x & 1) ? x - 1 : x, xs1 = (x & 1) ? x + 1 : x;
        const int ys0 = (y & 1) ? y - 1 : y, ys1 = (y & 1) ? y + 1 : y;
        for (int ry_ = ys0; ry_ <= ys1; ry_ += 2)
            for (int rx_ = xs0; rx_ <= xs1; rx_ += 2) {
                if (!f2c_ring_fine(rx_, ry_, nxc, nyc)) continue;
                const double w = double((2 - abs(x - rx_)) * (2 - abs(y - ry_))) * 0.0625;
                const size_t base = size_t(cj0 + ry_ / 2) * size_t(P.rs) + (ci0 + rx_ / 2);
                double xb[9];
#pragma unroll
                for (int q = 0; q < 9; ++q) {
                    xb[q] = xbar[size_t(q) * P.pitch + base];
                    nb[q] += w * coef * xb[q];
                    dtau += dcoef * w * xb[q] * (f[q] - feq[q]);
                }
                if (rx_ == x && ry_ == y) feq_adj(rho, ux, uy, xb, a12[0], a12[1], a12[2]);
            }
#pragma unroll
        for (int q = 0; q < 9; ++q) a12[3 + q] = nb[q];
        double fb[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) fb[q] = 0.0;
        macro_neq_adj(f, a12, fb);
#pragma unroll
        for (int q = 0; q < 9; ++q) ybar[lidx(C, q, x - CX[q], y - CY[q])] += fb[q];
    }
    block_partial(0.0, dtau, partial, pslot);
}

// Clears xbar at the ring nodes after k_adj_f2c_filt has read it.
__global__ void k_adj_f2c_clear(const KLevel P, int ci0, int cj0, int nxc, int nyc, double* __restrict__ xbar) {
    const int rx = nxc - 2, ry = nyc - 2;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 2 * (rx + ry)) return;
    int a, b;
    box_node(k, rx, ry, a, b);
    const size_t base = size_t(cj0 + 1 + b) * size_t(P.rs) + (ci0 + 1 + a);
#pragma unroll
    for (int q = 0; q < 9; ++q) xbar[size_t(q) * P.pitch + base] = 0.0;
}

// Adjoint of the side values (rho, u, f^neq) recorded from the parent's pulled
// populations at its box-boundary nodes: prebar(node) += J^T sbar (per node).
__global__ void k_adj_side(const KLevel P, int ci0, int cj0, int nxc, int nyc, const double* __restrict__ A,
                           const double* __restrict__ sbar, double* __restrict__ prebar) {
    const int kk = blockIdx.x * blockDim.x + threadIdx.x;
    if (kk >= 2 * (nxc + nyc)) return;
    int a, b;
    box_node(kk, nxc, nyc, a, b);
    const int i = ci0 + a, j = cj0 + b;
    double g[9], fb[9];
    pull(P, A, i, j, g);
#pragma unroll
    for (int q = 0; q < 9; ++q) fb[q] = 0.0;
    macro_neq_adj(g, sbar + size_t(kk) * kMacro, fb);
    const size_t base = size_t(j) * size_t(P.rs) + i;
#pragma unroll
    for (int q = 0; q < 9; ++q) prebar[size_t(q) * P.pitch + base] += fb[q];
}

// One block adds the n partial pairs to acc in a fixed order: thread t sums
// slots t + j * kRedThreads into four accumulators by j mod 4 (four loads in
// flight), then the accumulators and the threads are added in a fixed tree.
constexpr int kRedThreads = 1024;
__global__ __launch_bounds__(kRedThreads) void k_reduce_partials(const double* __restrict__ partial, int n,
                                                                 double* acc) {
    __shared__ double sa[kRedThreads], sb[kRedThreads];
    double a[4] = {0.0, 0.0, 0.0, 0.0}, b[4] = {0.0, 0.0, 0.0, 0.0};
    int k = threadIdx.x;
    for (; k + 3 * kRedThreads < n; k += 4 * kRedThreads) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            a[j] += partial[2 * size_t(k + j * kRedThreads)];
            b[j] += partial[2 * size_t(k + j * kRedThreads) + 1];
        }
    }
    for (int j = 0; k < n; k += kRedThreads, ++j) {
        a[j] += partial[2 * size_t(k)];
        b[j] += partial[2 * size_t(k) + 1];
    }
    sa[threadIdx.x] = (a[0] + a[1]) + (a[2] + a[3]);
    sb[threadIdx.x] = (b[0] + b[1]) + (b[2] + b[3]);
    __syncthreads();
    for (int h = kRedThreads / 2; h > 0; h >>= 1) {
        if (int(threadIdx.x) < h) sa[threadIdx.x] += sa[threadIdx.x + h], sb[threadIdx.x] += sb[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) acc[0] += sa[0], acc[1] += sb[0];
}

}  // namespace

int adj_blocks_collide(const KLevel& L) { return int(blocks(L.nx)) * L.ny; }
int adj_blocks_nodes(int n) { return int(blocks(size_t(n > 0 ? n : 1))); }
// the FV sub-step adjoint takes two lanes per node (k_adj_fv2) on 8-slot
// meshes that give at most one wave per SIMD at one node per lane
bool adj_fv_two_lanes(const KMesh& M) {
    return M.ell_width == 8 && size_t(M.nn) <= size_t(kAdjFvSimds) * kAdjFvBlock;
}
int adj_fv_blocks(const KMesh& M) {
    const size_t n = M.nn > 0 ? size_t(M.nn) : 1, n_int = size_t(M.nn - M.n_core);
    return int(blocks(adj_fv_two_lanes(M) ? 2 * (n + n_int) : n, kAdjFvBlock));
}

void launch_zero(double* p, size_t n, hipStream_t s) {
    if (n) k_zero<<<blocks(n), 256, 0, s>>>(p, n);
}
void launch_adj_force(const KAdj& K, double* mbar, const double* vwall, double jx, double jy, const double* fst,
                      hipStream_t s) {
    if (K.M.n_wall > 0)
        k_adj_force<<<blocks(K.M.n_wall), 256, 0, s>>>(K.M.n_wall, mbar, vwall, jx, jy, fst, K.vbar);
}
void launch_adj_fv_wall(const KAdj& K, const double* wmom, const double* ybar, double* zwall, hipStream_t s) {
    if (K.M.wall_bc && K.M.n_wall > 0)
        k_adj_fv_wall<<<blocks(K.M.n_wall), 256, 0, s>>>(K, wmom, ybar, zwall);
}
void launch_adj_fv(const KAdj& K, const double* Mrec, const double* ybar, const double* zwall, double* mbar,
                   const double* prep0, const double* prep1, double theta, double* p0bar, double* p1bar, int pslot,
                   const double* wmom_prev, double* zwall_prev, hipStream_t s) {
    // Small 8-slot meshes (at most one wave per SIMD of one node per lane) take
    // two lanes per node, so each lane waits on one round of dependent loads;
    // measured on the 33k-node bump workload, (objective + adjoint)/forward:
    // 4.43, against 4.55 with one lane per node and slot groups of four and
    // 4.68 with pairs.  Larger meshes: one lane per node, slots in pairs (236
    // VGPRs, two waves per SIMD).
    const unsigned nb = unsigned(adj_fv_blocks(K.M));
    if (adj_fv_two_lanes(K.M))
        k_adj_fv2<kAdjFvBlock><<<nb, kAdjFvBlock, 0, s>>>(K, Mrec, ybar, zwall, mbar, prep0, prep1, theta, p0bar,
                                                              p1bar, pslot, wmom_prev, zwall_prev);
    else if (K.M.ell_width == 8)
        k_adj_fv<8, kAdjFvBlock, 2><<<nb, kAdjFvBlock, 0, s>>>(K, Mrec, ybar, zwall, mbar, prep0, prep1, theta, p0bar,
                                                              p1bar, pslot, wmom_prev, zwall_prev);
    else
        k_adj_fv<16, kAdjFvBlock, 2><<<nb, kAdjFvBlock, 0, s>>>(K, Mrec, ybar, zwall, mbar, prep0, prep1, theta, p0bar,
                                                               p1bar, pslot, wmom_prev, zwall_prev);
}
void launch_adj_collide(const KAdj& K, const double* A, const double* bbar, double* prebar, int pslot, hipStream_t s) {
    dim3 grid(blocks(K.L.nx), K.L.ny);
    k_adj_collide<<<grid, 256, 0, s>>>(K, A, bbar, prebar, pslot);
}
void launch_adj_s2m(const KAdj& K, const double* A, int nd, const int32_t* node, const int32_t* ptr,
                    const int32_t* slot, const double* w, const double* pbar, double* prebar, hipStream_t s) {
    if (nd > 0) k_adj_s2m<<<blocks(nd), 256, 0, s>>>(K, A, nd, node, ptr, slot, w, pbar, prebar);
}
void launch_adj_bc(const KAdj& K, const double* A, double* prebar, int pslot, hipStream_t s) {
    if (!K.L.farfield) return;
    k_adj_bc<<<blocks(2 * size_t(K.L.nx - 2)), 256, 0, s>>>(K, A, prebar, 0, pslot);
    k_adj_bc<<<blocks(2 * size_t(K.L.ny - 2)), 256, 0, s>>>(K, A, prebar, 1, pslot + int(blocks(2 * size_t(K.L.nx - 2))));
    k_adj_bc<<<1, 256, 0, s>>>(K, A, prebar, 2, pslot + int(blocks(2 * size_t(K.L.nx - 2))) + int(blocks(2 * size_t(K.L.ny - 2))));
}
void launch_adj_push(const KAdj& K, const double* prebar, double* abar, hipStream_t s) {
    dim3 grid(blocks(K.L.nx), K.L.ny);
    k_adj_push<<<grid, 256, 0, s>>>(K, prebar, abar);
}
void launch_adj_m2s_a(const KAdj& K, const double* Mrec, int n, const int32_t* node, const int32_t* don,
                      const double* w, double* abar, double* m5bar, int pslot, hipStream_t s) {
    k_adj_m2s_a<<<adj_blocks_nodes(n), 256, 0, s>>>(K, Mrec, n, node, don, w, abar, m5bar, pslot);
}
void launch_adj_m2s_b(const KAdj& K, const double* Mrec, const int32_t* ptr, const int32_t* slot, const double* w,
                      const double* m5bar, double* mbar, hipStream_t s) {
    k_adj_m2s_b<<<blocks(K.M.nn), 256, 0, s>>>(K, Mrec, ptr, slot, w, m5bar, mbar);
}
void launch_adj_alpha_state(const KAdj& K, const double* abar, const double* mbar, const double* dfeq, bool with_mesh,
                            int pslot, hipStream_t s) {
    const int nmesh = with_mesh ? K.M.nn : 0;
    const size_t n = size_t(K.L.ny) * size_t(K.L.rs) + size_t(nmesh);
    k_adj_alpha_state<<<blocks(n), 256, 0, s>>>(K, abar, mbar, dfeq, nmesh, pslot);
}
void launch_adj_c2f_a(const KLevel& C, const double* side_prev, const double* side_cur, double theta, double* ybar,
                      double* vbar, double coef, double dcoef, double* partial, int pslot, hipStream_t s) {
    const int n = 2 * (C.nx - 1 + C.ny - 1);
    k_adj_c2f_a<<<adj_blocks_nodes(n), 256, 0, s>>>(C, side_prev, side_cur, theta, ybar, vbar, coef, dcoef, partial, pslot);
}
void launch_adj_c2f_b(int nxc, int nyc, const double* vbar, double theta, double* sbar_prev, double* sbar_cur,
                      hipStream_t s) {
    k_adj_c2f_b<<<adj_blocks_nodes(2 * (nxc + nyc)), 256, 0, s>>>(nxc, nyc, vbar, theta, sbar_prev, sbar_cur);
}
int f2c_adj_threads(int nxc, int nyc, int filter) {
    const int rx = nxc - 2, ry = nyc - 2;
    if (!filter) return 2 * (rx + ry);
    return 2 * ((2 * rx + 2) + (2 * ry + 2)) + 2 * (2 * rx + 2 * ry) +
           (rx > 1 && ry > 1 ? 2 * ((2 * rx - 2) + (2 * ry - 2)) : 0);
}
void launch_adj_f2c(const KLevel& P, const KLevel& C, int ci0, int cj0, int nxc, int nyc, const double* cprev,
                    double* xbar, double* ybar, double coef, double dcoef, double* partial, int pslot, int filter,
                    hipStream_t s) {
    const int n = f2c_adj_threads(nxc, nyc, filter);
    if (!filter) {
        k_adj_f2c<<<adj_blocks_nodes(n), 256, 0, s>>>(P, C, ci0, cj0, nxc, nyc, cprev, xbar, ybar, coef, dcoef, partial,
                                                      pslot);
        return;
    }
    k_adj_f2c_filt<<<adj_blocks_nodes(n), 256, 0, s>>>(P, C, ci0, cj0, nxc, nyc, cprev, xbar, ybar, coef, dcoef,
                                                       partial, pslot);
    const int nr = 2 * (nxc - 2 + nyc - 2);
    k_adj_f2c_clear<<<blocks(nr), 256, 0, s>>>(P, ci0, cj0, nxc, nyc, xbar);
}
void launch_adj_side(const KLevel& P, int ci0, int cj0, int nxc, int nyc, const double* A, const double* sbar,
                     double* prebar, hipStream_t s) {
    k_adj_side<<<adj_blocks_nodes(2 * (nxc + nyc)), 256, 0, s>>>(P, ci0, cj0, nxc, nyc, A, sbar, prebar);
}
void launch_reduce_partials(const double* partial, int n, double* acc, hipStream_t s) {
    k_reduce_partials<<<1, kRedThreads, 0, s>>>(partial, n, acc);
}

// ===========================================================================
// ---- Wall statistics: running sums of C_p, C_f, C_n, eqs. (12)-(13) ----
// ===========================================================================

namespace {

// One thread per wall node (plan indices 0 .. n_wall-1, the first mesh records).
// Pressure is rho c_s^2.  The finite-volume scheme integrates the continuous
// BGK equation, so its viscous stress is sigma = -Pi^neq with
// Pi^neq = sum_q c_q c_q f_q - rho c_s^2 I - rho u u.  Shifted storage holds
// f_q - w_q rho0, whose moments lack (rho0, 0, rho0 c_s^2 I), so there the
// isotropic part subtracted is (rho - rho0) c_s^2.  nrm: unit normal n into the
// fluid; t = (n_y, -n_x).  Adds (C_p, t.sigma.n / q, n.sigma.n / q) to
// sum[0 | 1 | 2][P]; each thread owns its node (no atomics).
template <typename T, bool SHIFT>
__global__ __launch_bounds__(256) void k_wall_stats(const T* __restrict__ f, int n_wall,
                                                    const double* __restrict__ nrm, double rho0, double inv_q,
                                                    double* __restrict__ sum) {
    const int P = blockIdx.x * blockDim.x + threadIdx.x;
    if (P >= n_wall) return;
    T v[9], m0s, uxs, uys;
    load_rec<T>(f + size_t(P) * kRec, v, m0s, uxs, uys);
    double m0 = 0, mx = 0, my = 0, pxx = 0, pxy = 0, pyy = 0;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const double x = double(v[q]);
        m0 += x;
        mx += CX[q] * x;
        my += CY[q] * x;
        pxx += (CX[q] * CX[q]) * x;
        pxy += (CX[q] * CY[q]) * x;
        pyy += (CY[q] * CY[q]) * x;
    }
    constexpr double cs2 = 1.0 / 3.0;
    const double rho = SHIFT ? rho0 + m0 : m0;
    const double drho = SHIFT ? m0 : m0 - rho0;
    const double ux = mx / rho, uy = my / rho;
    const double iso = (SHIFT ? drho : rho) * cs2;
    const double sxx = -(pxx - iso - rho * ux * ux);
    const double sxy = -(pxy - rho * ux * uy);
    const double syy = -(pyy - iso - rho * uy * uy);
    const double nx = nrm[2 * P], ny = nrm[2 * P + 1];
    const double snx = sxx * nx + sxy * ny, sny = sxy * nx + syy * ny;
    sum[P] += drho * cs2 * inv_q;
    sum[n_wall + P] += (ny * snx - nx * sny) * inv_q;
    sum[2 * size_t(n_wall) + P] += (nx * snx + ny * sny) * inv_q;
}

// Means in the caller's node order: out[k][slot[P]] = sum[k][P] / n.
__global__ void k_wall_stats_final(int n_wall, const double* __restrict__ sum, const int32_t* __restrict__ slot,
                                   double n, double* __restrict__ out) {
    const int P = blockIdx.x * blockDim.x + threadIdx.x;
    if (P >= n_wall) return;
    const int r = slot[P];
#pragma unroll
    for (int k = 0; k < 3; ++k) out[size_t(k) * n_wall + r] = sum[size_t(k) * n_wall + P] / n;
}

}  // namespace

void launch_wall_stats(int prec, const void* f, int n_wall, const double* nrm, double rho0, double inv_q, double* sum,
                       hipStream_t s) {
    if (n_wall <= 0) return;
    HLBM_DISPATCH(prec, (k_wall_stats<T, S><<<blocks(n_wall), 256, 0, s>>>((const T*)f, n_wall, nrm, rho0, inv_q, sum)));
}

void launch_wall_stats_final(int n_wall, const double* sum, const int32_t* slot, double n, double* out, hipStream_t s) {
    if (n_wall <= 0) return;
    k_wall_stats_final<<<blocks(n_wall), 256, 0, s>>>(n_wall, sum, slot, n, out);
}

// ---------------------------------------------------------------------------
// Workspace of hlbm_create_noalloc: a file-scope device array, one copy per
// device, held until the process ends.  Host code reaches it only through the
// address that hipGetSymbolAddress returns for the current device (the array's
// name is a host-side stand-in, not a device address).
// ---------------------------------------------------------------------------

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

int noalloc_workspace(void** ptr) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return HLBM_E_DEVICE;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return HLBM_E_DEVICE;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return HLBM_OK;
}

}  // namespace hlbm
