// gfx950 kernels of the GMRES(3) smoother (Sec. 3.2.2): one application on
// a level replaces the iterate u by the u + z, z in K_3(A, r), r = f - A u,
// of least residual norm.
//
// The paper obtains the minimiser with GMRES (Arnoldi).  Here it is computed
// from the Gram matrix of the scaled power basis q_i = (A/s)^i r, i = 0..3,
// which needs one global reduction per application instead of one per
// Arnoldi step:
//     minimise || q0 + c1 q1 + c2 q2 + c3 q3 ||   over (c1, c2, c3)
//     u_new = u - (c1 q0 + c2 q1 + c3 q2) / s,   r_new = q0 + sum_i c_i q_i,
// the 3 x 3 normal equations solved by Cholesky after symmetric diagonal
// scaling (an exact breakdown of the Krylov space lowers the degree).  s is
// a bound of the Laplacian part of A (sum over axes of 4 / h^2) and only
// keeps the powers in range.  Passes per application:
//   k_sm_power  x2   q1 = (A/s) q0, q2 = (A/s) q1          (pointwise stencil)
//   k_sm_gram        q3 on the fly, Gram partials of q0..q3
//   k_sm_coef        fixed-order reduction, 3 x 3 solve, coefficients on device
//   pre-smoothing:   k_sm_apply_restrict: u1 and r_new (q3 on an LDS tile),
//                    full-weighting restriction of r_new to the next level
//                    (k_sm_apply_restrict_z on the finest 3D level)
//   post-smoothing:  k_sm_prolong_resid (before the passes above): u2 = u1 +
//                    P e and q0 = f - A u2 through an LDS tile; k_sm_apply_out
//                    (after them): the smoothed iterate.
// Every reduction is deterministic (fixed trees, fixed order).

#include "mg_kcommon.hpp"

namespace mg {

using namespace kc;

namespace {

struct SmPos {
    int slot, b, nb;
};

__device__ __forceinline__ SmPos sm_pos(const SmSlots& st) {
    SmPos q;
    const int pid = xcd_remap(blockIdx.x, gridDim.x);
    int lo = 0, hi = st.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (st.s[mid].block0 <= pid)
            lo = mid;
        else
            hi = mid - 1;
    }
    q.slot = lo;
    q.b = pid - st.s[lo].block0;
    q.nb = (lo + 1 < st.n ? st.s[lo + 1].block0 : st.nblocks) - st.s[lo].block0;
    return q;
}

// 32-bit index arithmetic: a level has fewer than 2^31 points.
__device__ __forceinline__ void grid_pos(int p, int nx, int ny, int& gx, int& gy, int& gz) {
    gx = p % nx;
    const int rr = p / nx;
    gy = rr % ny;
    gz = rr / ny;
}

// q0 at p: fscale f (f typed TQ) or the q0 buffer.
template <typename T, typename TQ>
__device__ __forceinline__ cx<T> load_q0(const SmSlot& sl, const SmoothBufs& B, long long p) {
    if (sl.f) return (T)fscale_of(sl) * cvt<T>(gin(static_cast<const cx<TQ>*>(sl.f))[p]);
    return gin(static_cast<const cx<T>*>(B.q[0]))[p];
}

// q_stage = (A/s) q_{stage-1}.
template <int D, typename T, typename TQ>
__global__ void __launch_bounds__(NT) k_sm_power(const SmArgs a, int stage) {
    const SmPos q = sm_pos(a.st);
    const SmSlot sl = a.st.s[q.slot];
    if (gated_off(sl.gate)) return;
    const GLevel<T> L = glevel(*static_cast<const LevelView<T>*>(sl.lv));
    const SmoothBufs B = *sl.sb;
    int lo, hi;
    chunk_range(L.N, q.nb, q.b, lo, hi);
    const auto y = gout(static_cast<cx<T>*>(sl.sb->q[stage]));
    const int nx = L.n[0], ny = L.n[1];
    const bool from_f = stage == 1 && sl.f;
    const T fsc = (T)fscale_of(sl);
    const auto fin = gin(static_cast<const cx<TQ>*>(sl.f));
    const auto qin = gin(static_cast<const cx<T>*>(sl.sb->q[stage > 0 ? stage - 1 : 0]));
    for (int p = lo + (int)threadIdx.x; p < hi; p += NT) {
        int gx, gy, gz;
        grid_pos(p, nx, ny, gx, gy, gz);
        cx<T> ax;
        if (from_f)
            ax = stencil_at<D, T, TQ>(L, fin, fsc, p, gx, gy, gz);
        else
            ax = stencil_at<D, T, T>(L, qin, T(1), p, gx, gy, gz);
        y[p] = L.sinv * ax;
    }
}

// q_stage = (A/s) q_{stage-1} on the finest 3D level as a z-march.  A
// workgroup owns a PZX x PZY column of points and up to PZC of its planes;
// each thread keeps its point's input on planes z-1, z, z+1 in registers,
// plane z with a one-point ring goes through LDS (two buffers, one barrier
// per plane), and the next plane's inputs are requested before the current
// one is formed.  Every input value is fetched from HBM about once (plus the
// ring) instead of through the pointwise kernel's scattered z neighbours.
// The terms and their order are those of stencil_at.
__device__ __forceinline__ int iclampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }
__device__ __forceinline__ int imin3(int a, int b) { return a < b ? a : b; }

template <typename T, typename TI>
__device__ __forceinline__ void pz_march(const GLevel<T>& L, GIn<cx<TI>> x, T xs, GOut<cx<T>> y, int b,
                                         cx<T>* P) {
    const int nx = L.n[0], ny = L.n[1], nz = L.n[2];
    const long long nxy = (long long)nx * ny;
    int ntx, nty, ntz;
    pz_counts(L.n, ntx, nty, ntz);
    const int tx = b % ntx, ty = (b / ntx) % nty, tz = b / (ntx * nty);
    const int x0 = tx * PZX, y0 = ty * PZY, z0 = tz * PZC;
    const int z1 = z0 + PZC < nz ? z0 + PZC : nz;
    const int t = (int)threadIdx.x;
    const int lx = t % PZX, ly = t / PZX;
    const int gx = x0 + lx, gy = y0 + ly;
    const bool own = gx < nx && gy < ny;
    const int cgx = gx < nx ? gx : nx - 1, cgy = gy < ny ? gy : ny - 1;
    const long long pxy = (long long)cgy * nx + cgx;
    // ring point of this thread (t < PZR): LDS position and clamped grid index
    const bool ring = t < PZR;
    int rlx = 0, rly = 0;
    pz_ring(ring ? t : 0, rlx, rly);
    const int rgx = iclampi(x0 + rlx - 1, 0, nx - 1), rgy = iclampi(y0 + rly - 1, 0, ny - 1);
    const long long rxy = (long long)rgy * nx + rgx;
    auto plane = [&](int z) { return (long long)iclampi(z, 0, nz - 1) * nxy; };
    // x and y coefficients of this thread's point, the masks of its neighbours
    const cx<T> cmx = L.cm[0][cgx], cpx = L.cp[0][cgx], c0x = L.c0[0][cgx];
    const cx<T> cmy = L.cm[1][cgy], cpy = L.cp[1][cgy], c0y = L.c0[1][cgy];
    const bool bxm = gx > 0, bxp = gx < nx - 1, bym = gy > 0, byp = gy < ny - 1;
    const int c = (ly + 1) * PZW + lx + 1;
    cx<T> xm = cvt<T>(x[plane(z0 - 1) + pxy]);
    cx<T> xc = cvt<T>(x[plane(z0) + pxy]);
    cx<T> xp = cvt<T>(x[plane(z0 + 1) + pxy]);
    cx<T> rc = cvt<T>(x[plane(z0) + rxy]);
    T k2c = L.k2[plane(z0) + pxy];
    for (int z = z0; z < z1; ++z) {
        // inputs of the next plane first
        const cx<T> xn = cvt<T>(x[plane(z + 2) + pxy]);
        const cx<T> rn = cvt<T>(x[plane(z + 1) + rxy]);
        const T k2n = L.k2[plane(z + 1) + pxy];
        const cx<T> cmz = L.cm[2][z], cpz = L.cp[2][z], c0z = L.c0[2][z];
        cx<T>* Pb = P + (z & 1) * (PZW * PZH);
        Pb[c] = xc;
        if (ring) Pb[rly * PZW + rlx] = rc;
        __syncthreads();
        const bool bzm = z > 0, bzp = z < nz - 1;
        cx<T> d = c0x + c0y;
        d = d + c0z;
        d = d - k2c * L.sigma;
        cx<T> ax = d * xc;
        ax = ax + masked(bxm, cmx) * Pb[c - 1];
        ax = ax + masked(bxp, cpx) * Pb[c + 1];
        ax = ax + masked(bym, cmy) * Pb[c - PZW];
        ax = ax + masked(byp, cpy) * Pb[c + PZW];
        ax = ax + masked(bzm, cmz) * xm;
        ax = ax + masked(bzp, cpz) * xp;
        if (own) y[(long long)z * nxy + pxy] = L.sinv * (xs * ax);
        xm = xc;
        xc = xp;
        xp = xn;
        rc = rn;
        k2c = k2n;
    }
}

template <typename T, typename TQ>
__global__ void __launch_bounds__(NT) k_sm_power_z(const SmArgs a, int stage) {
    static_assert(PZX * PZY == NT, "one point of the column per thread");
    __shared__ cx<T> P[2 * PZW * PZH];
    const SmPos q = sm_pos(a.st);
    const SmSlot sl = a.st.s[q.slot];
    if (gated_off(sl.gate)) return;
    const GLevel<T> L = glevel(*static_cast<const LevelView<T>*>(sl.lv));
    const auto y = gout(static_cast<cx<T>*>(sl.sb->q[stage]));
    if (stage == 1 && sl.f)
        pz_march<T, TQ>(L, gin(static_cast<const cx<TQ>*>(sl.f)), (T)fscale_of(sl), y, q.b, P);
    else
        pz_march<T, T>(L, gin(static_cast<const cx<T>*>(sl.sb->q[stage > 0 ? stage - 1 : 0])), T(1), y, q.b, P);
}

// Gram partials of q0..q3 on the finest 3D level, q3 = (A/s) q2 formed by
// the same z-march as k_sm_power_z; one partial per column piece.
template <typename T, typename TQ>
__global__ void __launch_bounds__(NT) k_sm_gram_z(const SmArgs a) {
    __shared__ cx<T> P[2 * PZW * PZH];
    __shared__ cx<double> sm[(NT / 64) * NUM_GRAM];
    const SmPos q = sm_pos(a.st);
    const SmSlot sl = a.st.s[q.slot];
    if (gated_off(sl.gate)) return;
    const GLevel<T> L = glevel(*static_cast<const LevelView<T>*>(sl.lv));
    const SmoothBufs B = *sl.sb;
    const auto x = gin(static_cast<const cx<T>*>(B.q[2]));
    const auto q1p = gin(static_cast<const cx<T>*>(B.q[1]));
    const bool from_f = sl.f != nullptr;
    const auto fin = gin(static_cast<const cx<TQ>*>(sl.f));
    const auto q0p = gin(static_cast<const cx<T>*>(B.q[0]));
    const T fsc = (T)fscale_of(sl);
    auto q0_at = [&](long long i) { return from_f ? fsc * cvt<T>(fin[i]) : q0p[i]; };
    const int nx = L.n[0], ny = L.n[1], nz = L.n[2];
    const long long nxy = (long long)nx * ny;
    int ntx, nty, ntz;
    pz_counts(L.n, ntx, nty, ntz);
    const int b = q.b;
    const int tx = b % ntx, ty = (b / ntx) % nty, tz = b / (ntx * nty);
    const int x0 = tx * PZX, y0 = ty * PZY, z0 = tz * PZC;
    const int z1 = z0 + PZC < nz ? z0 + PZC : nz;
    const int t = (int)threadIdx.x;
    const int lx = t % PZX, ly = t / PZX;
    const int gx = x0 + lx, gy = y0 + ly;
    const bool own = gx < nx && gy < ny;
    const int cgx = gx < nx ? gx : nx - 1, cgy = gy < ny ? gy : ny - 1;
    const long long pxy = (long long)cgy * nx + cgx;
    const bool ring = t < PZR;
    int rlx = 0, rly = 0;
    pz_ring(ring ? t : 0, rlx, rly);
    const int rgx = iclampi(x0 + rlx - 1, 0, nx - 1), rgy = iclampi(y0 + rly - 1, 0, ny - 1);
    const long long rxy = (long long)rgy * nx + rgx;
    auto plane = [&](int z) { return (long long)iclampi(z, 0, nz - 1) * nxy; };
    const cx<T> cmx = L.cm[0][cgx], cpx = L.cp[0][cgx], c0x = L.c0[0][cgx];
    const cx<T> cmy = L.cm[1][cgy], cpy = L.cp[1][cgy], c0y = L.c0[1][cgy];
    const bool bxm = gx > 0, bxp = gx < nx - 1, bym = gy > 0, byp = gy < ny - 1;
    const int c = (ly + 1) * PZW + lx + 1;
    cx<double> g[NUM_GRAM];
#pragma unroll
    for (int v = 0; v < NUM_GRAM; ++v) g[v] = mk(0.0, 0.0);
    cx<T> xm = x[plane(z0 - 1) + pxy];
    cx<T> xc = x[plane(z0) + pxy];
    cx<T> xp = x[plane(z0 + 1) + pxy];
    cx<T> rc = x[plane(z0) + rxy];
    T k2c = L.k2[plane(z0) + pxy];
    cx<T> a0 = q0_at(plane(z0) + pxy), a1 = q1p[plane(z0) + pxy];
    for (int z = z0; z < z1; ++z) {
        const cx<T> xn = x[plane(z + 2) + pxy];
        const cx<T> rn = x[plane(z + 1) + rxy];
        const T k2n = L.k2[plane(z + 1) + pxy];
        const cx<T> a0n = q0_at(plane(z + 1) + pxy), a1n = q1p[plane(z + 1) + pxy];
        const cx<T> cmz = L.cm[2][z], cpz = L.cp[2][z], c0z = L.c0[2][z];
        cx<T>* Pb = P + (z & 1) * (PZW * PZH);
        Pb[c] = xc;
        if (ring) Pb[rly * PZW + rlx] = rc;
        __syncthreads();
        const bool bzm = z > 0, bzp = z < nz - 1;
        cx<T> d = c0x + c0y;
        d = d + c0z;
        d = d - k2c * L.sigma;
        cx<T> ax = d * xc;
        ax = ax + masked(bxm, cmx) * Pb[c - 1];
        ax = ax + masked(bxp, cpx) * Pb[c + 1];
        ax = ax + masked(bym, cmy) * Pb[c - PZW];
        ax = ax + masked(byp, cpy) * Pb[c + PZW];
        ax = ax + masked(bzm, cmz) * xm;
        ax = ax + masked(bzp, cpz) * xp;
        if (own) {
            const cx<double> v0 = cvt<double>(a0), v1 = cvt<double>(a1), v2 = cvt<double>(xc);
            const cx<double> v3 = cvt<double>(L.sinv * ax);
            g[0].r = fabs2(v0, g[0].r);
            g[1].r = fabs2(v1, g[1].r);
            g[2].r = fabs2(v2, g[2].r);
            g[3].r = fabs2(v3, g[3].r);
            g[4] = cfmac(v0, v1, g[4]);
            g[5] = cfmac(v0, v2, g[5]);
            g[6] = cfmac(v0, v3, g[6]);
            g[7] = cfmac(v1, v2, g[7]);
            g[8] = cfmac(v1, v3, g[8]);
            g[9] = cfmac(v2, v3, g[9]);
        }
        xm = xc;
        xc = xp;
        xp = xn;
        rc = rn;
        k2c = k2n;
        a0 = a0n;
        a1 = a1n;
    }
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < NUM_GRAM; ++v) {
        const double r = wave_sum(g[v].r);
        const double i = wave_sum(g[v].i);
        if (lane == 0) sm[wave * NUM_GRAM + v] = mk(r, i);
    }
    __syncthreads();
    if ((int)threadIdx.x < NUM_GRAM) {
        cx<double> s = mk(0.0, 0.0);
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) s = s + sm[w * NUM_GRAM + threadIdx.x];
        a.part[((long long)q.slot * a.pstride + threadIdx.x) * a.bstride + q.b] = s;
    }
}

// Gram partials of q0..q3, accumulated in FP64.
template <int D, typename T, typename TQ>
__global__ void __launch_bounds__(NT) k_sm_gram(const SmArgs a) {
    __shared__ cx<double> sm[(NT / 64) * NUM_GRAM];
    const SmPos q = sm_pos(a.st);
    const SmSlot sl = a.st.s[q.slot];
    if (gated_off(sl.gate)) return;
    const GLevel<T> L = glevel(*static_cast<const LevelView<T>*>(sl.lv));
    const SmoothBufs B = *sl.sb;
    int lo, hi;
    chunk_range(L.N, q.nb, q.b, lo, hi);
    const auto q1p = gin(static_cast<const cx<T>*>(B.q[1]));
    const auto q2p = gin(static_cast<const cx<T>*>(B.q[2]));
    const int nx = L.n[0], ny = L.n[1];
    cx<double> g[NUM_GRAM];
#pragma unroll
    for (int v = 0; v < NUM_GRAM; ++v) g[v] = mk(0.0, 0.0);
    for (int p = lo + (int)threadIdx.x; p < hi; p += NT) {
        int gx, gy, gz;
        grid_pos(p, nx, ny, gx, gy, gz);
        const cx<double> v0 = cvt<double>(load_q0<T, TQ>(sl, B, p));
        const cx<double> v1 = cvt<double>(q1p[p]);
        const cx<double> v2 = cvt<double>(q2p[p]);
        const cx<double> v3 = cvt<double>(L.sinv * stencil_at<D, T, T>(L, q2p, T(1), p, gx, gy, gz));
        g[0].r += abs2(v0);
        g[1].r += abs2(v1);
        g[2].r += abs2(v2);
        g[3].r += abs2(v3);
        g[4] = g[4] + cmulc(v0, v1);
        g[5] = g[5] + cmulc(v0, v2);
        g[6] = g[6] + cmulc(v0, v3);
        g[7] = g[7] + cmulc(v1, v2);
        g[8] = g[8] + cmulc(v1, v3);
        g[9] = g[9] + cmulc(v2, v3);
    }
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < NUM_GRAM; ++v) {
        const double r = wave_sum(g[v].r);
        const double i = wave_sum(g[v].i);
        if (lane == 0) sm[wave * NUM_GRAM + v] = mk(r, i);
    }
    __syncthreads();
    if ((int)threadIdx.x < NUM_GRAM) {
        cx<double> s = mk(0.0, 0.0);
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) s = s + sm[w * NUM_GRAM + threadIdx.x];
        a.part[((long long)q.slot * a.pstride + threadIdx.x) * a.bstride + q.b] = s;
    }
}

// One workgroup per slot: fixed-order sums of the Gram partials, then solve.
__global__ void __launch_bounds__(NT) k_sm_coef(const SmCoefArgs a, double brk) {
    __shared__ cx<double> sm[(NT / 64) * NUM_GRAM];
    __shared__ cx<double> G[NUM_GRAM];
    const int slot = blockIdx.x;
    const CoefSlot& cs = a.s[slot];
    if (gated_off(cs.gate)) return;
    const int cnt = cs.cnt;
    cx<double> g[NUM_GRAM];
#pragma unroll
    for (int v = 0; v < NUM_GRAM; ++v) g[v] = mk(0.0, 0.0);
    const cx<double>* base = a.part + (long long)cs.pslot * a.pstride * a.bstride;
    for (int b = threadIdx.x; b < cnt; b += NT) {
#pragma unroll
        for (int v = 0; v < NUM_GRAM; ++v) g[v] = g[v] + base[(long long)v * a.bstride + b];
    }
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < NUM_GRAM; ++v) {
        const double r = wave_sum(g[v].r);
        const double i = wave_sum(g[v].i);
        if (lane == 0) sm[wave * NUM_GRAM + v] = mk(r, i);
    }
    __syncthreads();
    if ((int)threadIdx.x < NUM_GRAM) {
        cx<double> s = mk(0.0, 0.0);
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) s = s + sm[w * NUM_GRAM + threadIdx.x];
        G[threadIdx.x] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) solve_coef(G, brk, cs.coef);
}

template <typename T>
__device__ __forceinline__ void load_coef(const cx<double>* c, cx<T>& c1, cx<T>& c2, cx<T>& c3) {
    c1 = cvt<T>(c[0]);
    c2 = cvt<T>(c[1]);
    c3 = cvt<T>(c[2]);
}

// Tile position of a fused kernel's workgroup.
template <int D, int TX, int TY, int TZ>
__device__ __forceinline__ void tile_origin(int tile, int nx, int ny, int& x0, int& y0, int& z0) {
    const int ntx = (nx + TX - 1) / TX, nty = (ny + TY - 1) / TY;
    const int tx = tile % ntx;
    const int rest = tile / ntx;
    x0 = tx * TX;
    y0 = (rest % nty) * TY;
    z0 = (D == 3) ? (rest / nty) * TZ : 0;
}

// ---------------------------------------------------------------------------
// Pre-smoothing end: u1 = u - (c1 q0 + c2 q1 + c3 q2)/s on the tile, r1 =
// q0 + c1 q1 + c2 q2 + c3 q3 on [0, T] (q3 from q2 staged on [-1, T+1]), and
// the full-weighting restriction of r1 to the coarse points owned by the tile.
// Slot fields: f (q0 = fscale f; null: q0 buffer), u (incoming iterate when
// NZ), c (coarse right-hand side out), sb.
// ---------------------------------------------------------------------------
template <int D, typename T, typename TQ, bool NZ, int TX, int TY, int TZ>
__global__ void __launch_bounds__(NT) k_sm_apply_restrict(const CycleArgs a) {
    constexpr int TZE = (D == 3) ? TZ : 1;
    constexpr int QX = TX + 3, QY = TY + 3, QZ = (D == 3) ? TZ + 3 : 1;
    constexpr int RX = TX + 1, RY = TY + 1, RZ = (D == 3) ? TZ + 1 : 1;
    constexpr int NQ = QX * QY * QZ, NR = RX * RY * RZ;
    constexpr int CX = TX / 2, CY = TY / 2, CZ = (D == 3) ? TZ / 2 : 1;
    static_assert(TX % 2 == 0 && TY % 2 == 0 && (D == 2 || TZ % 2 == 0), "even tiles");

    __shared__ cx<T> sq[NQ];
    __shared__ cx<T> sr[NR];

    const int pid = xcd_remap(blockIdx.x, gridDim.x);
    const int slot = find_slot(a.st.s, a.st.n, pid);
    const CycleSlot sl = a.st.s[slot];
    if (gated_off(sl.gate)) return;
    const LevelView<T>* Lp = static_cast<const LevelView<T>*>(sl.lv);
    const GLevel<T> L = glevel(*Lp);
    const SmoothBufs B = *sl.sb;
    const int nx = L.n[0], ny = L.n[1], nz = L.n[2];
    int x0, y0, z0;
    tile_origin<D, TX, TY, TZE>(pid - sl.tile0, nx, ny, x0, y0, z0);
    const auto q1p = gin(static_cast<const cx<T>*>(B.q[1]));
    const auto q2p = gin(static_cast<const cx<T>*>(B.q[2]));
    const auto q0p = gin(static_cast<const cx<T>*>(B.q[0]));
    const auto f = gin(static_cast<const cx<TQ>*>(sl.f));
    const T fs = (T)fscale_of(sl);
    cx<T> c1, c2, c3;
    load_coef<T>(B.coef, c1, c2, c3);

    {
        // every load of the tile first (clamped index), then the masked
        // stores: a load under a branch would be waited for on its own
        constexpr int KQ = (NQ + NT - 1) / NT;
        cx<T> v[KQ];
        bool in[KQ];
#pragma unroll
        for (int k = 0; k < KQ; ++k) {
            const int idx = (int)threadIdx.x + k * NT;
            const int id = idx < NQ ? idx : NQ - 1;
            const int lx = id % QX;
            const int rr = id / QX;
            const int ly = rr % QY;
            const int lz = rr / QY;
            const int gx = x0 - 1 + lx, gy = y0 - 1 + ly;
            const int gz = (D == 3) ? z0 - 1 + lz : 0;
            in[k] = gx >= 0 && gx < nx && gy >= 0 && gy < ny && (D == 2 || (gz >= 0 && gz < nz));
            const int cx_ = gx < 0 ? 0 : (gx < nx ? gx : nx - 1);
            const int cy_ = gy < 0 ? 0 : (gy < ny ? gy : ny - 1);
            const int cz_ = gz < 0 ? 0 : (gz < nz ? gz : nz - 1);
            v[k] = q2p[((long long)cz_ * ny + cy_) * nx + cx_];
        }
#pragma unroll
        for (int k = 0; k < KQ; ++k) {
            const int idx = (int)threadIdx.x + k * NT;
            if (idx < NQ) sq[idx] = masked(in[k], v[k]);
        }
    }
    __syncthreads();

    const auto u1p = gout(static_cast<cx<T>*>(B.u1));
    const auto up = gin(static_cast<const cx<T>*>(sl.u));
    // the point loads of every round first (clamped index), then the rounds
    constexpr int KR = (NR + NT - 1) / NT;
    cx<T> lq0[KR], lq1[KR], lu[KR];
    T lk2[KR];
#pragma unroll
    for (int k = 0; k < KR; ++k) {
        const int idx = (int)threadIdx.x + k * NT;
        const int id = idx < NR ? idx : NR - 1;
        const int lx = id % RX;
        const int rr = id / RX;
        const int ly = rr % RY;
        const int lz = rr / RY;
        const int gx = imin3(x0 + lx, nx - 1), gy = imin3(y0 + ly, ny - 1);
        const int gz = (D == 3) ? imin3(z0 + lz, nz - 1) : 0;
        const long long g = ((long long)gz * ny + gy) * nx + gx;
        lq0[k] = f ? fs * cvt<T>(f[g]) : q0p[g];
        lq1[k] = q1p[g];
        lk2[k] = L.k2[g];
        if constexpr (NZ) lu[k] = up[g];
        else lu[k] = mk<T>(0, 0);
    }
#pragma unroll
    for (int k = 0; k < KR; ++k) {
        const int idx = (int)threadIdx.x + k * NT;
        if (idx >= NR) break;
        const int lx = idx % RX;
        const int rr = idx / RX;
        const int ly = rr % RY;
        const int lz = rr / RY;
        const int gx = x0 + lx, gy = y0 + ly;
        const int gz = (D == 3) ? z0 + lz : 0;
        cx<T> r = mk<T>(0, 0);
        if (gx < nx && gy < ny && (D == 2 || gz < nz)) {
            const long long g = ((long long)gz * ny + gy) * nx + gx;
            const cx<T> q0 = lq0[k];
            const cx<T> q1 = lq1[k];
            const int c = ((D == 3 ? lz + 1 : 0) * QY + (ly + 1)) * QX + (lx + 1);
            const cx<T> q2 = sq[c];
            cx<T> aq = diag_at<D>(L, gx, gy, gz, lk2[k]) * q2 + L.cm[0][gx] * sq[c - 1] +
                       L.cp[0][gx] * sq[c + 1] + L.cm[1][gy] * sq[c - QX] + L.cp[1][gy] * sq[c + QX];
            if constexpr (D == 3) aq = aq + L.cm[2][gz] * sq[c - QX * QY] + L.cp[2][gz] * sq[c + QX * QY];
            const cx<T> q3 = L.sinv * aq;
            r = q0 + c1 * q1 + c2 * q2 + c3 * q3;
            const bool own = lx < TX && ly < TY && (D == 2 || lz < TZ);
            if (own) {
                cx<T> u = L.sinv * (c1 * q0 + c2 * q1 + c3 * q2);
                if constexpr (NZ) u = lu[k] - u;
                else u = mk<T>(0, 0) - u;
                u1p[g] = u;
            }
        }
        sr[idx] = r;
    }
    __syncthreads();

    const int ncx = Lp[1].n[0], ncy = Lp[1].n[1], ncz = Lp[1].n[2];
    const auto fc = gout(static_cast<cx<T>*>(sl.c));
    for (int idx = threadIdx.x; idx < CX * CY * CZ; idx += NT) {
        const int cxl = idx % CX;
        const int rr = idx / CX;
        const int cyl = rr % CY;
        const int czl = rr / CY;
        const int Cx = x0 / 2 + cxl, Cy = y0 / 2 + cyl;
        const int Cz = (D == 3) ? z0 / 2 + czl : 0;
        if (Cx < ncx && Cy < ncy && (D == 2 || Cz < ncz)) {
            cx<T> acc = mk<T>(0, 0);
#pragma unroll
            for (int oz = (D == 3 ? -1 : 0); oz <= (D == 3 ? 1 : 0); ++oz) {
                const int zz = (D == 3) ? 2 * czl + 1 + oz : 0;
                const T wz = (D == 3) ? (oz == 0 ? T(0.5) : T(0.25)) : T(1);
#pragma unroll
                for (int oy = -1; oy <= 1; ++oy) {
                    const T wy = wz * (oy == 0 ? T(0.5) : T(0.25));
                    const int row = (zz * RY + 2 * cyl + 1 + oy) * RX + 2 * cxl + 1;
#pragma unroll
                    for (int ox = -1; ox <= 1; ++ox) {
                        const T w = wy * (ox == 0 ? T(0.5) : T(0.25));
                        acc = acc + w * sr[row + ox];
                    }
                }
            }
            fc[((long long)Cz * ncy + Cy) * ncx + Cx] = acc;
        }
    }
}

// ---------------------------------------------------------------------------
// The same pre-smoothing end on the finest 3D level as a z-march over the
// columns of the power passes (PZX x PZY points, up to PZC planes).  Per
// plane: q2 of the plane with a ring goes through LDS (its z neighbours stay
// in registers), r1 is formed on the column and on its high x and y edges
// (the fine points that the restriction of the column's coarse points
// reaches beyond it), u1 on the column; the coarse points of the column take
// the 9 in-plane terms of each of their three fine planes as the planes go by
// (the march runs one plane past its chunk for the last of them), in the
// order of the tile form.  Every input value is fetched from HBM about once.
// ---------------------------------------------------------------------------
template <typename T, typename TQ, bool NZ>
__global__ void __launch_bounds__(NT) k_sm_apply_restrict_z(const CycleArgs a) {
    constexpr int QW = PZX + 3, QH = PZY + 3;    // q2 plane: x in [-1, PZX + 1], y in [-1, PZY + 1]
    constexpr int RW = PZX + 1, RH = PZY + 1;    // r1 plane: x in [0, PZX], y in [0, PZY]
    constexpr int NE = RW * RH - PZX * PZY;      // r1 points on the column's high x and y edges
    constexpr int NRG = QW * QH - RW * RH;       // q2 points around the r1 plane
    constexpr int CXN = PZX / 2, CYN = PZY / 2;  // coarse columns whose centre lies in the column
    static_assert(PZX * PZY == NT && PZX % 2 == 0 && PZY % 2 == 0 && PZC % 2 == 0, "column geometry");
    static_assert(NE == PZX + PZY + 1 && NE <= NT && NRG <= NT && CXN * CYN <= NT, "plane geometry");
    __shared__ cx<T> Q[2][QW * QH];
    __shared__ cx<T> R[2][RW * RH];
    __shared__ cx<T> CXS[3][QW], CYS[3][QH];   // cm, c0, cp of the column's x and y positions

    const int pid = xcd_remap(blockIdx.x, gridDim.x);
    const int slot = find_slot(a.st.s, a.st.n, pid);
    const CycleSlot sl = a.st.s[slot];
    if (gated_off(sl.gate)) return;
    const LevelView<T>* Lp = static_cast<const LevelView<T>*>(sl.lv);
    const GLevel<T> L = glevel(*Lp);
    const SmoothBufs B = *sl.sb;
    const int nx = L.n[0], ny = L.n[1], nz = L.n[2];
    const long long nxy = (long long)nx * ny;
    int ntx, nty, ntz;
    pz_counts(L.n, ntx, nty, ntz);
    const int b = pid - sl.tile0;
    const int tx = b % ntx, ty = (b / ntx) % nty, tz = b / (ntx * nty);
    const int x0 = tx * PZX, y0 = ty * PZY, z0 = tz * PZC;
    const int z1 = imin3(z0 + PZC, nz);
    const int zl = z1 < nz ? z1 : nz - 1;   // last plane of the march
    const auto q2p = gin(static_cast<const cx<T>*>(B.q[2]));
    const auto q1p = gin(static_cast<const cx<T>*>(B.q[1]));
    const auto q0p = gin(static_cast<const cx<T>*>(B.q[0]));
    const auto f = gin(static_cast<const cx<TQ>*>(sl.f));
    const bool from_f = sl.f != nullptr;
    const T fs = (T)fscale_of(sl);
    const auto up = gin(static_cast<const cx<T>*>(sl.u));
    const auto u1p = gout(static_cast<cx<T>*>(B.u1));
    cx<T> c1, c2, c3;
    load_coef<T>(B.coef, c1, c2, c3);
    auto plane = [&](int z) { return (long long)iclampi(z, 0, nz - 1) * nxy; };
    for (int i = (int)threadIdx.x; i < 3 * (QW + QH); i += NT) {
        const int w = i < 3 * QW ? i / QW : (i - 3 * QW) / QH;
        const int ax = i < 3 * QW ? 0 : 1;
        const int j = i < 3 * QW ? i % QW : (i - 3 * QW) % QH;
        const int g = ax == 0 ? iclampi(x0 + j - 1, 0, nx - 1) : iclampi(y0 + j - 1, 0, ny - 1);
        const cx<T> v = w == 0 ? L.cm[ax][g] : (w == 1 ? L.c0[ax][g] : L.cp[ax][g]);
        if (ax == 0) CXS[w][j] = v;
        else CYS[w][j] = v;
    }
    auto q0_at = [&](long long i) { return from_f ? fs * cvt<T>(f[i]) : q0p[i]; };

    const int t = (int)threadIdx.x;
    // a point of the r1 plane: mask, grid index (clamped for loads) and LDS
    // positions
    struct Pt {
        bool in;
        long long xy;
        int qx, qy, qc, rc;
    };
    auto pt_of = [&](int lx, int ly) {
        Pt p;
        const int gx = x0 + lx, gy = y0 + ly;
        p.in = gx < nx && gy < ny;
        p.xy = (long long)imin3(gy, ny - 1) * nx + imin3(gx, nx - 1);
        p.qx = lx + 1;
        p.qy = ly + 1;
        p.qc = p.qy * QW + p.qx;
        p.rc = ly * RW + lx;
        return p;
    };
    const Pt po = pt_of(t % PZX, t / PZX);
    // the edge points go to the last NE threads, the ring to the first NRG,
    // the coarse columns to the second wavefront: the waves share the extra work
    const int te = t - (NT - NE);
    const bool has_e = te >= 0;
    const Pt pe = pt_of(te >= 0 && te < PZX ? te : PZX, te >= 0 && te < PZX ? PZY : iclampi(te - PZX, 0, PZY));
    // q2 ring point of this thread (t < NRG), in LDS plane coordinates
    const bool has_r = t < NRG;
    int rqx, rqy;
    {
        const int r = has_r ? t : 0;
        if (r < QH) {
            rqx = 0;
            rqy = r;
        } else if (r < 2 * QH) {
            rqx = QW - 1;
            rqy = r - QH;
        } else if (r < 2 * QH + QW - 2) {
            rqx = r - 2 * QH + 1;
            rqy = 0;
        } else {
            rqx = r - 2 * QH - (QW - 2) + 1;
            rqy = QH - 1;
        }
    }
    const int rgx = x0 + rqx - 1, rgy = y0 + rqy - 1;
    const bool rin = rgx >= 0 && rgx < nx && rgy >= 0 && rgy < ny;
    const long long rxy = (long long)iclampi(rgy, 0, ny - 1) * nx + iclampi(rgx, 0, nx - 1);

    // registers: q2 of planes z-1, z, z+1 (and z+2 in flight), q0, q1, k2 (u)
    // of plane z (and z+1 in flight), for the column point (o) and the edge
    // point (e); the ring's q2 of plane z (and z+1)
    cx<T> om = masked(po.in, q2p[plane(z0 - 1) + po.xy]), oc = masked(po.in, q2p[plane(z0) + po.xy]);
    cx<T> op = masked(po.in, q2p[plane(z0 + 1) + po.xy]);
    cx<T> em = masked(pe.in, q2p[plane(z0 - 1) + pe.xy]), ec = masked(pe.in, q2p[plane(z0) + pe.xy]);
    cx<T> ep = masked(pe.in, q2p[plane(z0 + 1) + pe.xy]);
    cx<T> o0 = q0_at(plane(z0) + po.xy), o1 = q1p[plane(z0) + po.xy];
    cx<T> e0 = q0_at(plane(z0) + pe.xy), e1 = q1p[plane(z0) + pe.xy];
    T ok2 = L.k2[plane(z0) + po.xy], ek2 = L.k2[plane(z0) + pe.xy];
    cx<T> ou = mk<T>(0, 0);
    if constexpr (NZ) ou = up[plane(z0) + po.xy];
    cx<T> rcv = masked(rin, q2p[plane(z0) + rxy]);

    // restriction: coarse column (Cx, Cy) of this thread (t < CXN * CYN)
    const int ncx = Lp[1].n[0], ncy = Lp[1].n[1], ncz = Lp[1].n[2];
    const int tc = t - 64;
    const int cxl = (tc & 0xffff) % CXN, cyl = ((tc & 0xffff) / CXN) % CYN;
    const int Cx = x0 / 2 + cxl, Cy = y0 / 2 + cyl;
    const bool cown = tc >= 0 && tc < CXN * CYN && Cx < ncx && Cy < ncy;
    const auto fc = gout(static_cast<cx<T>*>(sl.c));
    cx<T> acc = mk<T>(0, 0);
    // the 9 in-plane terms of fine plane oz (-1, 0, 1) of a coarse point
    auto terms = [&](const cx<T>* Rb, int oz) {
        const T wz = oz == 0 ? T(0.5) : T(0.25);
#pragma unroll
        for (int oy = -1; oy <= 1; ++oy) {
            const T wy = wz * (oy == 0 ? T(0.5) : T(0.25));
            const int row = (2 * cyl + 1 + oy) * RW + 2 * cxl + 1;
#pragma unroll
            for (int ox = -1; ox <= 1; ++ox) {
                const T w = wy * (ox == 0 ? T(0.5) : T(0.25));
                acc = acc + w * Rb[row + ox];
            }
        }
    };

    for (int z = z0; z <= zl; ++z) {
        // inputs of the next plane first
        const cx<T> on = masked(po.in, q2p[plane(z + 2) + po.xy]);
        const cx<T> en = masked(pe.in, q2p[plane(z + 2) + pe.xy]);
        const cx<T> o0n = q0_at(plane(z + 1) + po.xy), o1n = q1p[plane(z + 1) + po.xy];
        const cx<T> e0n = q0_at(plane(z + 1) + pe.xy), e1n = q1p[plane(z + 1) + pe.xy];
        const T ok2n = L.k2[plane(z + 1) + po.xy], ek2n = L.k2[plane(z + 1) + pe.xy];
        cx<T> oun = mk<T>(0, 0);
        if constexpr (NZ) oun = up[plane(z + 1) + po.xy];
        const cx<T> rn = masked(rin, q2p[plane(z + 1) + rxy]);
        const cx<T> cmz = L.cm[2][z], cpz = L.cp[2][z], c0z = L.c0[2][z];
        const bool bzm = z > 0, bzp = z < nz - 1;
        cx<T>* Qb = Q[z & 1];
        cx<T>* Rb = R[z & 1];
        Qb[po.qc] = oc;
        if (has_e) Qb[pe.qc] = ec;
        if (has_r) Qb[rqy * QW + rqx] = rcv;
        __syncthreads();
        // r1 (and u1 on the column) at a point of the plane
        auto form = [&](const Pt& p, cx<T> q2m, cx<T> q2c, cx<T> q2pp, cx<T> q0, cx<T> q1, T k2, bool col,
                        cx<T> u) {
            cx<T> d = CXS[1][p.qx] + CYS[1][p.qy];
            d = d + c0z;
            d = d - k2 * L.sigma;
            cx<T> aq = d * q2c + CXS[0][p.qx] * Qb[p.qc - 1] + CXS[2][p.qx] * Qb[p.qc + 1] +
                       CYS[0][p.qy] * Qb[p.qc - QW] + CYS[2][p.qy] * Qb[p.qc + QW];
            aq = aq + masked(bzm, cmz) * q2m + masked(bzp, cpz) * q2pp;
            const cx<T> q3 = L.sinv * aq;
            const cx<T> r = q0 + c1 * q1 + c2 * q2c + c3 * q3;
            Rb[p.rc] = masked(p.in, r);
            if (col && p.in && z < z1) {
                cx<T> v = L.sinv * (c1 * q0 + c2 * q1 + c3 * q2c);
                if constexpr (NZ) v = u - v;
                else v = mk<T>(0, 0) - v;
                u1p[(long long)z * nxy + p.xy] = v;
            }
        };
        form(po, om, oc, op, o0, o1, ok2, true, ou);
        if (has_e) form(pe, em, ec, ep, e0, e1, ek2, false, ou);
        __syncthreads();
        if (cown) {
            if ((z & 1) == 0) {
                const int Ce = z / 2 - 1;   // its third plane
                if (z > z0) {
                    terms(Rb, 1);
                    if (Ce < ncz) fc[((long long)Ce * ncy + Cy) * ncx + Cx] = acc;
                }
                acc = mk<T>(0, 0);
                if (z < z0 + PZC && z / 2 < ncz) terms(Rb, -1);   // its first plane
            } else {
                terms(Rb, 0);
            }
        }
        om = oc;
        oc = op;
        op = on;
        em = ec;
        ec = ep;
        ep = en;
        o0 = o0n;
        o1 = o1n;
        e0 = e0n;
        e1 = e1n;
        ok2 = ok2n;
        ek2 = ek2n;
        ou = oun;
        rcv = rn;
    }
}

// ---------------------------------------------------------------------------
// Post-smoothing start: u2 = u1 + P e through an LDS tile (e on the coarse
// points around the tile, u2 on [-1, T]); writes u2 and q0 = fscale f - A u2
// on the tile.  Slot fields: f, fscale, c (coarse correction e), sb.
// ---------------------------------------------------------------------------
template <int D, typename T, typename TF, int TX, int TY, int TZ>
__global__ void __launch_bounds__(NT) k_sm_prolong_resid(const CycleArgs a) {
    constexpr int TZE = (D == 3) ? TZ : 1;
    constexpr int EX = TX / 2 + 2, EY = TY / 2 + 2, EZ = (D == 3) ? TZ / 2 + 2 : 1;
    constexpr int WX = TX + 2, WY = TY + 2, WZ = (D == 3) ? TZ + 2 : 1;
    constexpr int NE = EX * EY * EZ, NW = WX * WY * WZ;

    __shared__ cx<T> se[NE];
    __shared__ cx<T> s2[NW];

    const int pid = xcd_remap(blockIdx.x, gridDim.x);
    const int slot = find_slot(a.st.s, a.st.n, pid);
    const CycleSlot sl = a.st.s[slot];
    if (gated_off(sl.gate)) return;
    const LevelView<T>* Lp = static_cast<const LevelView<T>*>(sl.lv);
    const GLevel<T> L = glevel(*Lp);
    const SmoothBufs B = *sl.sb;
    const int nx = L.n[0], ny = L.n[1], nz = L.n[2];
    const int ncx = Lp[1].n[0], ncy = Lp[1].n[1], ncz = Lp[1].n[2];
    int x0, y0, z0;
    tile_origin<D, TX, TY, TZE>(pid - sl.tile0, nx, ny, x0, y0, z0);
    const auto f = gin(static_cast<const cx<TF>*>(sl.f));
    const T fs = (T)fscale_of(sl);
    const auto ec = gin(static_cast<const cx<T>*>(sl.c));
    const auto u1p = gin(static_cast<const cx<T>*>(B.u1));
    const int cxs = x0 / 2 - 1, cys = y0 / 2 - 1, czs = (D == 3) ? z0 / 2 - 1 : 0;

    // every load of a stage first (clamped index), masked at use: a load
    // under a bounds branch would be waited for on its own
    {
        constexpr int KE = (NE + NT - 1) / NT;
        cx<T> v[KE];
        bool in[KE];
#pragma unroll
        for (int k = 0; k < KE; ++k) {
            const int idx = (int)threadIdx.x + k * NT;
            const int id = idx < NE ? idx : NE - 1;
            const int lx = id % EX;
            const int rr = id / EX;
            const int ly = rr % EY;
            const int lz = rr / EY;
            const int Cx = cxs + lx, Cy = cys + ly, Cz = czs + lz;
            in[k] = Cx >= 0 && Cx < ncx && Cy >= 0 && Cy < ncy && (D == 2 || (Cz >= 0 && Cz < ncz));
            const int ccx = iclampi(Cx, 0, ncx - 1), ccy = iclampi(Cy, 0, ncy - 1);
            const int ccz = (D == 3) ? iclampi(Cz, 0, ncz - 1) : 0;
            v[k] = ec[((long long)ccz * ncy + ccy) * ncx + ccx];
        }
#pragma unroll
        for (int k = 0; k < KE; ++k) {
            const int idx = (int)threadIdx.x + k * NT;
            if (idx < NE) se[idx] = masked(in[k], v[k]);
        }
    }
    __syncthreads();

    constexpr int KW = (NW + NT - 1) / NT;
    cx<T> lu1[KW];
#pragma unroll
    for (int k = 0; k < KW; ++k) {
        const int idx = (int)threadIdx.x + k * NT;
        const int id = idx < NW ? idx : NW - 1;
        const int lx = id % WX;
        const int rr = id / WX;
        const int ly = rr % WY;
        const int lz = rr / WY;
        const int gx = iclampi(x0 - 1 + lx, 0, nx - 1), gy = iclampi(y0 - 1 + ly, 0, ny - 1);
        const int gz = (D == 3) ? iclampi(z0 - 1 + lz, 0, nz - 1) : 0;
        lu1[k] = u1p[((long long)gz * ny + gy) * nx + gx];
    }
#pragma unroll
    for (int k = 0; k < KW; ++k) {
        const int idx = (int)threadIdx.x + k * NT;
        if (idx >= NW) break;
        const int lx = idx % WX;
        const int rr = idx / WX;
        const int ly = rr % WY;
        const int lz = rr / WY;
        const int gx = x0 - 1 + lx, gy = y0 - 1 + ly;
        const int gz = (D == 3) ? z0 - 1 + lz : 0;
        cx<T> u2 = mk<T>(0, 0);
        if (gx >= 0 && gx < nx && gy >= 0 && gy < ny && (D == 2 || (gz >= 0 && gz < nz))) {
            int ix0, ix1, iy0, iy1;
            T wx0, wx1, wy0, wy1;
            interp_1d<T>(gx, cxs, ix0, ix1, wx0, wx1);
            interp_1d<T>(gy, cys, iy0, iy1, wy0, wy1);
            cx<T> pe;
            if constexpr (D == 2) {
                pe = (wy0 * wx0) * se[iy0 * EX + ix0] + (wy0 * wx1) * se[iy0 * EX + ix1] +
                     (wy1 * wx0) * se[iy1 * EX + ix0] + (wy1 * wx1) * se[iy1 * EX + ix1];
            } else {
                int iz0, iz1;
                T wz0, wz1;
                interp_1d<T>(gz, czs, iz0, iz1, wz0, wz1);
                const int p00 = (iz0 * EY + iy0) * EX, p01 = (iz0 * EY + iy1) * EX;
                const int p10 = (iz1 * EY + iy0) * EX, p11 = (iz1 * EY + iy1) * EX;
                pe = (wz0 * wy0 * wx0) * se[p00 + ix0] + (wz0 * wy0 * wx1) * se[p00 + ix1] +
                     (wz0 * wy1 * wx0) * se[p01 + ix0] + (wz0 * wy1 * wx1) * se[p01 + ix1] +
                     (wz1 * wy0 * wx0) * se[p10 + ix0] + (wz1 * wy0 * wx1) * se[p10 + ix1] +
                     (wz1 * wy1 * wx0) * se[p11 + ix0] + (wz1 * wy1 * wx1) * se[p11 + ix1];
            }
            u2 = lu1[k] + pe;
        }
        s2[idx] = u2;
    }
    __syncthreads();

    const auto u2p = gout(static_cast<cx<T>*>(B.u2));
    const auto q0p = gout(static_cast<cx<T>*>(B.q[0]));
    constexpr int NO = TX * TY * TZE, KO = (NO + NT - 1) / NT;
    T lk2[KO];
    cx<T> lf[KO];
#pragma unroll
    for (int k = 0; k < KO; ++k) {
        const int idx = (int)threadIdx.x + k * NT;
        const int id = idx < NO ? idx : NO - 1;
        const int lx = id % TX;
        const int rr = id / TX;
        const int ly = rr % TY;
        const int lz = rr / TY;
        const int gx = imin3(x0 + lx, nx - 1), gy = imin3(y0 + ly, ny - 1);
        const int gz = (D == 3) ? imin3(z0 + lz, nz - 1) : 0;
        const long long g = ((long long)gz * ny + gy) * nx + gx;
        lk2[k] = L.k2[g];
        lf[k] = cvt<T>(f[g]);
    }
#pragma unroll
    for (int k = 0; k < KO; ++k) {
        const int idx = (int)threadIdx.x + k * NT;
        if (idx >= NO) break;
        const int lx = idx % TX;
        const int rr = idx / TX;
        const int ly = rr % TY;
        const int lz = rr / TY;
        const int gx = x0 + lx, gy = y0 + ly;
        const int gz = (D == 3) ? z0 + lz : 0;
        if (gx < nx && gy < ny && (D == 2 || gz < nz)) {
            const long long g = ((long long)gz * ny + gy) * nx + gx;
            const int c = ((D == 3 ? lz + 1 : 0) * WY + (ly + 1)) * WX + (lx + 1);
            const cx<T> u2c = s2[c];
            cx<T> au = diag_at<D>(L, gx, gy, gz, lk2[k]) * u2c + L.cm[0][gx] * s2[c - 1] +
                       L.cp[0][gx] * s2[c + 1] + L.cm[1][gy] * s2[c - WX] + L.cp[1][gy] * s2[c + WX];
            if constexpr (D == 3) au = au + L.cm[2][gz] * s2[c - WX * WY] + L.cp[2][gz] * s2[c + WX * WY];
            u2p[g] = u2c;
            q0p[g] = fs * lf[k] - au;
        }
    }
}

// Post-smoothing end: out = u2 - (c1 q0 + c2 q1 + c3 q2)/s (or out +=).
template <typename T, typename TO, bool ACC>
__global__ void __launch_bounds__(NT) k_sm_apply_out(const SmArgs a) {
    const SmPos q = sm_pos(a.st);
    const SmSlot sl = a.st.s[q.slot];
    if (gated_off(sl.gate)) return;
    const GLevel<T> L = glevel(*static_cast<const LevelView<T>*>(sl.lv));
    const SmoothBufs B = *sl.sb;
    int lo, hi;
    chunk_range(L.N, q.nb, q.b, lo, hi);
    cx<T> c1, c2, c3;
    load_coef<T>(B.coef + 4, c1, c2, c3);
    const auto q0p = gin(static_cast<const cx<T>*>(B.q[0]));
    const auto q1p = gin(static_cast<const cx<T>*>(B.q[1]));
    const auto q2p = gin(static_cast<const cx<T>*>(B.q[2]));
    const auto u2p = gin(static_cast<const cx<T>*>(B.u2));
    const auto out = gout(static_cast<cx<TO>*>(sl.out));
    for (int p = lo + (int)threadIdx.x; p < hi; p += NT) {
        const cx<T> v = u2p[p] - L.sinv * (c1 * q0p[p] + c2 * q1p[p] + c3 * q2p[p]);
        if constexpr (ACC)
            out[p] = out[p].get() + cvt<TO>(v);
        else
            out[p] = cvt<TO>(v);
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_sm_power(int dim, bool f32, bool level0, int stage, const SmArgs& a, hipStream_t s) {
    if (a.st.n <= 0) return hipSuccess;
    if (stage != 1 && stage != 2) return hipErrorInvalidValue;
    dim3 grid(a.st.nblocks);
#define PW(D, T, TQ) hipLaunchKernelGGL((k_sm_power<D, T, TQ>), grid, dim3(NT), 0, s, a, stage)
    if (dim == 2) {
        if (!f32) PW(2, double, double);
        else if (level0) PW(2, float, double);
        else PW(2, float, float);
    } else {
        if (!f32) PW(3, double, double);
        else if (level0) PW(3, float, double);
        else PW(3, float, float);
    }
#undef PW
    return hipGetLastError();
}

hipError_t launch_sm_power_z(bool f32, bool level0, int stage, const SmArgs& a, hipStream_t s) {
    if (a.st.n <= 0) return hipSuccess;
    if (stage != 1 && stage != 2) return hipErrorInvalidValue;
    dim3 grid(a.st.nblocks);
    if (!f32)
        hipLaunchKernelGGL((k_sm_power_z<double, double>), grid, dim3(NT), 0, s, a, stage);
    else if (level0)
        hipLaunchKernelGGL((k_sm_power_z<float, double>), grid, dim3(NT), 0, s, a, stage);
    else
        hipLaunchKernelGGL((k_sm_power_z<float, float>), grid, dim3(NT), 0, s, a, stage);
    return hipGetLastError();
}

hipError_t launch_sm_gram_z(bool f32, bool level0, const SmArgs& a, hipStream_t s) {
    if (a.st.n <= 0) return hipSuccess;
    dim3 grid(a.st.nblocks);
    if (!f32)
        hipLaunchKernelGGL((k_sm_gram_z<double, double>), grid, dim3(NT), 0, s, a);
    else if (level0)
        hipLaunchKernelGGL((k_sm_gram_z<float, double>), grid, dim3(NT), 0, s, a);
    else
        hipLaunchKernelGGL((k_sm_gram_z<float, float>), grid, dim3(NT), 0, s, a);
    return hipGetLastError();
}

int power_z_tiles(const int n[3]) {
    int ntx, nty, ntz;
    pz_counts(n, ntx, nty, ntz);
    return ntx * nty * ntz;
}

hipError_t launch_sm_gram(int dim, bool f32, bool level0, const SmArgs& a, hipStream_t s) {
    if (a.st.n <= 0) return hipSuccess;
    dim3 grid(a.st.nblocks);
#define GR(D, T, TQ) hipLaunchKernelGGL((k_sm_gram<D, T, TQ>), grid, dim3(NT), 0, s, a)
    if (dim == 2) {
        if (!f32) GR(2, double, double);
        else if (level0) GR(2, float, double);
        else GR(2, float, float);
    } else {
        if (!f32) GR(3, double, double);
        else if (level0) GR(3, float, double);
        else GR(3, float, float);
    }
#undef GR
    return hipGetLastError();
}

hipError_t launch_sm_coef(bool f32, const SmCoefArgs& a, int nslots, hipStream_t s) {
    if (nslots <= 0) return hipSuccess;
    // an exhausted Krylov space shows as a relative Cholesky pivot at the
    // rounding level of the vectors' precision
    const double brk = f32 ? 1e-5 : 1e-13;
    hipLaunchKernelGGL(k_sm_coef, dim3(nslots), dim3(NT), 0, s, a, brk);
    return hipGetLastError();
}

template <typename T, typename TQ, bool NZ>
static hipError_t ar_launch(int dim, int shape, const CycleArgs& a, hipStream_t s) {
    dim3 grid(a.st.ntiles);
#define AR(D, X, Y, Z) hipLaunchKernelGGL((k_sm_apply_restrict<D, T, TQ, NZ, X, Y, Z>), grid, dim3(NT), 0, s, a);
    MG_SHAPE_SWITCH(AR)
#undef AR
    return hipGetLastError();
}

hipError_t launch_sm_apply_restrict(int dim, bool f32, bool level0, bool nonzero, int shape, const CycleArgs& a,
                                    hipStream_t s) {
    if (a.st.n <= 0) return hipSuccess;
    if (!f32)
        return nonzero ? ar_launch<double, double, true>(dim, shape, a, s)
                       : ar_launch<double, double, false>(dim, shape, a, s);
    if (nonzero) return hipErrorInvalidValue;   // the complex64 cycle always starts from zero
    return level0 ? ar_launch<float, double, false>(dim, shape, a, s) : ar_launch<float, float, false>(dim, shape, a, s);
}

hipError_t launch_sm_apply_restrict_z(bool f32, bool nonzero, const CycleArgs& a, hipStream_t s) {
    if (a.st.n <= 0) return hipSuccess;
    dim3 grid(a.st.ntiles);
    if (!f32) {
        if (nonzero)
            hipLaunchKernelGGL((k_sm_apply_restrict_z<double, double, true>), grid, dim3(NT), 0, s, a);
        else
            hipLaunchKernelGGL((k_sm_apply_restrict_z<double, double, false>), grid, dim3(NT), 0, s, a);
    } else {
        if (nonzero) return hipErrorInvalidValue;   // the complex64 cycle always starts from zero
        hipLaunchKernelGGL((k_sm_apply_restrict_z<float, double, false>), grid, dim3(NT), 0, s, a);
    }
    return hipGetLastError();
}

template <typename T, typename TF>
static hipError_t pr_launch(int dim, int shape, const CycleArgs& a, hipStream_t s) {
    dim3 grid(a.st.ntiles);
#define PR(D, X, Y, Z) hipLaunchKernelGGL((k_sm_prolong_resid<D, T, TF, X, Y, Z>), grid, dim3(NT), 0, s, a);
    MG_SHAPE_SWITCH(PR)
#undef PR
    return hipGetLastError();
}

hipError_t launch_sm_prolong_resid(int dim, bool f32, bool level0, int shape, const CycleArgs& a, hipStream_t s) {
    if (a.st.n <= 0) return hipSuccess;
    if (!f32) return pr_launch<double, double>(dim, shape, a, s);
    return level0 ? pr_launch<float, double>(dim, shape, a, s) : pr_launch<float, float>(dim, shape, a, s);
}

hipError_t launch_sm_apply_out(bool f32, bool level0, bool accumulate, const SmArgs& a, hipStream_t s) {
    if (a.st.n <= 0) return hipSuccess;
    dim3 grid(a.st.nblocks);
#define AO(T, TO, ACC) hipLaunchKernelGGL((k_sm_apply_out<T, TO, ACC>), grid, dim3(NT), 0, s, a)
    if (!f32) {
        if (accumulate) AO(double, double, true);
        else AO(double, double, false);
    } else if (level0) {
        if (accumulate) AO(float, double, true);
        else AO(float, double, false);
    } else {
        AO(float, float, false);
    }
#undef AO
    return hipGetLastError();
}

}  // namespace mg
