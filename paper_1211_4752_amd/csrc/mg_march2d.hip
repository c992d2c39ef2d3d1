// 2D GMRES(3) smoothing passes (Sec. 3.2.2) as row-marching wavefronts for
// gfx950.
//
// The minimiser of || q0 + c1 q1 + c2 q2 + c3 q3 ||, q_i = (A/s)^i r, comes
// from the Gram matrix of the q_i (mg_smooth.hip).  Here one wavefront owns
// a strip of MTX = 56 columns (lanes 4..59; 4 halo lanes on each side) and
// TY rows, and marches down the rows: every step loads one new row of the
// inputs and produces one new row of each power, each from the three most
// recent rows of the previous one held in registers; x-neighbours come from
// the adjacent lanes by shuffles.  Each input is read once per pass (plus the
// few warm-up rows and halo lanes, L2 hits), nothing but the outputs is
// written, and no LDS is used.
//   k_mg_gram<PRE>    pre-smoothing: q0 = fscale f (or the q0 buffer);
//   k_mg_gram<POST>   post-smoothing: u2 = u1 + P e, q0 = fscale f - A u2;
//                     Gram partials of q0..q3 per strip.
//   k_mg_apply_restrict  q0..q3 again, u1 = u - (c1 q0 + c2 q1 + c3 q2)/s,
//                     r1 = q0 + sum_i c_i q_i and its full-weighting
//                     restriction (pre-smoothing).
//   k_mg_apply_out    u2 and q0..q2 again, out = u2 - (c1 q0 + c2 q1 +
//                     c3 q2)/s (post-smoothing).
// Values outside the grid are zero (Dirichlet ghosts) at every stage.

#include "mg_kcommon.hpp"

namespace mg {

using namespace kc;

namespace {

constexpr int MW = 64;              // lanes per wavefront = workgroup size
constexpr int MH = 4;               // halo lanes on the left
constexpr int MTX = MW - 2 * MH;    // owned columns per strip

__device__ __forceinline__ int imin(int a, int b) { return a < b ? a : b; }

// Neighbour exchange across the wavefront by DPP lane shifts (VALU, no LDS):
// wave_shr:1 gives lane i the value of lane i - 1, wave_shl:1 that of lane
// i + 1; the end lanes receive 0 and are halo lanes whose results are unused.
__device__ __forceinline__ int dpp_from_left(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xF, 0xF, true); }
__device__ __forceinline__ int dpp_from_right(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xF, 0xF, true); }

template <bool LEFT>
__device__ __forceinline__ double lane_shift(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    int lo = (int)(unsigned)(b & 0xffffffffull), hi = (int)(unsigned)(b >> 32);
    lo = LEFT ? dpp_from_left(lo) : dpp_from_right(lo);
    hi = LEFT ? dpp_from_left(hi) : dpp_from_right(hi);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
template <bool LEFT>
__device__ __forceinline__ float lane_shift(float v) {
    const int b = __builtin_bit_cast(int, v);
    return __builtin_bit_cast(float, LEFT ? dpp_from_left(b) : dpp_from_right(b));
}
template <typename T>
__device__ __forceinline__ cx<T> shfl_up1(cx<T> v) {
    return mk<T>(lane_shift<true>(v.r), lane_shift<true>(v.i));
}
template <typename T>
__device__ __forceinline__ cx<T> shfl_dn1(cx<T> v) {
    return mk<T>(lane_shift<false>(v.r), lane_shift<false>(v.i));
}

// Per-lane column data of a strip.
template <typename T>
struct Lane {
    int gx;
    bool colv;
    bool own;
    cx<T> cmx, c0x, cpx;
};

template <typename T>
__device__ __forceinline__ Lane<T> lane_of(const GLevel<T>& L, int x0) {
    Lane<T> c;
    const int lane = threadIdx.x;
    c.gx = x0 - MH + lane;
    c.colv = c.gx >= 0 && c.gx < L.n[0];
    c.own = c.colv && lane >= MH && lane < MH + MTX;
    const int g = c.colv ? c.gx : 0;
    c.cmx = c.colv ? L.cm[0][g] : mk<T>(0, 0);
    c.c0x = c.colv ? L.c0[0][g] : mk<T>(0, 0);
    c.cpx = c.colv ? L.cp[0][g] : mk<T>(0, 0);
    return c;
}

// A at row y of the stage whose rows y-1, y, y+1 are am, a0, ap (this lane);
// every lane must call it (shuffles).  Caller masks the result.
template <typename T>
__device__ __forceinline__ cx<T> row_apply(const GLevel<T>& L, const Lane<T>& c, cx<T> am, cx<T> a0, cx<T> ap, int y,
                                           T k2) {
    const cx<T> left = shfl_up1(a0);
    const cx<T> right = shfl_dn1(a0);
    const int yy = (y >= 0 && y < L.n[1]) ? y : 0;
    const cx<T> d = c.c0x + L.c0[1][yy] - k2 * L.sigma;
    return d * a0 + c.cmx * left + c.cpx * right + L.cm[1][yy] * am + L.cp[1][yy] * ap;
}

template <typename T>
__device__ __forceinline__ bool rowv(const GLevel<T>& L, int y) {
    return y >= 0 && y < L.n[1];
}

template <typename T>
__device__ __forceinline__ T load_k2(const GLevel<T>& L, const Lane<T>& c, int y) {
    return (c.colv && rowv(L, y)) ? L.k2[(long long)y * L.n[0] + c.gx] : T(0);
}

// Bilinear interpolation of the coarse correction: per-lane x part.
template <typename T>
struct InterpX {
    int i0, i1;
    T w0, w1;
};

template <typename T>
__device__ __forceinline__ void interp_axis(int g, int nc, int& i0, int& i1, T& w0, T& w1) {
    if (g & 1) {
        i0 = i1 = (g - 1) / 2;
        w0 = T(1);
        w1 = T(0);
    } else {
        i0 = g / 2 - 1;
        i1 = g / 2;
        w0 = T(0.5);
        w1 = T(0.5);
    }
    if (i0 < 0 || i0 >= nc) {
        i0 = 0;
        w0 = T(0);
    }
    if (i1 < 0 || i1 >= nc) {
        i1 = 0;
        w1 = T(0);
    }
}

template <typename T>
__device__ __forceinline__ void gram_add(cx<double>* g, cx<T> a0, cx<T> a1, cx<T> a2, cx<T> a3) {
    const cx<double> v0 = cvt<double>(a0), v1 = cvt<double>(a1), v2 = cvt<double>(a2), v3 = cvt<double>(a3);
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

// One row of a pass's inputs at this lane, loaded ahead of its use (two rows
// in the Gram passes, one in the apply passes, where the extra registers
// would cost occupancy) so that the loads are in flight while row t is
// computed.
template <typename T, typename TQ>
struct RowIn {
    cx<T> u;                 // u1 (post-smoothing) or the incoming iterate
    cx<T> e00, e01, e10, e11;   // coarse correction around the point
    T v0, v1;                // row weights of the interpolation
    cx<TQ> f;                // right-hand side (or q0)
    T k2;
};

template <typename T, typename TQ, bool POST, bool Q0BUF>
__device__ __forceinline__ void load_row(RowIn<T, TQ>& r, const GLevel<T>& L, const GLevel<T>& Lc,
                                         const Lane<T>& c, const InterpX<T>& ix, const cx<T>* u, const cx<T>* e,
                                         const void* f, int y) {
    const cx<T> Z = mk<T>(0, 0);
    r.u = r.e00 = r.e01 = r.e10 = r.e11 = Z;
    r.v0 = r.v1 = T(0);
    r.f = mk<TQ>(0, 0);
    r.k2 = T(0);
    if (!(c.colv && rowv(L, y))) return;
    const long long gi = (long long)y * L.n[0] + c.gx;
    if constexpr (POST) {
        int j0, j1;
        interp_axis<T>(y, Lc.n[1], j0, j1, r.v0, r.v1);
        const auto ev = gin(e);
        const long long r0 = (long long)j0 * Lc.n[0], r1 = (long long)j1 * Lc.n[0];
        r.e00 = ev[r0 + ix.i0];
        r.e01 = ev[r0 + ix.i1];
        r.e10 = ev[r1 + ix.i0];
        r.e11 = ev[r1 + ix.i1];
    }
    if (u) r.u = gin(u)[gi];
    if constexpr (Q0BUF)
        r.f = cvt<TQ>(gin(static_cast<const cx<T>*>(f))[gi]);
    else
        r.f = gin(static_cast<const cx<TQ>*>(f))[gi];
    r.k2 = L.k2[gi];
}

template <typename T, typename TQ>
__device__ __forceinline__ cx<T> u2_of(const RowIn<T, TQ>& r, const InterpX<T>& ix) {
    return r.u + (r.v0 * ix.w0) * r.e00 + (r.v0 * ix.w1) * r.e01 + (r.v1 * ix.w0) * r.e10 + (r.v1 * ix.w1) * r.e11;
}

// ---------------------------------------------------------------------------
// Gram pass.  Step t takes row t of the first stage and produces, of the
// chain S0 -> S1 -> ..., row t - k of stage k; the Gram products are taken
// at the row where the last power is formed.
// ---------------------------------------------------------------------------
template <typename T, typename TQ, bool POST, int TY>
__global__ void __launch_bounds__(MW) k_mg_gram(const CycleArgs a, cx<double>* part, int pstride, int bstride) {
    const int pid = xcd_remap(blockIdx.x, gridDim.x);
    const int slot = find_slot(a.st.s, a.st.n, pid);
    const CycleSlot& sl = a.st.s[slot];
    if (gated_off(sl.gate)) return;
    const int tile = pid - sl.tile0;
    const LevelView<T>* Lp = static_cast<const LevelView<T>*>(sl.lv);
    const GLevel<T> L = glevel(*Lp);
    const GLevel<T> Lc = glevel(Lp[1]);
    const SmoothBufs B = *sl.sb;
    const int nx = L.n[0];
    const int ntx = (nx + MTX - 1) / MTX;
    const int x0 = (tile % ntx) * MTX, y0 = (tile / ntx) * TY;
    const Lane<T> c = lane_of(L, x0);
    InterpX<T> ix;
    interp_axis<T>(c.colv ? c.gx : 0, Lc.n[0], ix.i0, ix.i1, ix.w0, ix.w1);
    const T fs = (T)fscale_of(sl);
    const cx<T> Z = mk<T>(0, 0);
    cx<double> g[NUM_GRAM];
#pragma unroll
    for (int v = 0; v < NUM_GRAM; ++v) g[v] = mk(0.0, 0.0);
    const int yend = imin(y0 + TY, L.n[1]);

    if constexpr (POST) {
        const cx<T>* u1 = static_cast<const cx<T>*>(B.u1);
        const cx<T>* e = static_cast<const cx<T>*>(sl.c);
        // u2 rows t, t-1, t-2; q0 rows t-1..t-4; q1 rows t-2..t-4; q2 rows t-3..t-5
        cx<T> a0 = Z, a1 = Z, a2 = Z;
        cx<T> b1 = Z, b2 = Z, b3 = Z, b4 = Z;
        cx<T> c2 = Z, c3 = Z, c4 = Z;
        cx<T> d3 = Z, d4 = Z, d5 = Z;
        cx<T> fprev = Z;
        T k0 = 0, k1 = 0, kk2 = 0, k3 = 0, k4 = 0;   // k^2 at rows t..t-4
        RowIn<T, TQ> cur, n1, n2;
        load_row<T, TQ, true, false>(cur, L, Lc, c, ix, u1, e, sl.f, y0 - 4);
        load_row<T, TQ, true, false>(n1, L, Lc, c, ix, u1, e, sl.f, y0 - 3);
        for (int t = y0 - 4; t < yend + 4; ++t) {
            load_row<T, TQ, true, false>(n2, L, Lc, c, ix, u1, e, sl.f, t + 2);
            a2 = a1;
            a1 = a0;
            a0 = u2_of(cur, ix);
            k4 = k3;
            k3 = kk2;
            kk2 = k1;
            k1 = k0;
            k0 = cur.k2;
            const bool m1 = c.colv && rowv(L, t - 1);
            cx<T> v = row_apply<T>(L, c, a2, a1, a0, t - 1, k1);
            b4 = b3;
            b3 = b2;
            b2 = b1;
            b1 = m1 ? fprev - v : Z;
            fprev = fs * cvt<T>(cur.f);
            v = row_apply<T>(L, c, b3, b2, b1, t - 2, kk2);
            c4 = c3;
            c3 = c2;
            c2 = (c.colv && rowv(L, t - 2)) ? L.sinv * v : Z;
            v = row_apply<T>(L, c, c4, c3, c2, t - 3, k3);
            d5 = d4;
            d4 = d3;
            d3 = (c.colv && rowv(L, t - 3)) ? L.sinv * v : Z;
            v = row_apply<T>(L, c, d5, d4, d3, t - 4, k4);
            const int yr = t - 4;
            if (c.own && yr >= y0 && yr < yend) gram_add<T>(g, b4, c4, d4, L.sinv * v);
            cur = n1;
            n1 = n2;
        }
    } else {
        // q0 rows t..t-3; q1 rows t-1..t-3; q2 rows t-2..t-4
        const bool q0buf = sl.f == nullptr;
        const void* src = q0buf ? B.q[0] : sl.f;
        const T qs = q0buf ? T(1) : fs;
        cx<T> a0 = Z, a1 = Z, a2 = Z, a3 = Z;
        cx<T> b1 = Z, b2 = Z, b3 = Z;
        cx<T> c2 = Z, c3 = Z, c4 = Z;
        T k0 = 0, k1 = 0, kk2 = 0, k3 = 0;
        RowIn<T, TQ> cur, n1, n2;
        auto ld = [&](RowIn<T, TQ>& r, int y) {
            if (q0buf)
                load_row<T, TQ, false, true>(r, L, Lc, c, ix, nullptr, nullptr, src, y);
            else
                load_row<T, TQ, false, false>(r, L, Lc, c, ix, nullptr, nullptr, src, y);
        };
        ld(cur, y0 - 3);
        ld(n1, y0 - 2);
        for (int t = y0 - 3; t < yend + 3; ++t) {
            ld(n2, t + 2);
            a3 = a2;
            a2 = a1;
            a1 = a0;
            a0 = qs * cvt<T>(cur.f);
            k3 = kk2;
            kk2 = k1;
            k1 = k0;
            k0 = cur.k2;
            cx<T> v = row_apply<T>(L, c, a2, a1, a0, t - 1, k1);
            b3 = b2;
            b2 = b1;
            b1 = (c.colv && rowv(L, t - 1)) ? L.sinv * v : Z;
            v = row_apply<T>(L, c, b3, b2, b1, t - 2, kk2);
            c4 = c3;
            c3 = c2;
            c2 = (c.colv && rowv(L, t - 2)) ? L.sinv * v : Z;
            v = row_apply<T>(L, c, c4, c3, c2, t - 3, k3);
            const int yr = t - 3;
            if (c.own && yr >= y0 && yr < yend) gram_add<T>(g, a3, b3, c3, L.sinv * v);
            cur = n1;
            n1 = n2;
        }
    }
    cx<double>* P = part + (long long)slot * pstride * bstride;
#pragma unroll
    for (int v = 0; v < NUM_GRAM; ++v) {
        const double r = wave_sum(g[v].r);
        const double i = wave_sum(g[v].i);
        if (threadIdx.x == 0) P[(long long)v * bstride + tile] = mk(r, i);
    }
}

// ---------------------------------------------------------------------------
// Pre-smoothing apply + restriction.  Powers as in the Gram pass; r1 and u1
// at row t - 3; the coarse row whose centre is row t - 4 is restricted once
// rows t-5..t-3 of r1 exist.
// ---------------------------------------------------------------------------
template <typename T, typename TQ, bool NZ, int TY>
__global__ void __launch_bounds__(MW) k_mg_apply_restrict(const CycleArgs a) {
    const int pid = xcd_remap(blockIdx.x, gridDim.x);
    const int slot = find_slot(a.st.s, a.st.n, pid);
    const CycleSlot& sl = a.st.s[slot];
    if (gated_off(sl.gate)) return;
    const LevelView<T>* Lp = static_cast<const LevelView<T>*>(sl.lv);
    const GLevel<T> L = glevel(*Lp);
    const GLevel<T> Lc = glevel(Lp[1]);
    const SmoothBufs B = *sl.sb;
    const int nx = L.n[0], ny = L.n[1];
    const int ntx = (nx + MTX - 1) / MTX;
    const int tile = pid - sl.tile0;
    const int x0 = (tile % ntx) * MTX, y0 = (tile / ntx) * TY;
    const Lane<T> c = lane_of(L, x0);
    InterpX<T> ix;
    ix.i0 = ix.i1 = 0;
    ix.w0 = ix.w1 = T(0);
    const T fs = (T)fscale_of(sl);
    const bool q0buf = sl.f == nullptr;
    const void* src = q0buf ? B.q[0] : sl.f;
    const T qs = q0buf ? T(1) : fs;
    const cx<T>* up = static_cast<const cx<T>*>(sl.u);
    const auto u1p = gout(static_cast<cx<T>*>(B.u1));
    const auto fc = gout(static_cast<cx<T>*>(sl.c));
    const int ncx = Lc.n[0], ncy = Lc.n[1];
    const cx<T> c1 = cvt<T>(B.coef[0]), cc2 = cvt<T>(B.coef[1]), cc3 = cvt<T>(B.coef[2]);
    const cx<T> Z = mk<T>(0, 0);
    const int yend = imin(y0 + TY, ny);
    // restriction centres of this strip: odd gx among the owned lanes
    const bool ccol = c.own && (c.gx & 1) && (c.gx - 1) / 2 < ncx;

    cx<T> a0 = Z, a1 = Z, a2 = Z, a3 = Z;
    cx<T> b1 = Z, b2 = Z, b3 = Z;
    cx<T> c2 = Z, c3 = Z, c4 = Z;
    cx<T> r3 = Z, r4 = Z, r5 = Z;   // r1 at rows t-3, t-4, t-5
    cx<T> w0 = Z, w1 = Z, w2 = Z, w3 = Z;   // incoming iterate at rows t..t-3 (NZ)
    T k0 = 0, k1 = 0, kk2 = 0, k3 = 0;
    RowIn<T, TQ> cur, n1;
    auto ld = [&](RowIn<T, TQ>& r, int y) {
        if (q0buf)
            load_row<T, TQ, false, true>(r, L, Lc, c, ix, NZ ? up : nullptr, nullptr, src, y);
        else
            load_row<T, TQ, false, false>(r, L, Lc, c, ix, NZ ? up : nullptr, nullptr, src, y);
    };
    ld(cur, y0 - 3);
    for (int t = y0 - 3; t <= yend + 3; ++t) {
        ld(n1, t + 1);
        a3 = a2;
        a2 = a1;
        a1 = a0;
        a0 = qs * cvt<T>(cur.f);
        if constexpr (NZ) {
            w3 = w2;
            w2 = w1;
            w1 = w0;
            w0 = cur.u;
        }
        k3 = kk2;
        kk2 = k1;
        k1 = k0;
        k0 = cur.k2;
        cx<T> v = row_apply<T>(L, c, a2, a1, a0, t - 1, k1);
        b3 = b2;
        b2 = b1;
        b1 = (c.colv && rowv(L, t - 1)) ? L.sinv * v : Z;
        v = row_apply<T>(L, c, b3, b2, b1, t - 2, kk2);
        c4 = c3;
        c3 = c2;
        c2 = (c.colv && rowv(L, t - 2)) ? L.sinv * v : Z;
        v = row_apply<T>(L, c, c4, c3, c2, t - 3, k3);
        const int yr = t - 3;
        const bool m3 = c.colv && rowv(L, yr);
        const cx<T> q3 = m3 ? L.sinv * v : Z;
        r5 = r4;
        r4 = r3;
        r3 = m3 ? a3 + c1 * b3 + cc2 * c3 + cc3 * q3 : Z;
        if (c.own && yr >= y0 && yr < yend) {
            cx<T> u = L.sinv * (c1 * a3 + cc2 * b3 + cc3 * c3);
            if constexpr (NZ) u = w3 - u;
            else u = Z - u;
            u1p[(long long)yr * nx + c.gx] = u;
        }
        const int yc = yr - 1;
        const cx<T> vv = T(0.25) * r5 + T(0.5) * r4 + T(0.25) * r3;
        const cx<T> vl = shfl_up1(vv), vr = shfl_dn1(vv);
        if ((yc & 1) && yc >= y0 && yc < yend && (yc - 1) / 2 < ncy && ccol) {
            const int C = (yc - 1) / 2, Cx = (c.gx - 1) / 2;
            fc[(long long)C * ncx + Cx] = T(0.25) * vl + T(0.5) * vv + T(0.25) * vr;
        }
        cur = n1;
    }
}

// ---------------------------------------------------------------------------
// Post-smoothing apply: u2 rows t..t-3, q0 rows t-1..t-3, q1 rows t-2..t-4,
// q2 at row t-3; out at row t - 3.
// ---------------------------------------------------------------------------
template <typename T, typename TF, typename TO, bool ACC, int TY>
__global__ void __launch_bounds__(MW) k_mg_apply_out(const CycleArgs a) {
    const int pid = xcd_remap(blockIdx.x, gridDim.x);
    const int slot = find_slot(a.st.s, a.st.n, pid);
    const CycleSlot& sl = a.st.s[slot];
    if (gated_off(sl.gate)) return;
    const LevelView<T>* Lp = static_cast<const LevelView<T>*>(sl.lv);
    const GLevel<T> L = glevel(*Lp);
    const GLevel<T> Lc = glevel(Lp[1]);
    const SmoothBufs B = *sl.sb;
    const int nx = L.n[0], ny = L.n[1];
    const int ntx = (nx + MTX - 1) / MTX;
    const int tile = pid - sl.tile0;
    const int x0 = (tile % ntx) * MTX, y0 = (tile / ntx) * TY;
    const Lane<T> c = lane_of(L, x0);
    InterpX<T> ix;
    interp_axis<T>(c.colv ? c.gx : 0, Lc.n[0], ix.i0, ix.i1, ix.w0, ix.w1);
    const T fs = (T)fscale_of(sl);
    const cx<T>* u1 = static_cast<const cx<T>*>(B.u1);
    const cx<T>* e = static_cast<const cx<T>*>(sl.c);
    const auto out = gout(static_cast<cx<TO>*>(sl.out));
    const cx<T> c1 = cvt<T>(B.coef[4]), cc2 = cvt<T>(B.coef[5]), cc3 = cvt<T>(B.coef[6]);
    const cx<T> Z = mk<T>(0, 0);
    const int yend = imin(y0 + TY, ny);

    cx<T> a0 = Z, a1 = Z, a2 = Z, a3 = Z;
    cx<T> b1 = Z, b2 = Z, b3 = Z;
    cx<T> c2 = Z, c3 = Z, c4 = Z;
    cx<T> fprev = Z;
    T k0 = 0, k1 = 0, kk2 = 0, k3 = 0;
    RowIn<T, TF> cur, n1;
    load_row<T, TF, true, false>(cur, L, Lc, c, ix, u1, e, sl.f, y0 - 3);
    for (int t = y0 - 3; t < yend + 3; ++t) {
        load_row<T, TF, true, false>(n1, L, Lc, c, ix, u1, e, sl.f, t + 1);
        a3 = a2;
        a2 = a1;
        a1 = a0;
        a0 = u2_of(cur, ix);
        k3 = kk2;
        kk2 = k1;
        k1 = k0;
        k0 = cur.k2;
        const bool m1 = c.colv && rowv(L, t - 1);
        cx<T> v = row_apply<T>(L, c, a2, a1, a0, t - 1, k1);
        b3 = b2;
        b2 = b1;
        b1 = m1 ? fprev - v : Z;
        fprev = fs * cvt<T>(cur.f);
        v = row_apply<T>(L, c, b3, b2, b1, t - 2, kk2);
        c4 = c3;
        c3 = c2;
        c2 = (c.colv && rowv(L, t - 2)) ? L.sinv * v : Z;
        v = row_apply<T>(L, c, c4, c3, c2, t - 3, k3);
        const int yr = t - 3;
        if (c.own && yr >= y0 && yr < yend) {
            const long long gi = (long long)yr * nx + c.gx;
            const cx<T> q2 = L.sinv * v;
            const cx<T> w = a3 - L.sinv * (c1 * b3 + cc2 * c3 + cc3 * q2);
            if constexpr (ACC)
                out[gi] = out[gi].get() + cvt<TO>(w);
            else
                out[gi] = cvt<TO>(w);
        }
        cur = n1;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Geometry and launchers
// ---------------------------------------------------------------------------
namespace {
constexpr int MARCH_TY[NUM_TILE_SHAPES] = {32, 16, 8};
}

void march_counts(int shape, const int n[3], int nt[3]) {
    if (shape < 0 || shape >= NUM_TILE_SHAPES) shape = 0;
    nt[0] = (n[0] + MTX - 1) / MTX;
    nt[1] = (n[1] + MARCH_TY[shape] - 1) / MARCH_TY[shape];
    nt[2] = 1;
}

#define MG_MARCH_SWITCH(LAUNCH)         \
    switch (shape) {                    \
        case 1: LAUNCH(16); break;      \
        case 2: LAUNCH(8); break;       \
        default: LAUNCH(32); break;     \
    }

template <typename T, typename TQ, bool POST>
static hipError_t mg_gram_launch(int shape, const CycleArgs& a, cx<double>* part, int pstride, int bstride,
                                 hipStream_t s) {
#define GL(TY) \
    hipLaunchKernelGGL((k_mg_gram<T, TQ, POST, TY>), dim3(a.st.ntiles), dim3(MW), 0, s, a, part, pstride, bstride);
    MG_MARCH_SWITCH(GL)
#undef GL
    return hipGetLastError();
}

hipError_t launch_sm2_gram(bool f32, bool level0, bool post, int shape, const CycleArgs& a, cx<double>* part,
                           int pstride, int bstride, hipStream_t s) {
    if (a.st.n <= 0) return hipSuccess;
    if (!f32)
        return post ? mg_gram_launch<double, double, true>(shape, a, part, pstride, bstride, s)
                    : mg_gram_launch<double, double, false>(shape, a, part, pstride, bstride, s);
    if (level0)
        return post ? mg_gram_launch<float, double, true>(shape, a, part, pstride, bstride, s)
                    : mg_gram_launch<float, double, false>(shape, a, part, pstride, bstride, s);
    return post ? mg_gram_launch<float, float, true>(shape, a, part, pstride, bstride, s)
                : mg_gram_launch<float, float, false>(shape, a, part, pstride, bstride, s);
}

template <typename T, typename TQ, bool NZ>
static hipError_t mg_ar_launch(int shape, const CycleArgs& a, hipStream_t s) {
#define AL(TY) hipLaunchKernelGGL((k_mg_apply_restrict<T, TQ, NZ, TY>), dim3(a.st.ntiles), dim3(MW), 0, s, a);
    MG_MARCH_SWITCH(AL)
#undef AL
    return hipGetLastError();
}

hipError_t launch_sm2_apply_restrict(bool f32, bool level0, bool nonzero, int shape, const CycleArgs& a,
                                     hipStream_t s) {
    if (a.st.n <= 0) return hipSuccess;
    if (!f32)
        return nonzero ? mg_ar_launch<double, double, true>(shape, a, s) : mg_ar_launch<double, double, false>(shape, a, s);
    if (nonzero) return hipErrorInvalidValue;
    return level0 ? mg_ar_launch<float, double, false>(shape, a, s) : mg_ar_launch<float, float, false>(shape, a, s);
}

template <typename T, typename TF, typename TO, bool ACC>
static hipError_t mg_ao_launch(int shape, const CycleArgs& a, hipStream_t s) {
#define OL(TY) hipLaunchKernelGGL((k_mg_apply_out<T, TF, TO, ACC, TY>), dim3(a.st.ntiles), dim3(MW), 0, s, a);
    MG_MARCH_SWITCH(OL)
#undef OL
    return hipGetLastError();
}

hipError_t launch_sm2_apply_out(bool f32, bool level0, bool accumulate, int shape, const CycleArgs& a, hipStream_t s) {
    if (a.st.n <= 0) return hipSuccess;
    if (!f32)
        return accumulate ? mg_ao_launch<double, double, double, true>(shape, a, s)
                          : mg_ao_launch<double, double, double, false>(shape, a, s);
    if (level0)
        return accumulate ? mg_ao_launch<float, double, double, true>(shape, a, s)
                          : mg_ao_launch<float, double, double, false>(shape, a, s);
    return mg_ao_launch<float, float, float, false>(shape, a, s);
}

}  // namespace mg
