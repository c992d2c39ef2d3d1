// 2D GMRES(3) smoothing passes (Sec. 3.2.2) as LDS tiles, for the small
// coarse levels.
//
// The row-marching passes (mg_march2d.hip) stream a level through one
// wavefront per strip; on a small level the march itself -- a few owned rows
// after several warm-up rows, every row a dependent chain of stencils --
// sets the time.  Here a 256-thread workgroup owns a TTX x TTY tile, loads
// the tile and a halo of H points into LDS in one go, and forms the powers
// q1, q2, q3 on shrinking regions (halo H-1, H-2, ...), one barrier apart.
// The four passes compute what the marching ones compute (same stencil
// expression, same Gram products, same interpolation and full weighting;
// values outside the grid are zero at every stage):
//   k_tile_gram<PRE>      q0 = fscale f (or the q0 buffer), H = 3;
//   k_tile_gram<POST>     u2 = u1 + P e, q0 = fscale f - A u2, H = 4;
//                         Gram partials of q0..q3 per tile.
//   k_tile_apply_restrict q0..q3 (H = 4), u1 = u - (c1 q0 + c2 q1 + c3 q2)/s,
//                         r1 = q0 + sum_i c_i q_i on halo 1 and its
//                         full-weighting restriction.
//   k_tile_apply_out      u2, q0..q2 (H = 3), out = u2 - (c1 q0 + c2 q1 +
//                         c3 q2)/s.

#include <type_traits>

#include "mg_kcommon.hpp"

namespace mg {

using namespace kc;

namespace {

constexpr int TTX = 32, TTY = 16;   // owned points of a tile
constexpr int TNT = 256;            // threads per workgroup

// v where c holds, else 0 (component by component: a select of whole
// structures would go through scratch memory).
template <typename T>
__device__ __forceinline__ cx<T> keep(bool c, cx<T> v) {
    return mk<T>(c ? v.r : T(0), c ? v.i : T(0));
}

template <typename T>
__device__ __forceinline__ T keep(bool c, T v) {
    return c ? v : T(0);
}

template <int H>
struct TGeo {
    static constexpr int W = TTX + 2 * H;    // LDS row length; LDS (0, 0) is grid (x0 - H, y0 - H)
    static constexpr int HH = TTY + 2 * H;
    static constexpr int N = W * HH;
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Fills an LDS array laid out like the tile with value(gx, gy) at the grid
// points and 0 elsewhere.  A thread's points are unrolled and value() is
// evaluated at clamped coordinates for every one of them, so all their loads
// are in flight together (a load under a branch, or one per loop trip, would
// be waited for one at a time).
template <int H, typename V, typename F>
__device__ __forceinline__ void fill_tile(V* S, int gx0, int gy0, int nx, int ny, F&& value) {
    using G = TGeo<H>;
    constexpr int PER = (G::N + TNT - 1) / TNT;
    V v[PER];
    bool in[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int q = threadIdx.x + k * TNT;
        const int qq = q < G::N ? q : G::N - 1;
        const int gx = gx0 + qq % G::W, gy = gy0 + qq / G::W;
        in[k] = q < G::N && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
        v[k] = value(clampi(gx, 0, nx - 1), clampi(gy, 0, ny - 1));
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int q = threadIdx.x + k * TNT;
        if (q < G::N) S[q] = keep(in[k], v[k]);
    }
}

// Per-tile stencil coefficients in LDS: x tables per LDS column, y tables
// per LDS row (zero outside the grid), k^2 per point.
template <typename T, int H>
struct TCoef {
    cx<T> xm[TGeo<H>::W], x0[TGeo<H>::W], xp[TGeo<H>::W];
    cx<T> ym[TGeo<H>::HH], y0[TGeo<H>::HH], yp[TGeo<H>::HH];
    T k2[TGeo<H>::N];
};

template <typename T, int H>
__device__ __forceinline__ void load_coef(TCoef<T, H>& C, const GLevel<T>& L, int gx0, int gy0) {
    using G = TGeo<H>;
    const cx<T> Z = mk<T>(0, 0);
    for (int i = threadIdx.x; i < G::W; i += TNT) {
        const int gx = gx0 + i;
        const bool in = gx >= 0 && gx < L.n[0];
        const int g = in ? gx : 0;
        const cx<T> m = L.cm[0][g], c = L.c0[0][g], p = L.cp[0][g];
        C.xm[i] = keep(in, m);
        C.x0[i] = keep(in, c);
        C.xp[i] = keep(in, p);
    }
    for (int j = threadIdx.x; j < G::HH; j += TNT) {
        const int gy = gy0 + j;
        const bool in = gy >= 0 && gy < L.n[1];
        const int g = in ? gy : 0;
        const cx<T> m = L.cm[1][g], c = L.c0[1][g], p = L.cp[1][g];
        C.ym[j] = keep(in, m);
        C.y0[j] = keep(in, c);
        C.yp[j] = keep(in, p);
    }
    const int nx = L.n[0];
    fill_tile<H>(C.k2, gx0, gy0, L.n[0], L.n[1], [&](int gx, int gy) { return L.k2[(long long)gy * nx + gx]; });
}

// A x at LDS point (i, j) of an array laid out like the tile (the same terms
// in the same order as the marching passes).
template <typename T, int H>
__device__ __forceinline__ cx<T> tile_apply(const TCoef<T, H>& C, const GLevel<T>& L, const cx<T>* x, int i, int j) {
    using G = TGeo<H>;
    const int q = j * G::W + i;
    const cx<T> d = C.x0[i] + C.y0[j] - C.k2[q] * L.sigma;
    return cfma(C.yp[j], x[q + G::W],
                cfma(C.ym[j], x[q - G::W], cfma(C.xp[i], x[q + 1], cfma(C.xm[i], x[q - 1], d * x[q]))));
}

template <typename T>
__device__ __forceinline__ void gram_add(cx<double>* g, cx<T> a0, cx<T> a1, cx<T> a2, cx<T> a3) {
    const cx<double> v0 = cvt<double>(a0), v1 = cvt<double>(a1), v2 = cvt<double>(a2), v3 = cvt<double>(a3);
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

// (P e) at grid point (gx, gy): the coarse row(s) interpolated in x, then in
// y, as the marching passes form it.
template <typename T>
__device__ __forceinline__ cx<T> prolong_pt(const GLevel<T>& Lc, GIn<cx<T>> e, int gx, int gy) {
    int i0, i1;
    T w0, w1;
    interp_axis<T>(gx, Lc.n[0], i0, i1, w0, w1);
    auto ex = [&](int J) -> cx<T> {   // loads at a clamped row, masked after
        const long long b = (long long)clampi(J, 0, Lc.n[1] - 1) * Lc.n[0];
        return keep(J >= 0 && J < Lc.n[1], w0 * e[b + i0] + w1 * e[b + i1]);
    };
    const int J = gy >> 1;
    const cx<T> a = ex(J - 1), b = ex(J);
    return (gy & 1) ? b : T(0.5) * (a + b);
}

// Fixed-order sum of the workgroup's Gram partials into the launch's
// partial array (value v of tile at P[v * bstride + tile]).
__device__ __forceinline__ void gram_store(cx<double>* g, cx<double>* sred, cx<double>* P, int bstride, int tile) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < NUM_GRAM; ++v) {
        const double r = wave_sum(g[v].r), i = v < 4 ? 0.0 : wave_sum(g[v].i);
        if (lane == 0) sred[wave * NUM_GRAM + v] = mk(r, i);
    }
    __syncthreads();
    if ((int)threadIdx.x < NUM_GRAM) {
        cx<double> s = mk(0.0, 0.0);
#pragma unroll
        for (int w = 0; w < TNT / 64; ++w) s = s + sred[w * NUM_GRAM + threadIdx.x];
        P[(long long)threadIdx.x * bstride + tile] = s;
    }
}

template <typename T, typename TQ>
__device__ __forceinline__ GIn<cx<TQ>> q0_source(const CycleSlot& sl, const SmoothBufs& B) {
    if constexpr (std::is_same<T, TQ>::value)
        return gin(static_cast<const cx<TQ>*>(sl.f ? sl.f : B.q[0]));
    else
        return gin(static_cast<const cx<TQ>*>(sl.f));
}

// ---------------------------------------------------------------------------
// Gram pass
// ---------------------------------------------------------------------------
template <typename T, typename TQ, bool POST>
__global__ void __launch_bounds__(TNT) k_tile_gram(const CycleArgs a, cx<double>* part, int pstride, int bstride) {
    constexpr int H = POST ? 4 : 3;
    using G = TGeo<H>;
    __shared__ TCoef<T, H> C;
    __shared__ cx<T> S0[G::N], S1[G::N], S2[G::N], S3[POST ? G::N : 1];
    __shared__ cx<double> sred[(TNT / 64) * NUM_GRAM];
    const int pid = xcd_remap(blockIdx.x, gridDim.x);
    const int slot = find_slot(a.st.s, a.st.n, pid);
    const CycleSlot& sl = a.st.s[slot];
    if (gated_off(sl.gate)) return;
    const int tile = pid - sl.tile0;
    const LevelView<T>* Lp = static_cast<const LevelView<T>*>(sl.lv);
    const GLevel<T> L = glevel(*Lp);
    const GLevel<T> Lc = glevel(Lp[1]);
    const SmoothBufs B = *sl.sb;
    const int nx = L.n[0], ny = L.n[1];
    const int ntx = (nx + TTX - 1) / TTX;
    const int x0 = (tile % ntx) * TTX, y0 = (tile / ntx) * TTY;
    const int gx0 = x0 - H, gy0 = y0 - H;
    const T fs = (T)fscale_of(sl);
    const cx<T> Z = mk<T>(0, 0);
    auto ingrid = [&](int i, int j) {
        const int gx = gx0 + i, gy = gy0 + j;
        return gx >= 0 && gx < nx && gy >= 0 && gy < ny;
    };
    load_coef<T, H>(C, L, gx0, gy0);
    // first stage on the whole tile: u2 (POST) or q0
    cx<T>* X0 = POST ? S3 : S0;
    if constexpr (POST) {
        const auto u1 = gin(static_cast<const cx<T>*>(B.u1));
        const auto ev = gin(static_cast<const cx<T>*>(sl.c));
        fill_tile<H>(X0, gx0, gy0, nx, ny,
                     [&](int gx, int gy) { return u1[(long long)gy * nx + gx] + prolong_pt<T>(Lc, ev, gx, gy); });
    } else {
        const GIn<cx<TQ>> src = q0_source<T, TQ>(sl, B);
        const T qs = sl.f ? fs : T(1);
        fill_tile<H>(X0, gx0, gy0, nx, ny, [&](int gx, int gy) { return qs * cvt<T>(src[(long long)gy * nx + gx]); });
    }
    __syncthreads();
    // stages on shrinking regions: points (i, j) with h <= i < W - h, h <= j < HH - h
    auto stage = [&](int h, auto&& fn) {
        const int w = G::W - 2 * h, n = w * (G::HH - 2 * h);
        for (int q = threadIdx.x; q < n; q += TNT) fn(h + q % w, h + q / w);
    };
    if constexpr (POST) {
        const auto fv = gin(static_cast<const cx<TQ>*>(sl.f));
        stage(1, [&](int i, int j) {   // q0 = fscale f - A u2
            const int q = j * G::W + i;
            cx<T> v = Z;
            if (ingrid(i, j)) {
                const cx<T> fq = fs * cvt<T>(fv[(long long)(gy0 + j) * nx + gx0 + i]);
                v = fq - tile_apply<T, H>(C, L, X0, i, j);
            }
            S0[q] = v;
        });
        __syncthreads();
    }
    stage(H - 2, [&](int i, int j) {
        const int q = j * G::W + i;
        S1[q] = keep(ingrid(i, j), L.sinv * tile_apply<T, H>(C, L, S0, i, j));
    });
    __syncthreads();
    stage(H - 1, [&](int i, int j) {
        const int q = j * G::W + i;
        S2[q] = keep(ingrid(i, j), L.sinv * tile_apply<T, H>(C, L, S1, i, j));
    });
    __syncthreads();
    cx<double> g[NUM_GRAM];
#pragma unroll
    for (int v = 0; v < NUM_GRAM; ++v) g[v] = mk(0.0, 0.0);
    stage(H, [&](int i, int j) {
        if (ingrid(i, j)) {
            const int q = j * G::W + i;
            gram_add<T>(g, S0[q], S1[q], S2[q], L.sinv * tile_apply<T, H>(C, L, S2, i, j));
        }
    });
    gram_store(g, sred, part + (long long)slot * pstride * bstride, bstride, tile);
}

// ---------------------------------------------------------------------------
// Pre-smoothing apply + restriction
// ---------------------------------------------------------------------------
template <typename T, typename TQ, bool NZ>
__global__ void __launch_bounds__(TNT) k_tile_apply_restrict(const CycleArgs a) {
    constexpr int H = 4;
    using G = TGeo<H>;
    __shared__ TCoef<T, H> C;
    __shared__ cx<T> S0[G::N], S1[G::N], S2[G::N];
    const int pid = xcd_remap(blockIdx.x, gridDim.x);
    const int slot = find_slot(a.st.s, a.st.n, pid);
    const CycleSlot& sl = a.st.s[slot];
    if (gated_off(sl.gate)) return;
    const int tile = pid - sl.tile0;
    const LevelView<T>* Lp = static_cast<const LevelView<T>*>(sl.lv);
    const GLevel<T> L = glevel(*Lp);
    const GLevel<T> Lc = glevel(Lp[1]);
    const SmoothBufs B = *sl.sb;
    const int nx = L.n[0], ny = L.n[1];
    const int ntx = (nx + TTX - 1) / TTX;
    const int x0 = (tile % ntx) * TTX, y0 = (tile / ntx) * TTY;
    const int gx0 = x0 - H, gy0 = y0 - H;
    const T fs = (T)fscale_of(sl);
    const GIn<cx<TQ>> src = q0_source<T, TQ>(sl, B);
    const T qs = sl.f ? fs : T(1);
    const auto up = gin(static_cast<const cx<T>*>(sl.u));
    const auto u1p = gout(static_cast<cx<T>*>(B.u1));
    const auto fc = gout(static_cast<cx<T>*>(sl.c));
    // coefficients: from the Gram partials (their loads in flight with the
    // tile's), else from the coefficient record
    const bool fused = a.gpart && slot_tiles(a, slot) <= FUSED_COEF_TILES;
    CoefLoad cl;
    if (fused) coef_load(a, slot, cl);
    cx<T> c1 = cvt<T>(B.coef[0]), cc2 = cvt<T>(B.coef[1]), cc3 = cvt<T>(B.coef[2]);
    const cx<T> Z = mk<T>(0, 0);
    auto ingrid = [&](int i, int j) {
        const int gx = gx0 + i, gy = gy0 + j;
        return gx >= 0 && gx < nx && gy >= 0 && gy < ny;
    };
    load_coef<T, H>(C, L, gx0, gy0);
    fill_tile<H>(S0, gx0, gy0, nx, ny, [&](int gx, int gy) { return qs * cvt<T>(src[(long long)gy * nx + gx]); });
    __syncthreads();
    if (fused) {
        cx<double> co[4];
        coef_solve(cl, a.gbrk, co);
        c1 = cvt<T>(co[0]), cc2 = cvt<T>(co[1]), cc3 = cvt<T>(co[2]);
    }
    auto stage = [&](int h, auto&& fn) {
        const int w = G::W - 2 * h, n = w * (G::HH - 2 * h);
        for (int q = threadIdx.x; q < n; q += TNT) fn(h + q % w, h + q / w);
    };
    stage(1, [&](int i, int j) {
        const int q = j * G::W + i;
        S1[q] = keep(ingrid(i, j), L.sinv * tile_apply<T, H>(C, L, S0, i, j));
    });
    __syncthreads();
    stage(2, [&](int i, int j) {
        const int q = j * G::W + i;
        S2[q] = keep(ingrid(i, j), L.sinv * tile_apply<T, H>(C, L, S1, i, j));
    });
    __syncthreads();
    // halo 1: q3, r1 (into S0, read only at its own point here), and u1 on
    // the owned points
    stage(3, [&](int i, int j) {
        const int q = j * G::W + i;
        const bool in = ingrid(i, j);
        const cx<T> q0 = S0[q], q1 = S1[q], q2 = S2[q];
        const cx<T> q3 = keep(in, L.sinv * tile_apply<T, H>(C, L, S2, i, j));
        const bool own = in && i >= H && i < H + TTX && j >= H && j < H + TTY;
        if (own) {
            const long long gi = (long long)(gy0 + j) * nx + gx0 + i;
            cx<T> u = L.sinv * cfma(cc3, q2, cfma(cc2, q1, c1 * q0));
            if constexpr (NZ) u = up[gi] - u;
            else u = Z - u;
            u1p[gi] = u;
        }
        S0[q] = keep(in, cfma(cc3, q3, cfma(cc2, q2, cfma(c1, q1, q0))));
    });
    __syncthreads();
    // coarse points whose centre (2C + 1) lies on the tile's owned points
    const int ncx = Lc.n[0], ncy = Lc.n[1];
    for (int q = threadIdx.x; q < (TTX / 2) * (TTY / 2); q += TNT) {
        const int cxl = q % (TTX / 2), cyl = q / (TTX / 2);
        const int Cx = x0 / 2 + cxl, Cy = y0 / 2 + cyl;
        if (Cx >= ncx || Cy >= ncy) continue;
        const int i = 2 * Cx + 1 - gx0, j = 2 * Cy + 1 - gy0;
        cx<T> col[3];
#pragma unroll
        for (int o = -1; o <= 1; ++o) {
            const int qq = j * G::W + i + o;
            col[o + 1] = T(0.25) * S0[qq - G::W] + T(0.5) * S0[qq] + T(0.25) * S0[qq + G::W];
        }
        fc[(long long)Cy * ncx + Cx] = T(0.25) * col[0] + T(0.5) * col[1] + T(0.25) * col[2];
    }
}

// ---------------------------------------------------------------------------
// Post-smoothing apply
// ---------------------------------------------------------------------------
template <typename T, typename TF, typename TO, bool ACC>
__global__ void __launch_bounds__(TNT) k_tile_apply_out(const CycleArgs a) {
    constexpr int H = 3;
    using G = TGeo<H>;
    __shared__ TCoef<T, H> C;
    __shared__ cx<T> S0[G::N], S1[G::N], S2[G::N];
    const int pid = xcd_remap(blockIdx.x, gridDim.x);
    const int slot = find_slot(a.st.s, a.st.n, pid);
    const CycleSlot& sl = a.st.s[slot];
    if (gated_off(sl.gate)) return;
    const int tile = pid - sl.tile0;
    const LevelView<T>* Lp = static_cast<const LevelView<T>*>(sl.lv);
    const GLevel<T> L = glevel(*Lp);
    const GLevel<T> Lc = glevel(Lp[1]);
    const SmoothBufs B = *sl.sb;
    const int nx = L.n[0], ny = L.n[1];
    const int ntx = (nx + TTX - 1) / TTX;
    const int x0 = (tile % ntx) * TTX, y0 = (tile / ntx) * TTY;
    const int gx0 = x0 - H, gy0 = y0 - H;
    const T fs = (T)fscale_of(sl);
    const auto u1 = gin(static_cast<const cx<T>*>(B.u1));
    const auto ev = gin(static_cast<const cx<T>*>(sl.c));
    const auto fv = gin(static_cast<const cx<TF>*>(sl.f));
    const auto out = gout(static_cast<cx<TO>*>(sl.out));
    // coefficients: from the Gram partials (their loads in flight with the
    // tile's), else from the coefficient record
    const bool fused = a.gpart && slot_tiles(a, slot) <= FUSED_COEF_TILES;
    CoefLoad cl;
    if (fused) coef_load(a, slot, cl);
    cx<T> c1 = cvt<T>(B.coef[4]), cc2 = cvt<T>(B.coef[5]), cc3 = cvt<T>(B.coef[6]);
    const cx<T> Z = mk<T>(0, 0);
    auto ingrid = [&](int i, int j) {
        const int gx = gx0 + i, gy = gy0 + j;
        return gx >= 0 && gx < nx && gy >= 0 && gy < ny;
    };
    load_coef<T, H>(C, L, gx0, gy0);
    fill_tile<H>(S0, gx0, gy0, nx, ny,   // u2
                 [&](int gx, int gy) { return u1[(long long)gy * nx + gx] + prolong_pt<T>(Lc, ev, gx, gy); });
    __syncthreads();
    if (fused) {
        cx<double> co[4];
        coef_solve(cl, a.gbrk, co);
        c1 = cvt<T>(co[0]), cc2 = cvt<T>(co[1]), cc3 = cvt<T>(co[2]);
    }
    auto stage = [&](int h, auto&& fn) {
        const int w = G::W - 2 * h, n = w * (G::HH - 2 * h);
        for (int q = threadIdx.x; q < n; q += TNT) fn(h + q % w, h + q / w);
    };
    stage(1, [&](int i, int j) {   // q0 = fscale f - A u2
        const int q = j * G::W + i;
        cx<T> v = Z;
        if (ingrid(i, j)) {
            const cx<T> fq = fs * cvt<T>(fv[(long long)(gy0 + j) * nx + gx0 + i]);
            v = fq - tile_apply<T, H>(C, L, S0, i, j);
        }
        S1[q] = v;
    });
    __syncthreads();
    stage(2, [&](int i, int j) {
        const int q = j * G::W + i;
        S2[q] = keep(ingrid(i, j), L.sinv * tile_apply<T, H>(C, L, S1, i, j));
    });
    __syncthreads();
    stage(3, [&](int i, int j) {
        if (!ingrid(i, j)) return;
        const int q = j * G::W + i;
        const long long gi = (long long)(gy0 + j) * nx + gx0 + i;
        const cx<T> q2 = L.sinv * tile_apply<T, H>(C, L, S2, i, j);
        const cx<T> w = S0[q] - L.sinv * cfma(cc3, q2, cfma(cc2, S2[q], c1 * S1[q]));
        if constexpr (ACC)
            out[gi] = out[gi].get() + cvt<TO>(w);
        else
            out[gi] = cvt<TO>(w);
    });
}

}  // namespace

void tile2d_counts(const int n[3], int nt[3]) {
    nt[0] = (n[0] + TTX - 1) / TTX;
    nt[1] = (n[1] + TTY - 1) / TTY;
    nt[2] = 1;
}

hipError_t tile2d_gram(bool f32, bool level0, bool post, const CycleArgs& a, cx<double>* part, int pstride,
                       int bstride, hipStream_t s) {
#define TG(T, TQ, P) \
    hipLaunchKernelGGL((k_tile_gram<T, TQ, P>), dim3(a.st.ntiles), dim3(TNT), 0, s, a, part, pstride, bstride)
    if (!f32) {
        if (post) TG(double, double, true);
        else TG(double, double, false);
    } else if (level0) {
        if (post) TG(float, double, true);
        else TG(float, double, false);
    } else {
        if (post) TG(float, float, true);
        else TG(float, float, false);
    }
#undef TG
    return hipGetLastError();
}

hipError_t tile2d_apply_restrict(bool f32, bool level0, bool nonzero, const CycleArgs& a, hipStream_t s) {
#define TA(T, TQ, NZ) hipLaunchKernelGGL((k_tile_apply_restrict<T, TQ, NZ>), dim3(a.st.ntiles), dim3(TNT), 0, s, a)
    if (!f32) {
        if (nonzero) TA(double, double, true);
        else TA(double, double, false);
    } else {
        if (nonzero) return hipErrorInvalidValue;
        if (level0) TA(float, double, false);
        else TA(float, float, false);
    }
#undef TA
    return hipGetLastError();
}

hipError_t tile2d_apply_out(bool f32, bool level0, bool accumulate, const CycleArgs& a, hipStream_t s) {
#define TO_(T, TF, TO, ACC) hipLaunchKernelGGL((k_tile_apply_out<T, TF, TO, ACC>), dim3(a.st.ntiles), dim3(TNT), 0, s, a)
    if (!f32) {
        if (accumulate) TO_(double, double, double, true);
        else TO_(double, double, double, false);
    } else if (level0) {
        if (accumulate) TO_(float, double, double, true);
        else TO_(float, double, double, false);
    } else {
        TO_(float, float, float, false);
    }
#undef TO_
    return hipGetLastError();
}

}  // namespace mg
