// Fused 2D GMRES(3) smoothing passes (Sec. 3.2.2) for gfx950.
//
// The minimiser of || q0 + c1 q1 + c2 q2 + c3 q3 ||, q_i = (A/s)^i r, is
// found from the Gram matrix of the q_i (see mg_smooth.hip).  In 2D every
// power is formed inside an LDS tile from the level's inputs, so one
// smoothing step reads each input twice and stores only what the cycle
// keeps:
//   k_sm2_gram    r (from f, or from u1 + P e after the coarse-grid
//                 correction) on the tile with a halo of 3, then q1, q2, q3
//                 on shrinking halos; Gram partials of q0..q3 per tile.
//   k_sm2_apply_restrict   the same powers on a wider halo, u1 = -(c1 q0 +
//                 c2 q1 + c3 q2)/s on the tile, r1 = q0 + sum_i c_i q_i on
//                 the tile plus the points the restriction reads, and the
//                 full-weighting restriction of r1 (pre-smoothing).
//   k_sm2_apply_out  u2 = u1 + P e and its powers, out = u2 - (c1 q0 + c2 q1
//                 + c3 q2)/s on the tile (post-smoothing).
// LDS holds two arrays of the tile plus halo H (ping-pong); the values of
// a power at a thread's own points that a later step still needs are kept in
// registers.  Points outside the grid hold zeros (Dirichlet ghosts), so every
// power obeys the level operator's boundary rows.

#include "mg_kcommon.hpp"

namespace mg {

using namespace kc;

namespace {

// Region geometry: arrays of (TX + 2H) x (TY + 2H), local point (lx, ly)
// relative to the tile origin, lx in [-H, TX + H).
template <int TX, int TY, int H>
struct Reg {
    static constexpr int X = TX + 2 * H;
    static constexpr int Y = TY + 2 * H;
    static constexpr int N = X * Y;
    __device__ static constexpr int at(int lx, int ly) { return (ly + H) * X + (lx + H); }
};

// Operator row at grid point (gx, gy) applied to an LDS array at index c.
template <typename T, int X>
__device__ __forceinline__ cx<T> lds_stencil(const LevelView<T>& L, const cx<T>* a, int c, int gx, int gy, T k2) {
    return diag_at<2>(L, gx, gy, 0, k2) * a[c] + L.cm[0][gx] * a[c - 1] + L.cp[0][gx] * a[c + 1] +
           L.cm[1][gy] * a[c - X] + L.cp[1][gy] * a[c + X];
}

// dst = (A/s) src on the local rectangle [lo, hi_x] x [lo, hi_y] (inclusive,
// relative to the tile), zero outside the grid.
template <typename T, int TX, int TY, int H>
__device__ __forceinline__ void power_step(const LevelView<T>& L, const cx<T>* src, cx<T>* dst, int x0, int y0, int lo,
                                           int hix, int hiy) {
    using R = Reg<TX, TY, H>;
    const int W = hix - lo + 1, Hh = hiy - lo + 1;
    const int nx = L.n[0], ny = L.n[1];
    for (int idx = threadIdx.x; idx < W * Hh; idx += NT) {
        const int lx = lo + idx % W, ly = lo + idx / W;
        const int gx = x0 + lx, gy = y0 + ly;
        cx<T> v = mk<T>(0, 0);
        if (gx >= 0 && gx < nx && gy >= 0 && gy < ny)
            v = L.sinv * lds_stencil<T, R::X>(L, src, R::at(lx, ly), gx, gy, L.k2[(long long)gy * nx + gx]);
        dst[R::at(lx, ly)] = v;
    }
}

// Coarse correction e on the coarse points that bilinear interpolation to the
// fine local rectangle [-h, TX + h) needs: coarse index range [x0/2 + elo,
// x0/2 + ehi] per axis.
template <int TX, int TY, int h>
struct CoarseWin {
    static constexpr int LO = -((h + 2) / 2);
    static constexpr int HIX = TX / 2 + ((h % 2 == 0) ? h / 2 - 1 : (h - 1) / 2);
    static constexpr int HIY = TY / 2 + ((h % 2 == 0) ? h / 2 - 1 : (h - 1) / 2);
    static constexpr int EX = HIX - LO + 1;
    static constexpr int EY = HIY - LO + 1;
    static constexpr int N = EX * EY;
};

// u2 = u1 + P e on the local rectangle [-h, T + h), zero outside the grid,
// into dst (region H >= h).
template <typename T, int TX, int TY, int H, int h>
__device__ __forceinline__ void correct_step(const LevelView<T>& L, const LevelView<T>& Lc, const cx<T>* u1,
                                             const cx<T>* ec, cx<T>* se, cx<T>* dst, int x0, int y0) {
    using R = Reg<TX, TY, H>;
    using E = CoarseWin<TX, TY, h>;
    const int ncx = Lc.n[0], ncy = Lc.n[1];
    const int cxs = x0 / 2 + E::LO, cys = y0 / 2 + E::LO;
    for (int idx = threadIdx.x; idx < E::N; idx += NT) {
        const int Cx = cxs + idx % E::EX, Cy = cys + idx / E::EX;
        cx<T> v = mk<T>(0, 0);
        if (Cx >= 0 && Cx < ncx && Cy >= 0 && Cy < ncy) v = ec[(long long)Cy * ncx + Cx];
        se[idx] = v;
    }
    __syncthreads();
    const int nx = L.n[0], ny = L.n[1];
    constexpr int W = TX + 2 * h, Hh = TY + 2 * h;
    for (int idx = threadIdx.x; idx < W * Hh; idx += NT) {
        const int lx = -h + idx % W, ly = -h + idx / W;
        const int gx = x0 + lx, gy = y0 + ly;
        cx<T> v = mk<T>(0, 0);
        if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) {
            int ix0, ix1, iy0, iy1;
            T wx0, wx1, wy0, wy1;
            interp_1d<T>(gx, cxs, ix0, ix1, wx0, wx1);
            interp_1d<T>(gy, cys, iy0, iy1, wy0, wy1);
            const cx<T> pe = (wy0 * wx0) * se[iy0 * E::EX + ix0] + (wy0 * wx1) * se[iy0 * E::EX + ix1] +
                             (wy1 * wx0) * se[iy1 * E::EX + ix0] + (wy1 * wx1) * se[iy1 * E::EX + ix1];
            v = u1[(long long)gy * nx + gx] + pe;
        }
        dst[R::at(lx, ly)] = v;
    }
}

// q0 on the local rectangle [-h, T + h): fs f (TQ) or the q0 buffer, or (RES)
// fs f - A src with src holding u2 on [-h-1, T+h]; zero outside the grid.
template <typename T, typename TQ, int TX, int TY, int H, int h, bool RES>
__device__ __forceinline__ void q0_step(const LevelView<T>& L, const void* f, T fs, const cx<T>* q0buf,
                                        const cx<T>* src, cx<T>* dst, int x0, int y0) {
    using R = Reg<TX, TY, H>;
    const int nx = L.n[0], ny = L.n[1];
    constexpr int W = TX + 2 * h, Hh = TY + 2 * h;
    for (int idx = threadIdx.x; idx < W * Hh; idx += NT) {
        const int lx = -h + idx % W, ly = -h + idx / W;
        const int gx = x0 + lx, gy = y0 + ly;
        cx<T> v = mk<T>(0, 0);
        if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) {
            const long long g = (long long)gy * nx + gx;
            if constexpr (RES) {
                v = fs * cvt<T>(static_cast<const cx<TQ>*>(f)[g]) -
                    lds_stencil<T, R::X>(L, src, R::at(lx, ly), gx, gy, L.k2[g]);
            } else {
                v = f ? fs * cvt<T>(static_cast<const cx<TQ>*>(f)[g]) : q0buf[g];
            }
        }
        dst[R::at(lx, ly)] = v;
    }
}

// Tile origin of a workgroup.
template <int TX, int TY>
__device__ __forceinline__ void origin(int tile, int nx, int& x0, int& y0) {
    const int ntx = (nx + TX - 1) / TX;
    x0 = (tile % ntx) * TX;
    y0 = (tile / ntx) * TY;
}

constexpr int ceil_div(int a, int b) { return (a + b - 1) / b; }

// Gram partials of the 10 products of (q0, q1, q2, q3) over the tile.
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

__device__ __forceinline__ void gram_store(cx<double>* g, cx<double>* sm, cx<double>* part, int pstride, int bstride,
                                           int slot, int tile) {
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
        part[((long long)slot * pstride + threadIdx.x) * bstride + tile] = s;
    }
}

// ---------------------------------------------------------------------------
// Gram pass.  POST = false: q0 = fscale f (or the q0 buffer when slot.f is
// null); POST = true: q0 = fscale f - A (u1 + P e).  Partials per tile at
// part[(slot * pstride + v) * bstride + tile].
// ---------------------------------------------------------------------------
template <typename T, typename TQ, bool POST, int TX, int TY>
__global__ void __launch_bounds__(NT) k_sm2_gram(const CycleArgs a, cx<double>* part, int pstride, int bstride) {
    constexpr int H = POST ? 4 : 3;
    using R = Reg<TX, TY, H>;
    using E = CoarseWin<TX, TY, 4>;
    constexpr int PT = ceil_div(TX * TY, NT);
    __shared__ cx<T> sa[R::N];
    __shared__ cx<T> sb[R::N];
    __shared__ cx<T> se[POST ? E::N : 1];
    __shared__ cx<double> sm[(NT / 64) * NUM_GRAM];

    const int pid = xcd_remap(blockIdx.x, gridDim.x);
    const int slot = find_slot(a.st.s, a.st.n, pid);
    const CycleSlot& sl = a.st.s[slot];
    const int tile = pid - sl.tile0;
    const LevelView<T>* Lp = static_cast<const LevelView<T>*>(sl.lv);
    const LevelView<T> L = *Lp;
    const SmoothBufs B = *sl.sb;
    const int nx = L.n[0], ny = L.n[1];
    int x0, y0;
    origin<TX, TY>(tile, nx, x0, y0);
    const T fs = (T)sl.fscale;

    // q0 on [-3, T+3) into sb
    if constexpr (POST) {
        correct_step<T, TX, TY, H, 4>(L, Lp[1], static_cast<const cx<T>*>(B.u1), static_cast<const cx<T>*>(sl.c),
                                      se, sa, x0, y0);
        __syncthreads();
        q0_step<T, TQ, TX, TY, H, 3, true>(L, sl.f, fs, nullptr, sa, sb, x0, y0);
    } else {
        q0_step<T, TQ, TX, TY, H, 3, false>(L, sl.f, fs, static_cast<const cx<T>*>(B.q[0]), nullptr, sb, x0, y0);
    }
    __syncthreads();
    // own points' q0 to registers
    cx<T> r0[PT];
#pragma unroll
    for (int k = 0; k < PT; ++k) {
        const int idx = threadIdx.x + k * NT;
        r0[k] = idx < TX * TY ? sb[R::at(idx % TX, idx / TX)] : mk<T>(0, 0);
    }
    // q1 on [-2, T+2) into sa, q2 on [-1, T+1) into sb
    power_step<T, TX, TY, H>(L, sb, sa, x0, y0, -2, TX + 1, TY + 1);
    __syncthreads();
    power_step<T, TX, TY, H>(L, sa, sb, x0, y0, -1, TX, TY);
    __syncthreads();
    cx<double> g[NUM_GRAM];
#pragma unroll
    for (int v = 0; v < NUM_GRAM; ++v) g[v] = mk(0.0, 0.0);
#pragma unroll
    for (int k = 0; k < PT; ++k) {
        const int idx = threadIdx.x + k * NT;
        if (idx < TX * TY) {
            const int lx = idx % TX, ly = idx / TX;
            const int gx = x0 + lx, gy = y0 + ly;
            if (gx < nx && gy < ny) {
                const int c = R::at(lx, ly);
                const cx<T> q3 =
                    L.sinv * lds_stencil<T, R::X>(L, sb, c, gx, gy, L.k2[(long long)gy * nx + gx]);
                gram_add<T>(g, r0[k], sa[c], sb[c], q3);
            }
        }
    }
    gram_store(g, sm, part, pstride, bstride, slot, tile);
}

// ---------------------------------------------------------------------------
// Pre-smoothing apply + restriction (zero incoming iterate, or NZ: the
// iterate in slot.u with q0 in the q0 buffer).
// ---------------------------------------------------------------------------
template <typename T, typename TQ, bool NZ, int TX, int TY>
__global__ void __launch_bounds__(NT) k_sm2_apply_restrict(const CycleArgs a) {
    constexpr int H = 4;
    using R = Reg<TX, TY, H>;
    constexpr int RX = TX + 1, RY = TY + 1, NRR = RX * RY;
    constexpr int PR = ceil_div(NRR, NT);
    constexpr int CX = TX / 2, CY = TY / 2;
    __shared__ cx<T> sa[R::N];
    __shared__ cx<T> sb[R::N];

    const int pid = xcd_remap(blockIdx.x, gridDim.x);
    const int slot = find_slot(a.st.s, a.st.n, pid);
    const CycleSlot& sl = a.st.s[slot];
    const LevelView<T>* Lp = static_cast<const LevelView<T>*>(sl.lv);
    const LevelView<T> L = *Lp;
    const SmoothBufs B = *sl.sb;
    const int nx = L.n[0], ny = L.n[1];
    int x0, y0;
    origin<TX, TY>(pid - sl.tile0, nx, x0, y0);
    const T fs = (T)sl.fscale;
    cx<T> c1, c2, c3;
    c1 = cvt<T>(B.coef[0]);
    c2 = cvt<T>(B.coef[1]);
    c3 = cvt<T>(B.coef[2]);

    // q0 on [-3, T+3] (the halo of 3 plus one more point on the high side)
    {
        const int nxx = nx;
        constexpr int W = TX + 7, Hh = TY + 7;
        for (int idx = threadIdx.x; idx < W * Hh; idx += NT) {
            const int lx = -3 + idx % W, ly = -3 + idx / W;
            const int gx = x0 + lx, gy = y0 + ly;
            cx<T> v = mk<T>(0, 0);
            if (gx >= 0 && gx < nxx && gy >= 0 && gy < ny) {
                const long long g = (long long)gy * nxx + gx;
                v = sl.f ? fs * cvt<T>(static_cast<const cx<TQ>*>(sl.f)[g])
                         : static_cast<const cx<T>*>(B.q[0])[g];
            }
            sa[R::at(lx, ly)] = v;
        }
    }
    __syncthreads();
    // q0 at the points of [0, T] to registers
    cx<T> r0[PR];
#pragma unroll
    for (int k = 0; k < PR; ++k) {
        const int idx = threadIdx.x + k * NT;
        r0[k] = idx < NRR ? sa[R::at(idx % RX, idx / RX)] : mk<T>(0, 0);
    }
    // q1 on [-2, T+2] into sb, q2 on [-1, T+1] into sa
    power_step<T, TX, TY, H>(L, sa, sb, x0, y0, -2, TX + 2, TY + 2);
    __syncthreads();
    power_step<T, TX, TY, H>(L, sb, sa, x0, y0, -1, TX + 1, TY + 1);
    __syncthreads();
    // r1 and u1 on [0, T]
    cx<T> r1[PR];
    cx<T>* u1p = static_cast<cx<T>*>(B.u1);
    const cx<T>* up = static_cast<const cx<T>*>(sl.u);
#pragma unroll
    for (int k = 0; k < PR; ++k) {
        const int idx = threadIdx.x + k * NT;
        r1[k] = mk<T>(0, 0);
        if (idx < NRR) {
            const int lx = idx % RX, ly = idx / RX;
            const int gx = x0 + lx, gy = y0 + ly;
            if (gx < nx && gy < ny) {
                const long long g = (long long)gy * nx + gx;
                const int c = R::at(lx, ly);
                const cx<T> q1 = sb[c], q2 = sa[c];
                const cx<T> q3 = L.sinv * lds_stencil<T, R::X>(L, sa, c, gx, gy, L.k2[g]);
                r1[k] = r0[k] + c1 * q1 + c2 * q2 + c3 * q3;
                if (lx < TX && ly < TY) {
                    cx<T> u = L.sinv * (c1 * r0[k] + c2 * q1 + c3 * q2);
                    if constexpr (NZ) u = up[g] - u;
                    else u = mk<T>(0, 0) - u;
                    u1p[g] = u;
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PR; ++k) {
        const int idx = threadIdx.x + k * NT;
        if (idx < NRR) sb[idx] = r1[k];
    }
    __syncthreads();
    // full weighting of r1 (sb, row stride RX) to the owned coarse points
    const int ncx = Lp[1].n[0], ncy = Lp[1].n[1];
    cx<T>* fc = static_cast<cx<T>*>(sl.c);
    for (int idx = threadIdx.x; idx < CX * CY; idx += NT) {
        const int cxl = idx % CX, cyl = idx / CX;
        const int Cx = x0 / 2 + cxl, Cy = y0 / 2 + cyl;
        if (Cx < ncx && Cy < ncy) {
            cx<T> acc = mk<T>(0, 0);
#pragma unroll
            for (int oy = -1; oy <= 1; ++oy) {
                const T wy = oy == 0 ? T(0.5) : T(0.25);
                const int row = (2 * cyl + 1 + oy) * RX + 2 * cxl + 1;
#pragma unroll
                for (int ox = -1; ox <= 1; ++ox) acc = acc + (wy * (ox == 0 ? T(0.5) : T(0.25))) * sb[row + ox];
            }
            fc[(long long)Cy * ncx + Cx] = acc;
        }
    }
}

// ---------------------------------------------------------------------------
// Post-smoothing apply: u2 = u1 + P e on [-3, T+3), q0 = fs f - A u2, q1, q2
// on shrinking halos, out = u2 - (c1 q0 + c2 q1 + c3 q2)/s on the tile.
// ---------------------------------------------------------------------------
template <typename T, typename TF, typename TO, bool ACC, int TX, int TY>
__global__ void __launch_bounds__(NT) k_sm2_apply_out(const CycleArgs a) {
    constexpr int H = 3;
    using R = Reg<TX, TY, H>;
    using E = CoarseWin<TX, TY, 3>;
    constexpr int PT = ceil_div(TX * TY, NT);
    __shared__ cx<T> sa[R::N];
    __shared__ cx<T> sb[R::N];
    __shared__ cx<T> se[E::N];

    const int pid = xcd_remap(blockIdx.x, gridDim.x);
    const int slot = find_slot(a.st.s, a.st.n, pid);
    const CycleSlot& sl = a.st.s[slot];
    const LevelView<T>* Lp = static_cast<const LevelView<T>*>(sl.lv);
    const LevelView<T> L = *Lp;
    const SmoothBufs B = *sl.sb;
    const int nx = L.n[0], ny = L.n[1];
    int x0, y0;
    origin<TX, TY>(pid - sl.tile0, nx, x0, y0);
    cx<T> c1, c2, c3;
    c1 = cvt<T>(B.coef[4]);
    c2 = cvt<T>(B.coef[5]);
    c3 = cvt<T>(B.coef[6]);

    correct_step<T, TX, TY, H, 3>(L, Lp[1], static_cast<const cx<T>*>(B.u1), static_cast<const cx<T>*>(sl.c), se, sa,
                                  x0, y0);
    __syncthreads();
    cx<T> u2[PT];
#pragma unroll
    for (int k = 0; k < PT; ++k) {
        const int idx = threadIdx.x + k * NT;
        u2[k] = idx < TX * TY ? sa[R::at(idx % TX, idx / TX)] : mk<T>(0, 0);
    }
    q0_step<T, TF, TX, TY, H, 2, true>(L, sl.f, (T)sl.fscale, nullptr, sa, sb, x0, y0);
    __syncthreads();
    power_step<T, TX, TY, H>(L, sb, sa, x0, y0, -1, TX, TY);   // q1 on [-1, T] over u2
    __syncthreads();
    cx<TO>* out = static_cast<cx<TO>*>(sl.out);
#pragma unroll
    for (int k = 0; k < PT; ++k) {
        const int idx = threadIdx.x + k * NT;
        if (idx < TX * TY) {
            const int lx = idx % TX, ly = idx / TX;
            const int gx = x0 + lx, gy = y0 + ly;
            if (gx < nx && gy < ny) {
                const long long g = (long long)gy * nx + gx;
                const int c = R::at(lx, ly);
                const cx<T> q2 = L.sinv * lds_stencil<T, R::X>(L, sa, c, gx, gy, L.k2[g]);
                const cx<T> v = u2[k] - L.sinv * (c1 * sb[c] + c2 * sa[c] + c3 * q2);
                if constexpr (ACC)
                    out[g] = out[g] + cvt<TO>(v);
                else
                    out[g] = cvt<TO>(v);
            }
        }
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers (2D only; shapes as the fused omega-Jacobi kernels)
// ---------------------------------------------------------------------------
#define MG_SHAPE2_SWITCH(LAUNCH)          \
    switch (shape) {                      \
        case 1: LAUNCH(64, 8); break;     \
        case 2: LAUNCH(128, 8); break;    \
        default: LAUNCH(64, 16); break;   \
    }

template <typename T, typename TQ, bool POST>
static hipError_t g2_launch(int shape, const CycleArgs& a, cx<double>* part, int pstride, int bstride,
                            hipStream_t s) {
#define G2(X, Y) \
    hipLaunchKernelGGL((k_sm2_gram<T, TQ, POST, X, Y>), dim3(a.st.ntiles), dim3(NT), 0, s, a, part, pstride, bstride);
    MG_SHAPE2_SWITCH(G2)
#undef G2
    return hipGetLastError();
}

hipError_t launch_sm2_gram(bool f32, bool level0, bool post, int shape, const CycleArgs& a, cx<double>* part,
                           int pstride, int bstride, hipStream_t s) {
    if (a.st.n <= 0) return hipSuccess;
    if (!f32)
        return post ? g2_launch<double, double, true>(shape, a, part, pstride, bstride, s)
                    : g2_launch<double, double, false>(shape, a, part, pstride, bstride, s);
    if (level0)
        return post ? g2_launch<float, double, true>(shape, a, part, pstride, bstride, s)
                    : g2_launch<float, double, false>(shape, a, part, pstride, bstride, s);
    return post ? g2_launch<float, float, true>(shape, a, part, pstride, bstride, s)
                : g2_launch<float, float, false>(shape, a, part, pstride, bstride, s);
}

template <typename T, typename TQ, bool NZ>
static hipError_t ar2_launch(int shape, const CycleArgs& a, hipStream_t s) {
#define AR2(X, Y) hipLaunchKernelGGL((k_sm2_apply_restrict<T, TQ, NZ, X, Y>), dim3(a.st.ntiles), dim3(NT), 0, s, a);
    MG_SHAPE2_SWITCH(AR2)
#undef AR2
    return hipGetLastError();
}

hipError_t launch_sm2_apply_restrict(bool f32, bool level0, bool nonzero, int shape, const CycleArgs& a,
                                     hipStream_t s) {
    if (a.st.n <= 0) return hipSuccess;
    if (!f32) return nonzero ? ar2_launch<double, double, true>(shape, a, s) : ar2_launch<double, double, false>(shape, a, s);
    if (nonzero) return hipErrorInvalidValue;
    return level0 ? ar2_launch<float, double, false>(shape, a, s) : ar2_launch<float, float, false>(shape, a, s);
}

template <typename T, typename TF, typename TO, bool ACC>
static hipError_t ao2_launch(int shape, const CycleArgs& a, hipStream_t s) {
#define AO2(X, Y) hipLaunchKernelGGL((k_sm2_apply_out<T, TF, TO, ACC, X, Y>), dim3(a.st.ntiles), dim3(NT), 0, s, a);
    MG_SHAPE2_SWITCH(AO2)
#undef AO2
    return hipGetLastError();
}

hipError_t launch_sm2_apply_out(bool f32, bool level0, bool accumulate, int shape, const CycleArgs& a, hipStream_t s) {
    if (a.st.n <= 0) return hipSuccess;
    if (!f32)
        return accumulate ? ao2_launch<double, double, double, true>(shape, a, s)
                          : ao2_launch<double, double, double, false>(shape, a, s);
    if (level0)
        return accumulate ? ao2_launch<float, double, double, true>(shape, a, s)
                          : ao2_launch<float, double, double, false>(shape, a, s);
    return ao2_launch<float, float, float, false>(shape, a, s);
}

}  // namespace mg
