// Device helpers shared by the kernel translation units (gfx950, wave64).
#pragma once

#include "mg_device.hpp"

// dispatch over (dim, shape) of a fused kernel template K<D, TX, TY, TZ>
#define MG_SHAPE_SWITCH(LAUNCH)                                                    \
    if (dim == 2) {                                                                \
        switch (shape) {                                                           \
            case 1: LAUNCH(2, 64, 8, 1); break;                                    \
            case 2: LAUNCH(2, 128, 8, 1); break;                                   \
            default: LAUNCH(2, 64, 16, 1); break;                                  \
        }                                                                          \
    } else {                                                                       \
        switch (shape) {                                                           \
            case 1: LAUNCH(3, 32, 4, 2); break;                                    \
            case 2: LAUNCH(3, 16, 4, 4); break;                                    \
            default: LAUNCH(3, 16, 8, 4); break;                                   \
        }                                                                          \
    }


namespace mg {
namespace kc {

// Device memory seen as the global address space.  Pointers read out of the
// slot tables and level descriptors are generic, and loads through generic
// pointers are flat instructions, which also count against the LDS wait
// counter: every LDS wait or barrier would then drain them.  Accesses
// through these views are global instructions, so the loads of a pass stay
// in flight across its LDS traffic.  Elements are read and written by value
// (complex values member by member; the compiler merges the two halves).
template <typename T>
using gptr = __attribute__((address_space(1))) T*;

template <typename T>
struct GVal {
    __device__ static __forceinline__ T get(gptr<const T> q) { return *q; }
    __device__ static __forceinline__ void put(gptr<T> q, T v) { *q = v; }
};
template <typename U>
struct GVal<cx<U>> {
    __device__ static __forceinline__ cx<U> get(gptr<const cx<U>> q) { return mk<U>(q->r, q->i); }
    __device__ static __forceinline__ void put(gptr<cx<U>> q, cx<U> v) {
        q->r = v.r;
        q->i = v.i;
    }
};

// read-only view
template <typename T>
struct GIn {
    gptr<const T> p;
    __device__ __forceinline__ T operator[](long long i) const { return GVal<T>::get(p + i); }
    __device__ __forceinline__ explicit operator bool() const { return p != nullptr; }
};
// element of a writable view
template <typename T>
struct GRef {
    gptr<T> q;
    __device__ __forceinline__ void operator=(T v) const { GVal<T>::put(q, v); }
    __device__ __forceinline__ T get() const { return GVal<T>::get((gptr<const T>)q); }
};
// writable view
template <typename T>
struct GOut {
    gptr<T> p;
    __device__ __forceinline__ GRef<T> operator[](long long i) const { return GRef<T>{p + i}; }
    __device__ __forceinline__ explicit operator bool() const { return p != nullptr; }
};
// read-only view of streamed complex data (each element read once per
// pass, not again before it would be evicted): loads carry the nontemporal
// hint
struct GStream {
    gptr<const double> p;
    __device__ __forceinline__ cx<double> operator[](long long i) const {
        return mk(__builtin_nontemporal_load(p + 2 * i), __builtin_nontemporal_load(p + 2 * i + 1));
    }
};
__device__ __forceinline__ GStream gstream(const cx<double>* p) {
    return GStream{(gptr<const double>)p};
}
template <typename T>
__device__ __forceinline__ GIn<T> gin(const T* p) {
    return GIn<T>{(gptr<const T>)p};
}
template <typename T>
__device__ __forceinline__ GOut<T> gout(T* p) {
    return GOut<T>{(gptr<T>)p};
}

// A level descriptor with global views (same fields as LevelView).
template <typename T>
struct GLevel {
    int n[3];
    int ntiles[3];
    long long N;
    GIn<cx<T>> cm[3];
    GIn<cx<T>> c0[3];
    GIn<cx<T>> cp[3];
    GIn<T> k2;
    GIn<cx<double>> cinv;
    cx<T> sigma;
    cx<T> omega;
    T sinv;
};

template <typename T>
__device__ __forceinline__ GLevel<T> glevel(const LevelView<T>& v) {
    GLevel<T> g;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        g.n[a] = v.n[a];
        g.ntiles[a] = v.ntiles[a];
        g.cm[a] = gin(v.cm[a]);
        g.c0[a] = gin(v.c0[a]);
        g.cp[a] = gin(v.cp[a]);
    }
    g.N = v.N;
    g.k2 = gin(v.k2);
    g.cinv = gin(v.cinv);
    g.sigma = v.sigma;
    g.omega = v.omega;
    g.sinv = v.sinv;
    return g;
}

constexpr int NT = 256;      // threads per workgroup (4 wave64)
constexpr int NXCD = 8;      // MI355X: 8 XCDs, workgroups dealt round-robin

// Map the hardware workgroup id to a logical tile id such that each XCD gets
// one contiguous range of tiles (neighbouring tiles share halos in its L2).
__device__ __forceinline__ int xcd_remap(int pid, int num) {
    const int xcd = pid % NXCD;
    const int local = pid / NXCD;
    const int per = num / NXCD;
    const int extra = num % NXCD;
    return xcd * per + (xcd < extra ? xcd : extra) + local;
}

// v of the lane that DPP control CTRL selects (rows outside ROWMASK get 0).
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_f64(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffull), CTRL, ROWMASK, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, ROWMASK, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Sum over the 64 lanes of a wavefront (every lane active), returned to
// every lane, in a fixed order.  All on the VALU through DPP (no LDS
// permutes, which the waves of a CU would share): quad swaps, half-row and
// row mirrors give each 16-lane row its sum, the two row broadcasts carry
// the row sums into lane 63, which is read back.
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_f64<0xB1, 0xF>(v);    // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E, 0xF>(v);    // quad_perm [2,3,0,1]
    v += dpp_f64<0x141, 0xF>(v);   // row_half_mirror
    v += dpp_f64<0x140, 0xF>(v);   // row_mirror
    v += dpp_f64<0x142, 0xA>(v);   // row_bcast:15 into rows 1, 3
    v += dpp_f64<0x143, 0xC>(v);   // row_bcast:31 into rows 2, 3
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffull), 63);
    const int hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), 63);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Deterministic workgroup sum; the result is valid in thread 0.  sm holds
// NT/64 doubles.  Must be reached by every thread of the workgroup.
__device__ __forceinline__ double block_sum(double v, double* sm) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sm[wave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) t += sm[w];
    }
    return t;
}

// Slot of logical workgroup pid: the last slot whose first tile is <= pid
// (slots are listed in increasing first-tile order).
template <typename S>
__device__ __forceinline__ int find_slot(const S* s, int n, int pid) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s[mid].tile0 <= pid)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

template <int D, typename LV, typename T>
__device__ __forceinline__ cx<T> diag_at(const LV& L, int gx, int gy, int gz, T k2) {
    cx<T> d = L.c0[0][gx] + L.c0[1][gy];
    if constexpr (D == 3) d = d + L.c0[2][gz];
    return d - k2 * L.sigma;
}

template <typename T>
__device__ __forceinline__ void interp_1d(int g, int cs, int& i0, int& i1, T& w0, T& w1) {
    if (g & 1) {
        i0 = (g - 1) / 2 - cs;
        i1 = i0;
        w0 = T(1);
        w1 = T(0);
    } else {
        const int J = g / 2;
        i0 = J - 1 - cs;
        i1 = J - cs;
        w0 = T(0.5);
        w1 = T(0.5);
    }
}

// Slot, workgroup within the slot and its point range [lo, hi).
struct VecPos {
    int slot, b, nb, lo, hi;
};

__device__ __forceinline__ VecPos vec_pos(const VecSlots& st) {
    VecPos q;
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
    q.lo = q.hi = 0;
    return q;
}

__device__ __forceinline__ void chunk_range(long long N, int nblocks, int b, int& lo, int& hi) {
    const long long per = (N + nblocks - 1) / nblocks;
    long long l = per * b, h = l + per;
    if (l > N) l = N;
    if (h > N) h = N;
    lo = (int)l;
    hi = (int)h;
}


// v where c holds, else 0, component by component (a select of whole
// structures would go through scratch memory).
template <typename T>
__device__ __forceinline__ cx<T> masked(bool c, cx<T> v) {
    return mk<T>(c ? v.r : T(0), c ? v.i : T(0));
}

// Complex products accumulated by fused multiply-adds, two per component:
// acc + a b, and acc + conj(a) b.  (Written as (acc + a*b) the compiler
// fuses only the inner product and adds acc separately.)
template <typename T>
__device__ __forceinline__ cx<T> cfma(cx<T> a, cx<T> b, cx<T> acc) {
    return mk<T>(fma(-a.i, b.i, fma(a.r, b.r, acc.r)), fma(a.i, b.r, fma(a.r, b.i, acc.i)));
}
template <typename T>
__device__ __forceinline__ cx<T> cfmac(cx<T> a, cx<T> b, cx<T> acc) {
    return mk<T>(fma(a.i, b.i, fma(a.r, b.r, acc.r)), fma(-a.i, b.r, fma(a.r, b.i, acc.i)));
}
// acc + |a|^2
template <typename T>
__device__ __forceinline__ T fabs2(cx<T> a, T acc) {
    return fma(a.i, a.i, fma(a.r, a.r, acc));
}

// 3-point-per-axis stencil of the level operator at point p of x, x scaled by
// xs and converted to the compute precision T.  Every load is issued (a
// neighbour outside the grid reads the point itself) and the missing terms
// are masked to exact zeros: a load under a branch would make the compiler
// wait for all loads in flight before its use.
template <int D, typename T, typename TX, typename LV, typename PX>
__device__ __forceinline__ cx<T> stencil_at(const LV& L, PX x, T xs, long long p, int gx, int gy, int gz) {
    const int nx = L.n[0], ny = L.n[1], nz = L.n[2];
    const bool bxm = gx > 0, bxp = gx < nx - 1, bym = gy > 0, byp = gy < ny - 1;
    const bool bzm = D == 3 && gz > 0, bzp = D == 3 && gz < nz - 1;
    const long long sz = (long long)nx * ny;
    const int az = D == 3 ? gz : 0;
    // every load first (the scheduler would otherwise sink them to their uses
    // and wait for them one by one)
    const auto v0 = x[p];
    const auto vxm = x[bxm ? p - 1 : p], vxp = x[bxp ? p + 1 : p];
    const auto vym = x[bym ? p - nx : p], vyp = x[byp ? p + nx : p];
    const auto vzm = x[bzm ? p - sz : p], vzp = x[bzp ? p + sz : p];
    const cx<T> cmx = L.cm[0][gx], cpx = L.cp[0][gx], c0x = L.c0[0][gx];
    const cx<T> cmy = L.cm[1][gy], cpy = L.cp[1][gy], c0y = L.c0[1][gy];
    cx<T> cmz = mk<T>(0, 0), cpz = cmz, c0z = cmz;   // the z arrays exist in 3D only
    if constexpr (D == 3) {
        cmz = L.cm[2][az];
        cpz = L.cp[2][az];
        c0z = L.c0[2][az];
    }
    const T k2 = L.k2[p];
    __builtin_amdgcn_sched_barrier(0);
    cx<T> d = c0x + c0y;
    if constexpr (D == 3) d = d + c0z;
    d = d - k2 * L.sigma;
    cx<T> ax = d * cvt<T>(v0);
    ax = ax + masked(bxm, cmx) * cvt<T>(vxm);
    ax = ax + masked(bxp, cpx) * cvt<T>(vxp);
    ax = ax + masked(bym, cmy) * cvt<T>(vym);
    ax = ax + masked(byp, cpy) * cvt<T>(vyp);
    if constexpr (D == 3) {
        ax = ax + masked(bzm, cmz) * cvt<T>(vzm);
        ax = ax + masked(bzp, cpz) * cvt<T>(vzp);
    }
    return xs * ax;
}

__device__ __forceinline__ cx<double> conjd(cx<double> z) { return mk(z.r, -z.i); }

// Coefficients of the least-squares residual polynomial from the Gram matrix.
// brk: relative pivot below which the Krylov space counts as exhausted.
__device__ inline void solve_coef(const cx<double>* G, double brk, cx<double>* out) {
    const double g00 = G[0].r;
    out[0] = out[1] = out[2] = mk(0.0, 0.0);
    out[3] = mk(g00, 0.0);
    if (!(g00 > 0.0) || !(G[1].r > 0.0)) return;
    const double d0 = sqrt(g00), d1 = sqrt(G[1].r), d2 = sqrt(G[2].r), d3 = sqrt(G[3].r);
    // right-hand side b_i = -G_i0 / (d_i d0), G_i0 = conj(G_0i)
    const cx<double> b1 = (-1.0 / (d1 * d0)) * conjd(G[4]);
    int deg = 1;
    cx<double> L21 = mk(0.0, 0.0), L31 = mk(0.0, 0.0), L32 = mk(0.0, 0.0);
    double L22 = 0.0, L33 = 0.0;
    cx<double> b2 = mk(0.0, 0.0), b3 = mk(0.0, 0.0);
    if (d2 > 0.0) {
        L21 = (1.0 / (d1 * d2)) * conjd(G[7]);
        const double p2 = 1.0 - abs2(L21);
        if (p2 > brk) {
            deg = 2;
            L22 = sqrt(p2);
            b2 = (-1.0 / (d2 * d0)) * conjd(G[5]);
            if (d3 > 0.0) {
                L31 = (1.0 / (d1 * d3)) * conjd(G[8]);
                const cx<double> S32 = (1.0 / (d2 * d3)) * conjd(G[9]);
                L32 = (1.0 / L22) * (S32 - L31 * conjd(L21));
                const double p3 = 1.0 - abs2(L31) - abs2(L32);
                if (p3 > brk) {
                    deg = 3;
                    L33 = sqrt(p3);
                    b3 = (-1.0 / (d3 * d0)) * conjd(G[6]);
                }
            }
        }
    }
    // L y = b, L^H x = y
    cx<double> x1, x2 = mk(0.0, 0.0), x3 = mk(0.0, 0.0);
    const cx<double> y1 = b1;
    if (deg == 1) {
        x1 = y1;
    } else {
        const cx<double> y2 = (1.0 / L22) * (b2 - L21 * y1);
        if (deg == 3) {
            const cx<double> y3 = (1.0 / L33) * (b3 - L31 * y1 - L32 * y2);
            x3 = (1.0 / L33) * y3;
        }
        x2 = (1.0 / L22) * (y2 - conjd(L32) * x3);
        x1 = y1 - conjd(L21) * x2 - conjd(L31) * x3;
    }
    out[0] = (d0 / d1) * x1;
    out[1] = deg >= 2 ? (d0 / d2) * x2 : mk(0.0, 0.0);
    out[2] = deg == 3 ? (d0 / d3) * x3 : mk(0.0, 0.0);
}

// Tiles of slot `slot` of a fused-kernel launch.
__device__ __forceinline__ int slot_tiles(const CycleArgs& a, int slot) {
    return (slot + 1 < a.st.n ? a.st.s[slot + 1].tile0 : a.st.ntiles) - a.st.s[slot].tile0;
}

// The smoothing coefficients of slot `slot` of a 2D GMRES(3) apply launch
// from the Gram partials of the preceding Gram pass (same slots and tiles,
// at most FUSED_COEF_TILES of them), formed by one wavefront in two steps:
// coef_load issues the loads (lane l takes tiles l, l + 64, ...), so that
// their latency passes while the caller loads its tile; coef_solve sums in a
// fixed order (lanes, then the wave sum) and solves.  Every lane of every
// wavefront gets the same values.
struct CoefLoad {
    static constexpr int KB = FUSED_COEF_TILES / 64;
    cx<double> v[KB][NUM_GRAM];
    int cnt;
};

__device__ __forceinline__ void coef_load(const CycleArgs& a, int slot, CoefLoad& cl) {
    const int lane = threadIdx.x & 63;
    cl.cnt = slot_tiles(a, slot);
    const cx<double>* P = a.gpart + (long long)slot * a.gpstride * a.gbstride;
#pragma unroll
    for (int k = 0; k < CoefLoad::KB; ++k) {
        const int b = lane + 64 * k;
        const int bb = b < cl.cnt ? b : 0;
#pragma unroll
        for (int g = 0; g < NUM_GRAM; ++g) cl.v[k][g] = P[(long long)g * a.gbstride + bb];
    }
}

__device__ __forceinline__ void coef_solve(const CoefLoad& cl, double brk, cx<double>* out) {
    const int lane = threadIdx.x & 63;
    cx<double> G[NUM_GRAM];
#pragma unroll
    for (int g = 0; g < NUM_GRAM; ++g) {
        double r = 0.0, i = 0.0;
#pragma unroll
        for (int k = 0; k < CoefLoad::KB; ++k) {
            const bool in = lane + 64 * k < cl.cnt;
            r += in ? cl.v[k][g].r : 0.0;
            i += in ? cl.v[k][g].i : 0.0;
        }
        G[g] = mk(wave_sum(r), g < 4 ? 0.0 : wave_sum(i));
    }
    solve_coef(G, brk, out);
}

}  // namespace kc
}  // namespace mg
