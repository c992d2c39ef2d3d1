// The coarse tail of the V-cycle (Sec. 3.1) in one launch: every level of at
// most TAIL_POINTS points, the coarsest direct solve and the way back up, one
// 1024-thread workgroup per right-hand side, passes separated by workgroup
// barriers.  The vectors of levels of at most SMALL_POINTS points (right-hand
// sides, iterates, corrections, the smoother's powers) live in LDS and each
// thread holds its point's stencil coefficients in registers through a
// level's passes; larger tail levels (up to 4 points per thread) use global
// work vectors.  The coarsest solve multiplies by the inverse of the
// coarsest operator, formed in FP64 at set-up.  Smoothing is omega-Jacobi
// (Sec. 3.2.1) or one GMRES(3) step (Sec. 3.2.2) with the minimiser from the
// Gram matrix of the scaled power basis, reduced inside the workgroup.

#include "mg_kcommon.hpp"

namespace mg {

using namespace kc;

namespace {

constexpr int NTT = 1024;
constexpr int MAX_TAIL_LEVELS = 16;

template <int D>
__device__ __forceinline__ void pos3(int p, int nx, int ny, int& gx, int& gy, int& gz) {
    gx = p % nx;
    const int rr = p / nx;
    gy = rr % ny;
    gz = (D == 3) ? rr / ny : 0;
}

template <typename T>
__device__ __forceinline__ void axis_w(int g, int nc, int& i0, int& i1, T& w0, T& w1) {
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

// (P e)(p): bilinear / trilinear interpolation from the next level.
template <int D, typename T>
__device__ __forceinline__ cx<T> prolong_at(const LevelView<T>& Lc, const cx<T>* e, int gx, int gy, int gz) {
    int x0, x1, y0, y1, z0 = 0, z1 = 0;
    T wx0, wx1, wy0, wy1, wz0 = T(1), wz1 = T(0);
    axis_w<T>(gx, Lc.n[0], x0, x1, wx0, wx1);
    axis_w<T>(gy, Lc.n[1], y0, y1, wy0, wy1);
    if constexpr (D == 3) axis_w<T>(gz, Lc.n[2], z0, z1, wz0, wz1);
    const int sx = Lc.n[0], sxy = Lc.n[0] * Lc.n[1];
    cx<T> v = mk<T>(0, 0);
#pragma unroll
    for (int kz = 0; kz < (D == 3 ? 2 : 1); ++kz) {
        const int zz = kz ? z1 : z0;
        const T wz = kz ? wz1 : wz0;
#pragma unroll
        for (int ky = 0; ky < 2; ++ky) {
            const int yy = ky ? y1 : y0;
            const T wy = ky ? wy1 : wy0;
            const cx<T>* row = e + zz * sxy + yy * sx;
            v = v + (wz * wy * wx0) * row[x0] + (wz * wy * wx1) * row[x1];
        }
    }
    return v;
}

// Full weighting of r at coarse point (cx, cy, cz) of the next level.
template <int D, typename T>
__device__ __forceinline__ cx<T> restrict_at(const LevelView<T>& L, const cx<T>* r, int cx_, int cy, int cz) {
    const int nx = L.n[0], ny = L.n[1];
    cx<T> acc = mk<T>(0, 0);
#pragma unroll
    for (int oz = (D == 3 ? -1 : 0); oz <= (D == 3 ? 1 : 0); ++oz) {
        const T wz = (D == 3) ? (oz == 0 ? T(0.5) : T(0.25)) : T(1);
        const int zb = (D == 3) ? (2 * cz + 1 + oz) * nx * ny : 0;
#pragma unroll
        for (int oy = -1; oy <= 1; ++oy) {
            const T wy = wz * (oy == 0 ? T(0.5) : T(0.25));
            const cx<T>* row = r + zb + (2 * cy + 1 + oy) * nx + 2 * cx_ + 1;
#pragma unroll
            for (int ox = -1; ox <= 1; ++ox) acc = acc + (wy * (ox == 0 ? T(0.5) : T(0.25))) * row[ox];
        }
    }
    return acc;
}

// Stencil coefficients of one point, held in registers through a level's
// passes (LDS levels: one point per thread).
template <typename T>
struct PtCoef {
    cx<T> d;                       // sum of the c0 - sigma k^2
    cx<T> m[3], pl[3];             // minus / plus neighbour per axis (0 at the boundary)
    int gx, gy, gz;
};

template <int D, typename T>
__device__ __forceinline__ PtCoef<T> pt_coef(const LevelView<T>& L, int p) {
    PtCoef<T> c;
    pos3<D>(p, L.n[0], L.n[1], c.gx, c.gy, c.gz);
    c.d = diag_at<D>(L, c.gx, c.gy, c.gz, L.k2[p]);
    const int g[3] = {c.gx, c.gy, c.gz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        c.m[a] = c.pl[a] = mk<T>(0, 0);
        if (a < D) {
            if (g[a] > 0) c.m[a] = L.cm[a][g[a]];
            if (g[a] < L.n[a] - 1) c.pl[a] = L.cp[a][g[a]];
        }
    }
    return c;
}

// (A x)(p) * sc with the point's coefficients in registers.
template <int D, typename T>
__device__ __forceinline__ cx<T> apply_pt(const PtCoef<T>& c, const LevelView<T>& L, const cx<T>* x, int p, T sc) {
    const int nx = L.n[0], nxy = L.n[0] * L.n[1];
    cx<T> ax = c.d * x[p];
    if (c.gx > 0) ax = ax + c.m[0] * x[p - 1];
    if (c.gx < nx - 1) ax = ax + c.pl[0] * x[p + 1];
    if (c.gy > 0) ax = ax + c.m[1] * x[p - nx];
    if (c.gy < L.n[1] - 1) ax = ax + c.pl[1] * x[p + nx];
    if constexpr (D == 3) {
        if (c.gz > 0) ax = ax + c.m[2] * x[p - nxy];
        if (c.gz < L.n[2] - 1) ax = ax + c.pl[2] * x[p + nxy];
    }
    return sc * ax;
}

// (A x)(p) * sc reading the coefficients from global memory.
template <int D, typename T>
__device__ __forceinline__ cx<T> apply_gl(const LevelView<T>& L, const cx<T>* x, int p, T sc) {
    int gx, gy, gz;
    pos3<D>(p, L.n[0], L.n[1], gx, gy, gz);
    return stencil_at<D, T, T>(L, x, sc, p, gx, gy, gz);
}

constexpr int PPT = TAIL_POINTS / NTT;   // points per thread on a tail level in global memory

// Gram partials of the thread's points and the workgroup coefficient solve
// (coefficients land in sc[0..2]).
__device__ void gram_finish(cx<double>* g, double brk, cx<double>* sred, cx<double>* sc) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < NUM_GRAM; ++v) {
        const double r = wave_sum(g[v].r), i = wave_sum(g[v].i);
        if (lane == 0) sred[wave * NUM_GRAM + v] = mk(r, i);
    }
    __syncthreads();
    if ((int)threadIdx.x < NUM_GRAM) {
        cx<double> t = mk(0.0, 0.0);
        for (int w = 0; w < NTT / 64; ++w) t = t + sred[w * NUM_GRAM + threadIdx.x];
        sred[(NTT / 64) * NUM_GRAM + threadIdx.x] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) solve_coef(sred + (NTT / 64) * NUM_GRAM, brk, sc);
    __syncthreads();
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

// Vectors of one level of the tail: in LDS (small levels) or global memory.
template <typename T>
struct LvVec {
    cx<T>* f;
    cx<T>* u;
    cx<T>* q[3];
};

// Pre-smoothing of level k (zero initial guess) and the restriction of its
// residual into fc.  SMALL: at most one point per thread, coefficients in
// registers; otherwise up to PPT points per thread.
template <int D, typename T, bool GM, bool SMALL>
__device__ void level_down(const LevelView<T>& L, const LevelView<T>& Lc, const LvVec<T>& v, cx<T>* fc, double brk,
                           cx<double>* sred, cx<double>* sc) {
    const int N = (int)L.N;
    constexpr int NP = SMALL ? 1 : PPT;
    PtCoef<T> pc;
    if constexpr (SMALL)
        if ((int)threadIdx.x < N) pc = pt_coef<D, T>(L, threadIdx.x);
    auto A = [&](const cx<T>* x, int p, T s) -> cx<T> {
        if constexpr (SMALL) return apply_pt<D, T>(pc, L, x, p, s);
        else return apply_gl<D, T>(L, x, p, s);
    };
    if constexpr (GM) {
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int p = threadIdx.x + i * NTT;
            if (p < N) v.q[1][p] = A(v.f, p, L.sinv);
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int p = threadIdx.x + i * NTT;
            if (p < N) v.q[2][p] = A(v.q[1], p, L.sinv);
        }
        __syncthreads();
        cx<double> g[NUM_GRAM];
#pragma unroll
        for (int j = 0; j < NUM_GRAM; ++j) g[j] = mk(0.0, 0.0);
        cx<T> q3[NP];
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int p = threadIdx.x + i * NTT;
            q3[i] = mk<T>(0, 0);
            if (p < N) {
                q3[i] = A(v.q[2], p, L.sinv);
                gram_add<T>(g, v.f[p], v.q[1][p], v.q[2][p], q3[i]);
            }
        }
        gram_finish(g, brk, sred, sc);
        const cx<T> c1 = cvt<T>(sc[0]), c2 = cvt<T>(sc[1]), c3 = cvt<T>(sc[2]);
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int p = threadIdx.x + i * NTT;
            if (p < N) {
                const cx<T> q0 = v.f[p], q1 = v.q[1][p], q2 = v.q[2][p];
                v.u[p] = mk<T>(0, 0) - L.sinv * (c1 * q0 + c2 * q1 + c3 * q2);
                v.q[1][p] = q0 + c1 * q1 + c2 * q2 + c3 * q3[i];   // the new residual
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int p = threadIdx.x + i * NTT;
            if (p < N) {
                cx<T> d;
                if constexpr (SMALL) d = pc.d;
                else {
                    int gx, gy, gz;
                    pos3<D>(p, L.n[0], L.n[1], gx, gy, gz);
                    d = diag_at<D>(L, gx, gy, gz, L.k2[p]);
                }
                v.u[p] = cdiv(L.omega * v.f[p], d);
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int p = threadIdx.x + i * NTT;
            if (p < N) v.q[1][p] = v.f[p] - A(v.u, p, T(1));
        }
    }
    __syncthreads();
    for (int p = threadIdx.x; p < (int)Lc.N; p += NTT) {
        int cx_, cy, cz;
        pos3<D>(p, Lc.n[0], Lc.n[1], cx_, cy, cz);
        fc[p] = restrict_at<D, T>(L, v.q[1], cx_, cy, cz);
    }
    __syncthreads();
}

// Coarse-grid correction u2 = u1 + P ec and post-smoothing of level k; the
// correction of the level lands in v.u.
template <int D, typename T, bool GM, bool SMALL>
__device__ void level_up(const LevelView<T>& L, const LevelView<T>& Lc, const LvVec<T>& v, const cx<T>* ec,
                         double brk, cx<double>* sred, cx<double>* sc) {
    const int N = (int)L.N;
    constexpr int NP = SMALL ? 1 : PPT;
    PtCoef<T> pc;
    if constexpr (SMALL)
        if ((int)threadIdx.x < N) pc = pt_coef<D, T>(L, threadIdx.x);
    auto A = [&](const cx<T>* x, int p, T s) -> cx<T> {
        if constexpr (SMALL) return apply_pt<D, T>(pc, L, x, p, s);
        else return apply_gl<D, T>(L, x, p, s);
    };
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        const int p = threadIdx.x + i * NTT;
        if (p < N) {
            int gx, gy, gz;
            pos3<D>(p, L.n[0], L.n[1], gx, gy, gz);
            v.u[p] = v.u[p] + prolong_at<D, T>(Lc, ec, gx, gy, gz);
        }
    }
    __syncthreads();
    if constexpr (GM) {
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int p = threadIdx.x + i * NTT;
            if (p < N) v.q[0][p] = v.f[p] - A(v.u, p, T(1));
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int p = threadIdx.x + i * NTT;
            if (p < N) v.q[1][p] = A(v.q[0], p, L.sinv);
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int p = threadIdx.x + i * NTT;
            if (p < N) v.q[2][p] = A(v.q[1], p, L.sinv);
        }
        __syncthreads();
        cx<double> g[NUM_GRAM];
#pragma unroll
        for (int j = 0; j < NUM_GRAM; ++j) g[j] = mk(0.0, 0.0);
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int p = threadIdx.x + i * NTT;
            if (p < N) gram_add<T>(g, v.q[0][p], v.q[1][p], v.q[2][p], A(v.q[2], p, L.sinv));
        }
        gram_finish(g, brk, sred, sc);
        const cx<T> c1 = cvt<T>(sc[0]), c2 = cvt<T>(sc[1]), c3 = cvt<T>(sc[2]);
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int p = threadIdx.x + i * NTT;
            if (p < N) v.u[p] = v.u[p] - L.sinv * (c1 * v.q[0][p] + c2 * v.q[1][p] + c3 * v.q[2][p]);
        }
        __syncthreads();
    } else {
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int p = threadIdx.x + i * NTT;
            if (p < N) {
                cx<T> d;
                if constexpr (SMALL) d = pc.d;
                else {
                    int gx, gy, gz;
                    pos3<D>(p, L.n[0], L.n[1], gx, gy, gz);
                    d = diag_at<D>(L, gx, gy, gz, L.k2[p]);
                }
                v.q[0][p] = v.u[p] + cdiv(L.omega * (v.f[p] - A(v.u, p, T(1))), d);
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int p = threadIdx.x + i * NTT;
            if (p < N) v.u[p] = v.q[0][p];
        }
        __syncthreads();
    }
}

template <int D, typename T, bool GM>
__global__ void __launch_bounds__(NTT) k_tail(const TailArgs a) {
    __shared__ cx<T> sf[TAIL_LDS];            // right-hand side of every LDS level
    __shared__ cx<T> su[TAIL_LDS];            // iterate, then correction, of every LDS level
    __shared__ cx<T> sq[3][SMALL_POINTS];     // powers / residuals of the LDS level in progress
    __shared__ cx<double> sred[(NTT / 64 + 1) * NUM_GRAM];
    __shared__ cx<double> sc[4];
    const TailSlot& ts = a.s[blockIdx.x];
    if (gated_off(ts.gate)) return;
    const LevelView<T>* Lv = static_cast<const LevelView<T>*>(ts.lv);
    const SmoothBufs* SB = ts.sb;
    const int last = ts.nlev - 1;
    // levels 0 .. big-1 of the tail keep their vectors in global memory
    int big = 0;
    while (big < last && Lv[big].N > SMALL_POINTS) ++big;
    __shared__ int off[MAX_TAIL_LEVELS + 1];   // LDS offsets of the small levels
    if (threadIdx.x == 0) {
        for (int k = 0; k <= big; ++k) off[k] = 0;
        for (int k = big; k <= last && k < MAX_TAIL_LEVELS; ++k) off[k + 1] = off[k] + (int)Lv[k].N;
    }
    __syncthreads();
    auto vecs = [&](int k) -> LvVec<T> {
        LvVec<T> v;
        if (k < big) {
            const SmoothBufs& B = SB[k];
            v.f = static_cast<cx<T>*>(B.f);
            v.u = static_cast<cx<T>*>(B.u1);
            for (int i = 0; i < 3; ++i) v.q[i] = static_cast<cx<T>*>(B.q[i]);
        } else {
            v.f = sf + off[k];
            v.u = su + off[k];
            for (int i = 0; i < 3; ++i) v.q[i] = sq[i];
        }
        return v;
    };

    if (big == 0) {   // right-hand side of the first tail level into LDS
        const cx<T>* fg = static_cast<const cx<T>*>(SB[0].f);
        for (int p = threadIdx.x; p < (int)Lv[0].N; p += NTT) sf[p] = fg[p];
        __syncthreads();
    }
    for (int k = 0; k < last; ++k) {
        const LvVec<T> v = vecs(k);
        cx<T>* fc = vecs(k + 1).f;
        if (k < big) level_down<D, T, GM, false>(Lv[k], Lv[k + 1], v, fc, a.brk, sred, sc);
        else level_down<D, T, GM, true>(Lv[k], Lv[k + 1], v, fc, a.brk, sred, sc);
    }
    {   // coarsest: e = A^{-1} f with the FP64 inverse
        const LevelView<T> C = Lv[last];
        const int n = (int)C.N;
        const LvVec<T> v = vecs(last);
        for (int p = threadIdx.x; p < n; p += NTT) {
            const cx<double>* row = C.cinv + (long long)p * n;
            cx<double> s = mk(0.0, 0.0);
            for (int j = 0; j < n; ++j) s = s + row[j] * cvt<double>(v.f[j]);
            v.u[p] = cvt<T>(s);
        }
        __syncthreads();
    }
    for (int k = last - 1; k >= 0; --k) {
        const LvVec<T> v = vecs(k);
        const cx<T>* ec = vecs(k + 1).u;
        if (k < big) level_up<D, T, GM, false>(Lv[k], Lv[k + 1], v, ec, a.brk, sred, sc);
        else level_up<D, T, GM, true>(Lv[k], Lv[k + 1], v, ec, a.brk, sred, sc);
    }
    {   // correction of the first tail level
        cx<T>* eg = static_cast<cx<T>*>(SB[0].e);
        const cx<T>* src = vecs(0).u;
        for (int p = threadIdx.x; p < (int)Lv[0].N; p += NTT) eg[p] = src[p];
    }
}

}  // namespace

hipError_t launch_tail(int dim, bool f32, const TailArgs& a, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    dim3 grid(a.n);
#define TL(D, T)                                                                       \
    if (a.gmres)                                                                       \
        hipLaunchKernelGGL((k_tail<D, T, true>), grid, dim3(NTT), 0, s, a);             \
    else                                                                               \
        hipLaunchKernelGGL((k_tail<D, T, false>), grid, dim3(NTT), 0, s, a);
    if (dim == 2) {
        if (f32) {
            TL(2, float)
        } else {
            TL(2, double)
        }
    } else {
        if (f32) {
            TL(3, float)
        } else {
            TL(3, double)
        }
    }
#undef TL
    return hipGetLastError();
}

}  // namespace mg
