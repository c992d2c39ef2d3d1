// The coarse tail of the V-cycle (Sec. 3.1) in one launch: every level of at
// most TAIL_POINTS points, the coarsest direct solve and the way back up, one
// 1024-thread workgroup per right-hand side.  The vectors of levels of at
// most SMALL_POINTS points (right-hand sides, iterates, corrections, the
// smoother's powers) live in LDS and each thread holds its point's stencil
// coefficients in registers through a level's passes; a larger first tail
// level (up to PPT points per thread) keeps its vectors in global memory.
// Levels of at most 64 points, the coarsest solve among them, run in the
// first wavefront alone, with no workgroup barriers.  The coarsest solve
// multiplies by the inverse of the coarsest operator, formed in FP64 at
// set-up.  Smoothing is omega-Jacobi (Sec. 3.2.1) or one GMRES(3) step
// (Sec. 3.2.2) with the minimiser from the Gram matrix of the scaled power
// basis; the Gram reduction needs one workgroup barrier, after which every
// thread forms the coefficients itself.
//
// Level descriptors are copied into registers once per level, and every
// vector is reached through a typed view (LDS or global), so that no memory
// access goes through a generic pointer.

#include "mg_kcommon.hpp"

namespace mg {

using namespace kc;

namespace {

constexpr int NTT = 1024;
constexpr int NWAVE = NTT / 64;
constexpr int MAX_TAIL_LEVELS = 16;
constexpr int PPT = TAIL_POINTS / NTT;   // points per thread on the tail level in global memory
constexpr int WAVE_POINTS = 64;          // levels this small run in the first wavefront alone

template <int D>
__device__ __forceinline__ void pos3(int p, int nx, int ny, int& gx, int& gy, int& gz) {
    gx = p % nx;
    const int rr = p / nx;
    gy = rr % ny;
    gz = (D == 3) ? rr / ny : 0;
}

// A vector in LDS (pointer into the kernel's shared arrays).
template <typename T>
struct LVec {
    cx<T>* p;
    __device__ __forceinline__ cx<T> operator[](int i) const { return p[i]; }
    __device__ __forceinline__ void set(int i, cx<T> v) const { p[i] = v; }
};
// A vector in global memory.
template <typename T>
struct GVec {
    gptr<cx<T>> p;
    __device__ __forceinline__ cx<T> operator[](int i) const { return GVal<cx<T>>::get((gptr<const cx<T>>)(p + i)); }
    __device__ __forceinline__ void set(int i, cx<T> v) const { GVal<cx<T>>::put(p + i, v); }
};
template <typename T>
__device__ __forceinline__ GVec<T> gvec(void* p) {
    return GVec<T>{(gptr<cx<T>>)static_cast<cx<T>*>(p)};
}

// The vectors of one level.
template <typename V>
struct LvVec {
    V f, u, q0, q1, q2;
};

// Barrier of the level's participants: the workgroup, or nothing when the
// first wavefront runs the level alone (its LDS accesses stay in program
// order; the fence keeps the compiler from reordering them).
template <bool WAVE>
__device__ __forceinline__ void level_sync() {
    if constexpr (WAVE) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    } else {
        __syncthreads();
    }
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
template <int D, typename T, typename V>
__device__ __forceinline__ cx<T> prolong_at(const GLevel<T>& Lc, const V& e, int gx, int gy, int gz) {
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
            const int row = zz * sxy + yy * sx;
            v = v + (wz * wy * wx0) * e[row + x0] + (wz * wy * wx1) * e[row + x1];
        }
    }
    return v;
}

// Full weighting of r at coarse point (cx, cy, cz) of the next level.
template <int D, typename T, typename V>
__device__ __forceinline__ cx<T> restrict_at(const GLevel<T>& L, const V& r, int cx_, int cy, int cz) {
    const int nx = L.n[0], ny = L.n[1];
    cx<T> acc = mk<T>(0, 0);
#pragma unroll
    for (int oz = (D == 3 ? -1 : 0); oz <= (D == 3 ? 1 : 0); ++oz) {
        const T wz = (D == 3) ? (oz == 0 ? T(0.5) : T(0.25)) : T(1);
        const int zb = (D == 3) ? (2 * cz + 1 + oz) * nx * ny : 0;
#pragma unroll
        for (int oy = -1; oy <= 1; ++oy) {
            const T wy = wz * (oy == 0 ? T(0.5) : T(0.25));
            const int row = zb + (2 * cy + 1 + oy) * nx + 2 * cx_ + 1;
#pragma unroll
            for (int ox = -1; ox <= 1; ++ox) acc = acc + (wy * (ox == 0 ? T(0.5) : T(0.25))) * r[row + ox];
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
__device__ __forceinline__ PtCoef<T> pt_coef(const GLevel<T>& L, int p) {
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
template <int D, typename T, typename V>
__device__ __forceinline__ cx<T> apply_pt(const PtCoef<T>& c, const GLevel<T>& L, const V& x, int p, T sc) {
    const int nx = L.n[0], nxy = L.n[0] * L.n[1];
    cx<T> ax = c.d * x[p];
    if (c.gx > 0) ax = cfma(c.m[0], x[p - 1], ax);
    if (c.gx < nx - 1) ax = cfma(c.pl[0], x[p + 1], ax);
    if (c.gy > 0) ax = cfma(c.m[1], x[p - nx], ax);
    if (c.gy < L.n[1] - 1) ax = cfma(c.pl[1], x[p + nx], ax);
    if constexpr (D == 3) {
        if (c.gz > 0) ax = cfma(c.m[2], x[p - nxy], ax);
        if (c.gz < L.n[2] - 1) ax = cfma(c.pl[2], x[p + nxy], ax);
    }
    return sc * ax;
}

// (A x)(p) * sc reading the coefficients from global memory.
template <int D, typename T, typename V>
__device__ __forceinline__ cx<T> apply_gl(const GLevel<T>& L, const V& x, int p, T sc) {
    int gx, gy, gz;
    pos3<D>(p, L.n[0], L.n[1], gx, gy, gz);
    return stencil_at<D, T, T>(L, x, sc, (long long)p, gx, gy, gz);
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

__device__ __forceinline__ double rdlane(double v, int l) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffull), l);
    const int hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// The Gram matrix of the participants' partials and the coefficients of the
// minimising polynomial, returned to every thread.  WAVE: the first
// wavefront alone, which reduces and solves in registers.  Otherwise the
// waves holding points of the level (n points, ppt per thread) reduce their
// partials (n points), the first wavefront sums them in a fixed order and
// solves, and the coefficients reach the workgroup through LDS (two
// barriers).  sred
// holds NWAVE * NUM_GRAM + 4 complex values.
template <bool WAVE>
__device__ __forceinline__ void gram_coef(cx<double>* g, int n, double brk, cx<double>* sred, cx<double>* coef) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    cx<double> G[NUM_GRAM];
    if constexpr (WAVE) {
#pragma unroll
        for (int v = 0; v < NUM_GRAM; ++v) G[v] = mk(wave_sum(g[v].r), v < 4 ? 0.0 : wave_sum(g[v].i));
        solve_coef(G, brk, coef);
    } else {
        // waves with points: threadIdx.x < n (points threadIdx.x + i NTT)
        const int span = n < NTT ? n : NTT;
        const int nw = (span + 63) / 64;
        if (wave < nw) {
#pragma unroll
            for (int v = 0; v < NUM_GRAM; ++v) {
                const double r = wave_sum(g[v].r), i = v < 4 ? 0.0 : wave_sum(g[v].i);
                if (lane == 0) sred[wave * NUM_GRAM + v] = mk(r, i);
            }
        }
        __syncthreads();
        cx<double>* sc = sred + NWAVE * NUM_GRAM;
        if (wave == 0) {
            cx<double> t = mk(0.0, 0.0);
            if (lane < NUM_GRAM)
                for (int w = 0; w < nw; ++w) t = t + sred[w * NUM_GRAM + lane];
#pragma unroll
            for (int v = 0; v < NUM_GRAM; ++v) G[v] = mk(rdlane(t.r, v), rdlane(t.i, v));
            cx<double> c[4];
            solve_coef(G, brk, c);
            if (lane == 0) {
                sc[0] = c[0];
                sc[1] = c[1];
                sc[2] = c[2];
                sc[3] = c[3];
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 4; ++k) coef[k] = sc[k];
    }
}

// Pre-smoothing of a level (zero initial guess) and the restriction of its
// residual into fc.  NP points per thread (1: the point's coefficients in
// registers).  WAVE: run by the first wavefront alone.
template <int D, typename T, bool GM, int NP, bool WAVE, typename V, typename VC>
__device__ __forceinline__ void level_down(const GLevel<T>& L, const GLevel<T>& Lc, const LvVec<V>& v, const VC& fc,
                                           double brk, cx<double>* sred) {
    const int N = (int)L.N;
    constexpr int NT_ = WAVE ? 64 : NTT;
    PtCoef<T> pc;
    if constexpr (NP == 1)
        if ((int)threadIdx.x < N) pc = pt_coef<D, T>(L, threadIdx.x);
    auto A = [&](const V& x, int p, T s) -> cx<T> {
        if constexpr (NP == 1) return apply_pt<D, T>(pc, L, x, p, s);
        else return apply_gl<D, T>(L, x, p, s);
    };
    if constexpr (GM) {
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int p = threadIdx.x + i * NT_;
            if (p < N) v.q1.set(p, A(v.f, p, L.sinv));
        }
        level_sync<WAVE>();
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int p = threadIdx.x + i * NT_;
            if (p < N) v.q2.set(p, A(v.q1, p, L.sinv));
        }
        level_sync<WAVE>();
        cx<double> g[NUM_GRAM];
#pragma unroll
        for (int j = 0; j < NUM_GRAM; ++j) g[j] = mk(0.0, 0.0);
        cx<T> q3[NP];
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int p = threadIdx.x + i * NT_;
            q3[i] = mk<T>(0, 0);
            if (p < N) {
                q3[i] = A(v.q2, p, L.sinv);
                gram_add<T>(g, v.f[p], v.q1[p], v.q2[p], q3[i]);
            }
        }
        cx<double> co[4];
        gram_coef<WAVE>(g, N, brk, sred, co);
        const cx<T> c1 = cvt<T>(co[0]), c2 = cvt<T>(co[1]), c3 = cvt<T>(co[2]);
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int p = threadIdx.x + i * NT_;
            if (p < N) {
                const cx<T> q0 = v.f[p], q1 = v.q1[p], q2 = v.q2[p];
                v.u.set(p, mk<T>(0, 0) - L.sinv * (c1 * q0 + c2 * q1 + c3 * q2));
                v.q1.set(p, q0 + c1 * q1 + c2 * q2 + c3 * q3[i]);   // the new residual
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int p = threadIdx.x + i * NT_;
            if (p < N) {
                cx<T> d;
                if constexpr (NP == 1) d = pc.d;
                else {
                    int gx, gy, gz;
                    pos3<D>(p, L.n[0], L.n[1], gx, gy, gz);
                    d = diag_at<D>(L, gx, gy, gz, L.k2[p]);
                }
                v.u.set(p, cdiv(L.omega * v.f[p], d));
            }
        }
        level_sync<WAVE>();
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int p = threadIdx.x + i * NT_;
            if (p < N) v.q1.set(p, v.f[p] - A(v.u, p, T(1)));
        }
    }
    level_sync<WAVE>();
    for (int p = threadIdx.x; p < (int)Lc.N; p += NT_) {
        int cx_, cy, cz;
        pos3<D>(p, Lc.n[0], Lc.n[1], cx_, cy, cz);
        fc.set(p, restrict_at<D, T>(L, v.q1, cx_, cy, cz));
    }
    level_sync<WAVE>();
}

// Coarse-grid correction u2 = u1 + P ec and post-smoothing of a level; the
// correction of the level lands in v.u.
template <int D, typename T, bool GM, int NP, bool WAVE, typename V, typename VC>
__device__ __forceinline__ void level_up(const GLevel<T>& L, const GLevel<T>& Lc, const LvVec<V>& v, const VC& ec,
                                         double brk, cx<double>* sred) {
    const int N = (int)L.N;
    constexpr int NT_ = WAVE ? 64 : NTT;
    PtCoef<T> pc;
    if constexpr (NP == 1)
        if ((int)threadIdx.x < N) pc = pt_coef<D, T>(L, threadIdx.x);
    auto A = [&](const V& x, int p, T s) -> cx<T> {
        if constexpr (NP == 1) return apply_pt<D, T>(pc, L, x, p, s);
        else return apply_gl<D, T>(L, x, p, s);
    };
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        const int p = threadIdx.x + i * NT_;
        if (p < N) {
            int gx, gy, gz;
            pos3<D>(p, L.n[0], L.n[1], gx, gy, gz);
            v.u.set(p, v.u[p] + prolong_at<D, T>(Lc, ec, gx, gy, gz));
        }
    }
    level_sync<WAVE>();
    if constexpr (GM) {
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int p = threadIdx.x + i * NT_;
            if (p < N) v.q0.set(p, v.f[p] - A(v.u, p, T(1)));
        }
        level_sync<WAVE>();
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int p = threadIdx.x + i * NT_;
            if (p < N) v.q1.set(p, A(v.q0, p, L.sinv));
        }
        level_sync<WAVE>();
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int p = threadIdx.x + i * NT_;
            if (p < N) v.q2.set(p, A(v.q1, p, L.sinv));
        }
        level_sync<WAVE>();
        cx<double> g[NUM_GRAM];
#pragma unroll
        for (int j = 0; j < NUM_GRAM; ++j) g[j] = mk(0.0, 0.0);
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int p = threadIdx.x + i * NT_;
            if (p < N) gram_add<T>(g, v.q0[p], v.q1[p], v.q2[p], A(v.q2, p, L.sinv));
        }
        cx<double> co[4];
        gram_coef<WAVE>(g, N, brk, sred, co);
        const cx<T> c1 = cvt<T>(co[0]), c2 = cvt<T>(co[1]), c3 = cvt<T>(co[2]);
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int p = threadIdx.x + i * NT_;
            if (p < N) v.u.set(p, v.u[p] - L.sinv * (c1 * v.q0[p] + c2 * v.q1[p] + c3 * v.q2[p]));
        }
        level_sync<WAVE>();
    } else {
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int p = threadIdx.x + i * NT_;
            if (p < N) {
                cx<T> d;
                if constexpr (NP == 1) d = pc.d;
                else {
                    int gx, gy, gz;
                    pos3<D>(p, L.n[0], L.n[1], gx, gy, gz);
                    d = diag_at<D>(L, gx, gy, gz, L.k2[p]);
                }
                v.q0.set(p, v.u[p] + cdiv(L.omega * (v.f[p] - A(v.u, p, T(1))), d));
            }
        }
        level_sync<WAVE>();
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int p = threadIdx.x + i * NT_;
            if (p < N) v.u.set(p, v.q0[p]);
        }
        level_sync<WAVE>();
    }
}

// e = A^{-1} f on the coarsest level with the FP64 inverse.
template <typename T, bool WAVE>
__device__ __forceinline__ void coarsest(const GLevel<T>& C, const LVec<T>& f, const LVec<T>& u) {
    const int n = (int)C.N;
    constexpr int NT_ = WAVE ? 64 : NTT;
    for (int p = threadIdx.x; p < n; p += NT_) {
        cx<double> s = mk(0.0, 0.0);
        const long long row = (long long)p * n;
        int j = 0;
        for (; j + 8 <= n; j += 8) {   // eight independent loads in flight
            cx<double> m[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) m[k] = C.cinv[row + j + k];
#pragma unroll
            for (int k = 0; k < 8; ++k) s = s + m[k] * cvt<double>(f[j + k]);
        }
        for (; j < n; ++j) s = s + C.cinv[row + j] * cvt<double>(f[j]);
        u.set(p, cvt<T>(s));
    }
    level_sync<WAVE>();
}

template <int D, typename T, bool GM>
__global__ void __launch_bounds__(NTT) k_tail(const TailArgs a) {
    __shared__ cx<T> sf[TAIL_LDS];            // right-hand side of every LDS level
    __shared__ cx<T> su[TAIL_LDS];            // iterate, then correction, of every LDS level
    __shared__ cx<T> sq[3][SMALL_POINTS];     // powers / residuals of the LDS level in progress
    __shared__ cx<double> sred[NWAVE * NUM_GRAM + 4];
    const TailSlot ts = a.s[blockIdx.x];
    if (gated_off(ts.gate)) return;
    const LevelView<T>* Lv = static_cast<const LevelView<T>*>(ts.lv);
    const SmoothBufs* SB = ts.sb;
    const int last = ts.nlev - 1;
    const double brk = a.brk;
    // levels: an optional first one in global memory (more than SMALL_POINTS
    // points), then the LDS levels s0 .. last; levels kw .. last have at most
    // WAVE_POINTS points
    const int s0 = (last > 0 && Lv[0].N > SMALL_POINTS) ? 1 : 0;
    __shared__ int off[MAX_TAIL_LEVELS + 1];   // LDS offsets of the LDS levels
    int kw = last + 1;
    for (int k = s0; k <= last; ++k)
        if (Lv[k].N <= WAVE_POINTS) {
            kw = k;
            break;
        }
    if (threadIdx.x == 0) {
        off[s0] = 0;
        for (int k = s0; k <= last && k < MAX_TAIL_LEVELS; ++k) off[k + 1] = off[k] + (int)Lv[k].N;
    }
    __syncthreads();
    auto lds = [&](int k) -> LvVec<LVec<T>> {
        return LvVec<LVec<T>>{LVec<T>{sf + off[k]}, LVec<T>{su + off[k]}, LVec<T>{sq[0]}, LVec<T>{sq[1]},
                              LVec<T>{sq[2]}};
    };
    const bool w0 = threadIdx.x < 64;

    // down
    if (s0 == 1) {
        const SmoothBufs B = SB[0];
        const LvVec<GVec<T>> v{gvec<T>(B.f), gvec<T>(B.e), gvec<T>(B.q[0]), gvec<T>(B.q[1]), gvec<T>(B.q[2])};
        level_down<D, T, GM, PPT, false>(glevel(Lv[0]), glevel(Lv[1]), v, LVec<T>{sf + off[1]}, brk, sred);
    } else {
        const GVec<T> fg = gvec<T>(SB[0].f);
        for (int p = threadIdx.x; p < (int)Lv[0].N; p += NTT) sf[p] = fg[p];
        __syncthreads();
    }
    for (int k = s0; k < kw && k < last; ++k)
        level_down<D, T, GM, 1, false>(glevel(Lv[k]), glevel(Lv[k + 1]), lds(k), LVec<T>{sf + off[k + 1]}, brk, sred);
    if (kw <= last) {
        if (w0) {
            for (int k = kw; k < last; ++k)
                level_down<D, T, GM, 1, true>(glevel(Lv[k]), glevel(Lv[k + 1]), lds(k), LVec<T>{sf + off[k + 1]}, brk,
                                              sred);
            coarsest<T, true>(glevel(Lv[last]), LVec<T>{sf + off[last]}, LVec<T>{su + off[last]});
            for (int k = last - 1; k >= kw; --k)
                level_up<D, T, GM, 1, true>(glevel(Lv[k]), glevel(Lv[k + 1]), lds(k), LVec<T>{su + off[k + 1]}, brk,
                                            sred);
        }
        __syncthreads();
    } else {
        coarsest<T, false>(glevel(Lv[last]), LVec<T>{sf + off[last]}, LVec<T>{su + off[last]});
    }
    // up
    for (int k = (kw <= last ? kw : last) - 1; k >= s0; --k)
        level_up<D, T, GM, 1, false>(glevel(Lv[k]), glevel(Lv[k + 1]), lds(k), LVec<T>{su + off[k + 1]}, brk, sred);
    if (s0 == 1) {
        const SmoothBufs B = SB[0];
        const LvVec<GVec<T>> v{gvec<T>(B.f), gvec<T>(B.e), gvec<T>(B.q[0]), gvec<T>(B.q[1]), gvec<T>(B.q[2])};
        level_up<D, T, GM, PPT, false>(glevel(Lv[0]), glevel(Lv[1]), v, LVec<T>{su + off[1]}, brk, sred);
    } else {   // correction of the first tail level
        const GVec<T> eg = gvec<T>(SB[0].e);
        for (int p = threadIdx.x; p < (int)Lv[0].N; p += NTT) eg.set(p, su[p]);
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
