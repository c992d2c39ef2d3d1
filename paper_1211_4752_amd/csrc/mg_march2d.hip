// 2D GMRES(3) smoothing passes (Sec. 3.2.2) as row-marching wavefronts for
// gfx950.
//
// The minimiser of || q0 + c1 q1 + c2 q2 + c3 q3 ||, q_i = (A/s)^i r, comes
// from the Gram matrix of the q_i (mg_smooth.hip).  Here one wavefront owns
// a strip of MTX = 56 columns (lanes 4..59; 4 halo lanes on each side) and
// TY rows, and marches down the rows: every step takes one new row of the
// inputs and produces one new row of each power, each from the three most
// recent rows of the previous one held in registers; x-neighbours come from
// the adjacent lanes by DPP shifts.  Each input is read once per pass (plus
// the few warm-up rows and halo lanes, L2 hits), nothing but the outputs is
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
//
// Memory-level parallelism: the inputs of a row are loaded MAHEAD steps
// before the step that uses them, into a ring of register sets that the
// unrolled march indexes statically; every load is issued unconditionally
// (addresses clamped into the grid, values masked where they are used), so
// that no branch sits between a load and its use and the wait before a step
// covers only the loads of that step's row.  The coarse correction enters
// one coarse row (interpolated in x) every second fine row.  The y-axis
// coefficients of the strip's rows sit in a per-lane table (lane l: row
// y0 - YB + l) and are read with readlane, so the march makes no scalar
// loads.

#include <type_traits>

#include "mg_kcommon.hpp"

namespace mg {

using namespace kc;

namespace {

constexpr int MW = 64;              // lanes per wavefront = workgroup size
constexpr int MH = 4;               // halo lanes on the left
constexpr int MTX = MW - 2 * MH;    // owned columns per strip
constexpr int MAHEAD = 4;           // rows loaded ahead (even)
constexpr int YB = 8;               // first row of the y table: y0 - YB

__device__ __forceinline__ int imin(int a, int b) { return a < b ? a : b; }
__device__ __forceinline__ int iclamp(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

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

// Value of lane l (uniform l) to every lane.
__device__ __forceinline__ double rdlane(double v, int l) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffull), l);
    const int hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ float rdlane(float v, int l) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
template <typename T>
__device__ __forceinline__ cx<T> rdlane(cx<T> v, int l) {
    return mk<T>(rdlane(v.r, l), rdlane(v.i, l));
}

// Per-lane column data of a strip.
template <typename T>
struct Lane {
    int gx;       // column of the lane
    int gxc;      // the same, clamped into the grid (load addresses)
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
    c.gxc = iclamp(c.gx, 0, L.n[0] - 1);
    const cx<T> cm = L.cm[0][c.gxc], c0 = L.c0[0][c.gxc], cp = L.cp[0][c.gxc];
    const cx<T> Z = mk<T>(0, 0);
    c.cmx = c.colv ? cm : Z;
    c.c0x = c.colv ? c0 : Z;
    c.cpx = c.colv ? cp : Z;
    return c;
}

// y-axis coefficients of one row.
template <typename T>
struct YC {
    cx<T> c0, cm, cp;
};

// The table: lane l holds row y0 - YB + l (clamped into the grid).
template <typename T>
__device__ __forceinline__ YC<T> ytab_of(const GLevel<T>& L, int y0) {
    const int y = iclamp(y0 - YB + (int)threadIdx.x, 0, L.n[1] - 1);
    return YC<T>{L.c0[1][y], L.cm[1][y], L.cp[1][y]};
}

template <typename T>
__device__ __forceinline__ YC<T> yrow(const YC<T>& tab, int y0, int y) {
    const int l = y - (y0 - YB);
    return YC<T>{rdlane(tab.c0, l), rdlane(tab.cm, l), rdlane(tab.cp, l)};
}

// A at the row whose rows y-1, y, y+1 of the stage are am, a0, ap (this
// lane); every lane must call it (lane shifts).  Caller masks the result.
// d: the diagonal of that row at this lane.
template <typename T>
__device__ __forceinline__ cx<T> row_apply(const Lane<T>& c, const YC<T>& y, cx<T> d, cx<T> am, cx<T> a0, cx<T> ap) {
    const cx<T> left = shfl_up1(a0);
    const cx<T> right = shfl_dn1(a0);
    return cfma(y.cp, ap, cfma(y.cm, am, cfma(c.cpx, right, cfma(c.cmx, left, d * a0))));
}

// A register copy made exactly here.  The ring slot a value was loaded into
// dies at the copy, so the slot's next load can reuse its registers; left to
// itself the compiler may move the consumer of the slot past that load and
// then rotate the whole ring with copies that wait for every load.
__device__ __forceinline__ double pin(double v) {
    double r;
    asm volatile("v_mov_b64 %0, %1" : "=v"(r) : "v"(v));
    return r;
}
__device__ __forceinline__ float pin(float v) {
    float r;
    asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "v"(v));
    return r;
}

// Diagonal of row y at this lane (y-table entry yn of that row).
template <typename T>
__device__ __forceinline__ cx<T> row_diag(const GLevel<T>& L, const Lane<T>& c, const YC<T>& yn, T k2) {
    return c.c0x + yn.c0 - k2 * L.sigma;
}

template <typename T>
__device__ __forceinline__ bool rowv(const GLevel<T>& L, int y) {
    return y >= 0 && y < L.n[1];
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
__device__ __forceinline__ long long row_index(const GLevel<T>& L, const Lane<T>& c, int y) {
    return (long long)iclamp(y, 0, L.n[1] - 1) * L.n[0] + c.gxc;
}

// Inputs of one fine row at this lane, as loaded (masked where used).
// Pre-smoothing passes: q0 source and k^2, plus the incoming iterate (NZ).
template <typename T, typename TQ>
struct RowF {
    cx<TQ> f;
    T k2;
    cx<T> w;
};
// Post-smoothing passes: u1, f, k^2, plus out of row y - 3 (accumulating
// output pass; loaded after the step's store, so that the old value is dead
// when the new one is requested).
template <typename T, typename TF, typename TO>
struct RowU {
    cx<T> u;
    cx<TF> f;
    T k2;
    cx<TO> o;
};
// One coarse row of the correction at the lane's two interpolation columns.
template <typename T>
struct RowC {
    cx<T> e0, e1;
};

template <typename T, typename TQ, bool NZ>
__device__ __forceinline__ void load_f(RowF<T, TQ>& r, const GLevel<T>& L, const Lane<T>& c, GIn<cx<TQ>> f,
                                       GIn<cx<T>> w, int y) {
    const long long gi = row_index(L, c, y);
    r.f = f[gi];
    r.k2 = L.k2[gi];
    if constexpr (NZ) r.w = w[gi];
}

template <typename T, typename TF, typename TO>
__device__ __forceinline__ void load_u(RowU<T, TF, TO>& r, const GLevel<T>& L, const Lane<T>& c, GIn<cx<T>> u,
                                       GIn<cx<TF>> f, int y) {
    const long long gi = row_index(L, c, y);
    r.u = u[gi];
    r.f = f[gi];
    r.k2 = L.k2[gi];
}

template <typename T>
__device__ __forceinline__ void load_c(RowC<T>& r, const GLevel<T>& Lc, const InterpX<T>& ix, GIn<cx<T>> e, int J) {
    const long long b = (long long)iclamp(J, 0, Lc.n[1] - 1) * Lc.n[0];
    r.e0 = e[b + ix.i0];
    r.e1 = e[b + ix.i1];
}

// x-interpolated coarse row J (zero outside the coarse grid).
template <typename T>
__device__ __forceinline__ cx<T> ex_of(const RowC<T>& r, const GLevel<T>& Lc, const InterpX<T>& ix, int J) {
    const cx<T> v = ix.w0 * r.e0 + ix.w1 * r.e1;
    return (J >= 0 && J < Lc.n[1]) ? v : mk<T>(0, 0);
}

// The coarse correction interpolated to the fine rows of a march that
// starts at row tb: coarse row J = t / 2 enters at every even fine row t,
// MAHEAD / 2 coarse rows ahead.  PAR = tb & 1 (static: strips start at even
// rows).  The even steps of an unrolled group of MAHEAD steps are i = 2k + PAR.
template <typename T, int PAR>
struct CoarseRing {
    static constexpr int PC = MAHEAD / 2;
    RowC<T> pc[PC];
    cx<T> exA, exB;   // coarse rows floor(t/2) - 1 and floor(t/2)

    // Set-up, in the order of the loads in the march: the coarse row before
    // the first fine row (first), then per step of the first group the coarse
    // row that the step would load (prime<I>), then finish.
    __device__ __forceinline__ void first(RowC<T>& r0, const GLevel<T>& Lc, const InterpX<T>& ix, GIn<cx<T>> e,
                                          int tb) {
        load_c(r0, Lc, ix, e, (tb - 1) >> 1);
    }
    template <int I>
    __device__ __forceinline__ void prime(const GLevel<T>& Lc, const InterpX<T>& ix, GIn<cx<T>> e, int tb) {
        if constexpr (((I + PAR) & 1) == 0) load_c(pc[(I - PAR) / 2], Lc, ix, e, ((tb + PAR) >> 1) + (I - PAR) / 2);
    }
    __device__ __forceinline__ void finish(const RowC<T>& r0, const GLevel<T>& Lc, const InterpX<T>& ix, int tb) {
        exB = ex_of(r0, Lc, ix, (tb - 1) >> 1);
        exA = mk<T>(0, 0);
    }
    // correction at fine row t = t0 + i (i static)
    template <int I>
    __device__ __forceinline__ cx<T> step(const GLevel<T>& Lc, const InterpX<T>& ix, GIn<cx<T>> e, int t) {
        if constexpr (((I + PAR) & 1) == 0) {
            constexpr int k = (I - PAR) / 2;
            const int J = t >> 1;
            exA = exB;
            exB = ex_of(pc[k], Lc, ix, J);
            load_c(pc[k], Lc, ix, e, J + PC);
            return T(0.5) * (exA + exB);
        } else {
            return exB;
        }
    }
};

template <int N>
struct IntC {
    static constexpr int v = N;
};

// Static unroll: f(IntC<0>), ..., f(IntC<N-1>).
template <int I, int N, typename F>
__device__ __forceinline__ void unroll(F&& f) {
    if constexpr (I < N) {
        f(IntC<I>{});
        unroll<I + 1, N>(f);
    }
}

__device__ __forceinline__ int round_up(int v, int m) { return (v + m - 1) / m * m; }

// Register rings of the march: a value produced at step t sits in slot
// (t - tb) mod MAHEAD, so in a group of MAHEAD unrolled steps every slot
// index is static and the rotating rows need no register moves.  RI<I, K>:
// slot of the value produced K steps before step I of the group.
template <int I, int K>
constexpr int RI = ((I - K) % MAHEAD + MAHEAD) % MAHEAD;

template <typename T, typename TQ>
__device__ __forceinline__ GIn<cx<TQ>> q0_source(const CycleSlot& sl, const SmoothBufs& B) {
    // The q0 buffer (sl.f null: level 0 with an incoming iterate) is FP64,
    // which only FP64 passes read.
    if constexpr (std::is_same<T, TQ>::value)
        return gin(static_cast<const cx<TQ>*>(sl.f ? sl.f : B.q[0]));
    else
        return gin(static_cast<const cx<TQ>*>(sl.f));
}

// ---------------------------------------------------------------------------
// Gram pass.  Step t takes row t of the first stage and produces, of the
// chain S0 -> S1 -> ..., row t - k of stage k; the Gram products are taken
// at the row where the last power is formed.
// ---------------------------------------------------------------------------
template <typename T, typename TQ, bool POST, int TY>
__global__ void __launch_bounds__(MW) k_mg_gram(const CycleArgs a, cx<double>* part, int pstride, int bstride) {
    static_assert(TY % 2 == 0 && MAHEAD % 2 == 0 && TY + MAHEAD + 11 <= MW, "strip geometry");
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
    const YC<T> yt = ytab_of(L, y0);
    const T fs = (T)fscale_of(sl);
    const cx<T> Z = mk<T>(0, 0);
    cx<double> g[NUM_GRAM];
#pragma unroll
    for (int v = 0; v < NUM_GRAM; ++v) g[v] = mk(0.0, 0.0);
    const int yend = imin(y0 + TY, L.n[1]);
    auto ok = [&](int y) { return c.colv && rowv(L, y); };

    if constexpr (POST) {
        InterpX<T> ix;
        interp_axis<T>(c.gxc, Lc.n[0], ix.i0, ix.i1, ix.w0, ix.w1);
        const auto u1 = gin(static_cast<const cx<T>*>(B.u1));
        const auto ev = gin(static_cast<const cx<T>*>(sl.c));
        const auto fv = gin(static_cast<const cx<TQ>*>(sl.f));
        // rings by producing step: u2 of row s (A), fscale f of row s (F), q0 of
        // row s-1 (Bq), q1 of row s-2 (Cq), q2 of row s-3 (Dq), diagonal and
        // y coefficients of row s (DD, Y); the diagonal and y coefficients of
        // row t-4 are taken out of their slot before row t replaces them
        cx<T> A[MAHEAD], F[MAHEAD], Bq[MAHEAD], Cq[MAHEAD], Dq[MAHEAD], DD[MAHEAD];
        YC<T> Y[MAHEAD];
#pragma unroll
        for (int k = 0; k < MAHEAD; ++k) A[k] = F[k] = Bq[k] = Cq[k] = Dq[k] = DD[k] = Z;
        const int tb = y0 - 4;
        const int tn = tb + round_up(yend - y0 + 8, MAHEAD);
        RowU<T, TQ, T> pf[MAHEAD];
        CoarseRing<T, 0> cr;
        RowC<T> r0;
        cr.first(r0, Lc, ix, ev, tb);
        unroll<0, MAHEAD>([&](auto I) {
            constexpr int i = decltype(I)::v;
            cr.template prime<i>(Lc, ix, ev, tb);
            load_u<T, TQ, T>(pf[i], L, c, u1, fv, tb + i);
            __builtin_amdgcn_sched_barrier(0);
        });
        cr.finish(r0, Lc, ix, tb);
#pragma unroll
        for (int k = 0; k < MAHEAD; ++k) Y[k] = yrow(yt, y0, tb - MAHEAD + k);
        int t0 = tb;   // at least one group: the march has at least 6 steps
        do {
            unroll<0, MAHEAD>([&](auto I) {
                constexpr int i = decltype(I)::v;
                const int t = t0 + i;
                const cx<T> ey = cr.template step<i>(Lc, ix, ev, t);
                A[RI<i, 0>] = ok(t) ? pf[i].u + ey : Z;
                const cx<T> dd4 = DD[RI<i, 0>];
                const YC<T> y4 = Y[RI<i, 0>];
                Y[RI<i, 0>] = yrow(yt, y0, t);
                DD[RI<i, 0>] = row_diag(L, c, Y[RI<i, 0>], pin(pf[i].k2));
                F[RI<i, 0>] = fs * cvt<T>(pf[i].f);
                __builtin_amdgcn_sched_barrier(0);   // the ring slot is consumed before it is reloaded
                load_u<T, TQ, T>(pf[i], L, c, u1, fv, t + MAHEAD);
                cx<T> v = row_apply<T>(c, Y[RI<i, 1>], DD[RI<i, 1>], A[RI<i, 2>], A[RI<i, 1>], A[RI<i, 0>]);
                Bq[RI<i, 0>] = ok(t - 1) ? F[RI<i, 1>] - v : Z;
                v = row_apply<T>(c, Y[RI<i, 2>], DD[RI<i, 2>], Bq[RI<i, 2>], Bq[RI<i, 1>], Bq[RI<i, 0>]);
                Cq[RI<i, 0>] = ok(t - 2) ? L.sinv * v : Z;
                v = row_apply<T>(c, Y[RI<i, 3>], DD[RI<i, 3>], Cq[RI<i, 2>], Cq[RI<i, 1>], Cq[RI<i, 0>]);
                Dq[RI<i, 0>] = ok(t - 3) ? L.sinv * v : Z;
                v = row_apply<T>(c, y4, dd4, Dq[RI<i, 2>], Dq[RI<i, 1>], Dq[RI<i, 0>]);
                const int yr = t - 4;
                if (c.own && yr >= y0 && yr < yend) gram_add<T>(g, Bq[RI<i, 3>], Cq[RI<i, 2>], Dq[RI<i, 1>], L.sinv * v);
            });
            t0 += MAHEAD;
        } while (t0 < tn);
    } else {
        // rings by producing step: q0 of row s (A), q1 of row s-1 (Bq), q2 of
        // row s-2 (Cq), diagonal and y coefficients of row s (DD, Y)
        const GIn<cx<TQ>> src = q0_source<T, TQ>(sl, B);
        const T qs = sl.f ? fs : T(1);
        const GIn<cx<T>> none{};
        cx<T> A[MAHEAD], Bq[MAHEAD], Cq[MAHEAD], DD[MAHEAD];
        YC<T> Y[MAHEAD];
#pragma unroll
        for (int k = 0; k < MAHEAD; ++k) A[k] = Bq[k] = Cq[k] = DD[k] = Z;
        const int tb = y0 - 3;
        const int tn = tb + round_up(yend - y0 + 6, MAHEAD);
        RowF<T, TQ> pf[MAHEAD];
#pragma unroll
        for (int i = 0; i < MAHEAD; ++i) {
            load_f<T, TQ, false>(pf[i], L, c, src, none, tb + i);
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int k = 0; k < MAHEAD; ++k) Y[k] = yrow(yt, y0, tb - MAHEAD + k);
        int t0 = tb;   // at least one group: the march has at least 6 steps
        do {
            unroll<0, MAHEAD>([&](auto I) {
                constexpr int i = decltype(I)::v;
                const int t = t0 + i;
                A[RI<i, 0>] = ok(t) ? qs * cvt<T>(pf[i].f) : Z;
                Y[RI<i, 0>] = yrow(yt, y0, t);
                DD[RI<i, 0>] = row_diag(L, c, Y[RI<i, 0>], pin(pf[i].k2));
                __builtin_amdgcn_sched_barrier(0);   // the ring slot is consumed before it is reloaded
                load_f<T, TQ, false>(pf[i], L, c, src, none, t + MAHEAD);
                cx<T> v = row_apply<T>(c, Y[RI<i, 1>], DD[RI<i, 1>], A[RI<i, 2>], A[RI<i, 1>], A[RI<i, 0>]);
                Bq[RI<i, 0>] = ok(t - 1) ? L.sinv * v : Z;
                v = row_apply<T>(c, Y[RI<i, 2>], DD[RI<i, 2>], Bq[RI<i, 2>], Bq[RI<i, 1>], Bq[RI<i, 0>]);
                Cq[RI<i, 0>] = ok(t - 2) ? L.sinv * v : Z;
                v = row_apply<T>(c, Y[RI<i, 3>], DD[RI<i, 3>], Cq[RI<i, 2>], Cq[RI<i, 1>], Cq[RI<i, 0>]);
                const int yr = t - 3;
                if (c.own && yr >= y0 && yr < yend)
                    gram_add<T>(g, A[RI<i, 3>], Bq[RI<i, 2>], Cq[RI<i, 1>], L.sinv * v);
            });
            t0 += MAHEAD;
        } while (t0 < tn);
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
template <typename T, typename TQ, bool NZ, int TY, bool FC>
__global__ void __launch_bounds__(MW) k_mg_apply_restrict(const CycleArgs a) {
    static_assert(TY % 2 == 0 && MAHEAD % 2 == 0 && TY + MAHEAD + 11 <= MW, "strip geometry");
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
    const YC<T> yt = ytab_of(L, y0);
    const T fs = (T)fscale_of(sl);
    const GIn<cx<TQ>> src = q0_source<T, TQ>(sl, B);
    const T qs = sl.f ? fs : T(1);
    const auto up = gin(static_cast<const cx<T>*>(sl.u));
    const auto u1p = gout(static_cast<cx<T>*>(B.u1));
    const auto fc = gout(static_cast<cx<T>*>(sl.c));
    const int ncx = Lc.n[0], ncy = Lc.n[1];
    cx<T> c1, cc2, cc3;
    if (FC && slot_tiles(a, slot) <= FUSED_COEF_TILES) {   // from the Gram partials (coarse levels)
        CoefLoad cl;
        coef_load(a, slot, cl);
        cx<double> co[4];
        coef_solve(cl, a.gbrk, co);
        c1 = cvt<T>(co[0]), cc2 = cvt<T>(co[1]), cc3 = cvt<T>(co[2]);
    } else {
        c1 = cvt<T>(B.coef[0]), cc2 = cvt<T>(B.coef[1]), cc3 = cvt<T>(B.coef[2]);
    }
    const cx<T> Z = mk<T>(0, 0);
    const int yend = imin(y0 + TY, ny);
    // restriction centres of this strip: odd gx among the owned lanes
    const bool ccol = c.own && (c.gx & 1) && (c.gx - 1) / 2 < ncx;
    auto ok = [&](int y) { return c.colv && rowv(L, y); };

    // rings by producing step: q0 and the incoming iterate of row s (A, W),
    // q1 of row s-1 (Bq), q2 of row s-2 (Cq), r1 of row s-3 (Rr), diagonal
    // and y coefficients of row s (DD, Y)
    cx<T> A[MAHEAD], W[MAHEAD], Bq[MAHEAD], Cq[MAHEAD], Rr[MAHEAD], DD[MAHEAD];
    YC<T> Y[MAHEAD];
#pragma unroll
    for (int k = 0; k < MAHEAD; ++k) A[k] = W[k] = Bq[k] = Cq[k] = Rr[k] = DD[k] = Z;
    const int tb = y0 - 3;
    const int tn = tb + round_up(yend - y0 + 7, MAHEAD);
    RowF<T, TQ> pf[MAHEAD];
#pragma unroll
    for (int i = 0; i < MAHEAD; ++i) {
        load_f<T, TQ, NZ>(pf[i], L, c, src, up, tb + i);
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int k = 0; k < MAHEAD; ++k) Y[k] = yrow(yt, y0, tb - MAHEAD + k);
    int t0 = tb;   // at least one group: the march has at least 6 steps
    do {
        unroll<0, MAHEAD>([&](auto I) {
            constexpr int i = decltype(I)::v;
            const int t = t0 + i;
            A[RI<i, 0>] = ok(t) ? qs * cvt<T>(pf[i].f) : Z;
            if constexpr (NZ) W[RI<i, 0>] = mk<T>(pin(pf[i].w.r), pin(pf[i].w.i));
            Y[RI<i, 0>] = yrow(yt, y0, t);
            DD[RI<i, 0>] = row_diag(L, c, Y[RI<i, 0>], pin(pf[i].k2));
            __builtin_amdgcn_sched_barrier(0);   // the ring slot is consumed before it is reloaded
            load_f<T, TQ, NZ>(pf[i], L, c, src, up, t + MAHEAD);
            cx<T> v = row_apply<T>(c, Y[RI<i, 1>], DD[RI<i, 1>], A[RI<i, 2>], A[RI<i, 1>], A[RI<i, 0>]);
            Bq[RI<i, 0>] = ok(t - 1) ? L.sinv * v : Z;
            v = row_apply<T>(c, Y[RI<i, 2>], DD[RI<i, 2>], Bq[RI<i, 2>], Bq[RI<i, 1>], Bq[RI<i, 0>]);
            Cq[RI<i, 0>] = ok(t - 2) ? L.sinv * v : Z;
            v = row_apply<T>(c, Y[RI<i, 3>], DD[RI<i, 3>], Cq[RI<i, 2>], Cq[RI<i, 1>], Cq[RI<i, 0>]);
            // row t - 3: its q0, q1, q2 are A[RI<i, 3>], Bq[RI<i, 2>], Cq[RI<i, 1>]
            const int yr = t - 3;
            const bool m3 = ok(yr);
            const cx<T> q0 = A[RI<i, 3>], q1 = Bq[RI<i, 2>], q2 = Cq[RI<i, 1>];
            const cx<T> q3 = m3 ? L.sinv * v : Z;
            Rr[RI<i, 0>] = masked(m3, cfma(cc3, q3, cfma(cc2, q2, cfma(c1, q1, q0))));
            if (c.own && yr >= y0 && yr < yend) {
                cx<T> u = L.sinv * cfma(cc3, q2, cfma(cc2, q1, c1 * q0));
                if constexpr (NZ) u = W[RI<i, 3>] - u;
                else u = Z - u;
                u1p[(long long)yr * nx + c.gx] = u;
            }
            // the coarse row centred at fine row t - 4 exists when that row is
            // odd: at the even steps of a group (strips start at even rows,
            // so every group starts at an odd t)
            if constexpr ((i & 1) == 0) {
                const int yc = yr - 1;
                const cx<T> vv = T(0.25) * Rr[RI<i, 2>] + T(0.5) * Rr[RI<i, 1>] + T(0.25) * Rr[RI<i, 0>];
                const cx<T> vl = shfl_up1(vv), vr = shfl_dn1(vv);
                if (yc >= y0 && yc < yend && (yc - 1) / 2 < ncy && ccol) {
                    const int C = (yc - 1) / 2, Cx = (c.gx - 1) / 2;
                    fc[(long long)C * ncx + Cx] = T(0.25) * vl + T(0.5) * vv + T(0.25) * vr;
                }
            }
        });
        t0 += MAHEAD;
    } while (t0 < tn);
}

// ---------------------------------------------------------------------------
// Post-smoothing apply: u2 rows t..t-3, q0 rows t-1..t-3, q1 rows t-2..t-4,
// q2 at row t-3; out at row t - 3.
// ---------------------------------------------------------------------------
template <typename T, typename TF, typename TO, bool ACC, int TY, bool FC>
__global__ void __launch_bounds__(MW) k_mg_apply_out(const CycleArgs a) {
    static_assert(TY % 2 == 0 && MAHEAD % 2 == 0 && TY + MAHEAD + 11 <= MW, "strip geometry");
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
    const YC<T> yt = ytab_of(L, y0);
    InterpX<T> ix;
    interp_axis<T>(c.gxc, Lc.n[0], ix.i0, ix.i1, ix.w0, ix.w1);
    const T fs = (T)fscale_of(sl);
    const auto u1 = gin(static_cast<const cx<T>*>(B.u1));
    const auto ev = gin(static_cast<const cx<T>*>(sl.c));
    const auto fv = gin(static_cast<const cx<TF>*>(sl.f));
    const auto out = gout(static_cast<cx<TO>*>(sl.out));
    const auto outr = gin(static_cast<const cx<TO>*>(sl.out));
    cx<T> c1, cc2, cc3;
    if (FC && slot_tiles(a, slot) <= FUSED_COEF_TILES) {   // from the Gram partials (coarse levels)
        CoefLoad cl;
        coef_load(a, slot, cl);
        cx<double> co[4];
        coef_solve(cl, a.gbrk, co);
        c1 = cvt<T>(co[0]), cc2 = cvt<T>(co[1]), cc3 = cvt<T>(co[2]);
    } else {
        c1 = cvt<T>(B.coef[4]), cc2 = cvt<T>(B.coef[5]), cc3 = cvt<T>(B.coef[6]);
    }
    const cx<T> Z = mk<T>(0, 0);
    const int yend = imin(y0 + TY, ny);
    auto ok = [&](int y) { return c.colv && rowv(L, y); };

    // rings by producing step: u2 and fscale f of row s (A, F), q0 of row
    // s-1 (Bq), q1 of row s-2 (Cq), diagonal and y coefficients of row s
    // (DD, Y)
    cx<T> A[MAHEAD], F[MAHEAD], Bq[MAHEAD], Cq[MAHEAD], DD[MAHEAD];
    YC<T> Y[MAHEAD];
#pragma unroll
    for (int k = 0; k < MAHEAD; ++k) A[k] = F[k] = Bq[k] = Cq[k] = DD[k] = Z;
    const int tb = y0 - 3;
    const int tn = tb + round_up(yend - y0 + 6, MAHEAD);
    RowU<T, TF, TO> pf[MAHEAD];
    CoarseRing<T, 1> cr;
    RowC<T> r0;
    cr.first(r0, Lc, ix, ev, tb);
    unroll<0, MAHEAD>([&](auto I) {
        constexpr int i = decltype(I)::v;
        cr.template prime<i>(Lc, ix, ev, tb);
        load_u<T, TF, TO>(pf[i], L, c, u1, fv, tb + i);
        if constexpr (ACC) pf[i].o = outr[row_index(L, c, tb + i - 3)];
        __builtin_amdgcn_sched_barrier(0);
    });
    cr.finish(r0, Lc, ix, tb);
#pragma unroll
    for (int k = 0; k < MAHEAD; ++k) Y[k] = yrow(yt, y0, tb - MAHEAD + k);
    int t0 = tb;   // at least one group: the march has at least 6 steps
    do {
        unroll<0, MAHEAD>([&](auto I) {
            constexpr int i = decltype(I)::v;
            const int t = t0 + i;
            const cx<T> ey = cr.template step<i>(Lc, ix, ev, t);
            A[RI<i, 0>] = ok(t) ? pf[i].u + ey : Z;
            Y[RI<i, 0>] = yrow(yt, y0, t);
            DD[RI<i, 0>] = row_diag(L, c, Y[RI<i, 0>], pin(pf[i].k2));
            F[RI<i, 0>] = fs * cvt<T>(pf[i].f);
            __builtin_amdgcn_sched_barrier(0);   // the ring slot is consumed before it is reloaded
            load_u<T, TF, TO>(pf[i], L, c, u1, fv, t + MAHEAD);
            cx<T> v = row_apply<T>(c, Y[RI<i, 1>], DD[RI<i, 1>], A[RI<i, 2>], A[RI<i, 1>], A[RI<i, 0>]);
            Bq[RI<i, 0>] = ok(t - 1) ? F[RI<i, 1>] - v : Z;
            v = row_apply<T>(c, Y[RI<i, 2>], DD[RI<i, 2>], Bq[RI<i, 2>], Bq[RI<i, 1>], Bq[RI<i, 0>]);
            Cq[RI<i, 0>] = ok(t - 2) ? L.sinv * v : Z;
            v = row_apply<T>(c, Y[RI<i, 3>], DD[RI<i, 3>], Cq[RI<i, 2>], Cq[RI<i, 1>], Cq[RI<i, 0>]);
            const int yr = t - 3;
            if (c.own && yr >= y0 && yr < yend) {
                const long long gi = (long long)yr * nx + c.gx;
                const cx<T> q2 = L.sinv * v;
                const cx<T> w = A[RI<i, 3>] - L.sinv * cfma(cc3, q2, cfma(cc2, Cq[RI<i, 1>], c1 * Bq[RI<i, 2>]));
                if constexpr (ACC)
                    out[gi] = pf[i].o + cvt<TO>(w);
                else
                    out[gi] = cvt<TO>(w);
            }
            __builtin_amdgcn_sched_barrier(0);   // the ring slot is consumed before it is reloaded
            if constexpr (ACC) pf[i].o = outr[row_index(L, c, t + MAHEAD - 3)];
        });
        t0 += MAHEAD;
    } while (t0 < tn);
}

}  // namespace


// ---------------------------------------------------------------------------
// Geometry and launchers
// ---------------------------------------------------------------------------
namespace {
constexpr int MARCH_TY[MARCH_TILE] = {32, 16, 8, 4};
}

void march_counts(int shape, const int n[3], int nt[3]) {
    if (shape == MARCH_TILE) {
        tile2d_counts(n, nt);
        return;
    }
    if (shape < 0 || shape >= MARCH_TILE) shape = 0;
    nt[0] = (n[0] + MTX - 1) / MTX;
    nt[1] = (n[1] + MARCH_TY[shape] - 1) / MARCH_TY[shape];
    nt[2] = 1;
}

#define MG_MARCH_SWITCH(LAUNCH)         \
    switch (shape) {                    \
        case 1: LAUNCH(16); break;      \
        case 2: LAUNCH(8); break;       \
        case 3: LAUNCH(4); break;       \
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
    if (shape == MARCH_TILE) return tile2d_gram(f32, level0, post, a, part, pstride, bstride, s);
    if (!f32)
        return post ? mg_gram_launch<double, double, true>(shape, a, part, pstride, bstride, s)
                    : mg_gram_launch<double, double, false>(shape, a, part, pstride, bstride, s);
    if (level0)
        return post ? mg_gram_launch<float, double, true>(shape, a, part, pstride, bstride, s)
                    : mg_gram_launch<float, double, false>(shape, a, part, pstride, bstride, s);
    return post ? mg_gram_launch<float, float, true>(shape, a, part, pstride, bstride, s)
                : mg_gram_launch<float, float, false>(shape, a, part, pstride, bstride, s);
}

template <typename T, typename TQ, bool NZ, bool FC = false>
static hipError_t mg_ar_launch(int shape, const CycleArgs& a, hipStream_t s) {
#define AL(TY) hipLaunchKernelGGL((k_mg_apply_restrict<T, TQ, NZ, TY, FC>), dim3(a.st.ntiles), dim3(MW), 0, s, a);
    MG_MARCH_SWITCH(AL)
#undef AL
    return hipGetLastError();
}

hipError_t launch_sm2_apply_restrict(bool f32, bool level0, bool nonzero, int shape, const CycleArgs& a,
                                     hipStream_t s) {
    if (a.st.n <= 0) return hipSuccess;
    if (shape == MARCH_TILE) return tile2d_apply_restrict(f32, level0, nonzero, a, s);
    if (a.gpart) {   // coarse levels: zero iterate, vectors in the compute precision
        if (level0 || nonzero) return hipErrorInvalidValue;
        return f32 ? mg_ar_launch<float, float, false, true>(shape, a, s)
                   : mg_ar_launch<double, double, false, true>(shape, a, s);
    }
    if (!f32)
        return nonzero ? mg_ar_launch<double, double, true>(shape, a, s) : mg_ar_launch<double, double, false>(shape, a, s);
    if (nonzero) return hipErrorInvalidValue;
    return level0 ? mg_ar_launch<float, double, false>(shape, a, s) : mg_ar_launch<float, float, false>(shape, a, s);
}

template <typename T, typename TF, typename TO, bool ACC, bool FC = false>
static hipError_t mg_ao_launch(int shape, const CycleArgs& a, hipStream_t s) {
#define OL(TY) hipLaunchKernelGGL((k_mg_apply_out<T, TF, TO, ACC, TY, FC>), dim3(a.st.ntiles), dim3(MW), 0, s, a);
    MG_MARCH_SWITCH(OL)
#undef OL
    return hipGetLastError();
}

hipError_t launch_sm2_apply_out(bool f32, bool level0, bool accumulate, int shape, const CycleArgs& a, hipStream_t s) {
    if (a.st.n <= 0) return hipSuccess;
    if (shape == MARCH_TILE) return tile2d_apply_out(f32, level0, accumulate, a, s);
    if (a.gpart) {   // coarse levels
        if (level0 || accumulate) return hipErrorInvalidValue;
        return f32 ? mg_ao_launch<float, float, float, false, true>(shape, a, s)
                   : mg_ao_launch<double, double, double, false, true>(shape, a, s);
    }
    if (!f32)
        return accumulate ? mg_ao_launch<double, double, double, true>(shape, a, s)
                          : mg_ao_launch<double, double, double, false>(shape, a, s);
    if (level0)
        return accumulate ? mg_ao_launch<float, double, double, true>(shape, a, s)
                          : mg_ao_launch<float, double, double, false>(shape, a, s);
    return mg_ao_launch<float, float, float, false>(shape, a, s);
}

}  // namespace mg
