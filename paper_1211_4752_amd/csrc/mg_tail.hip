// The coarse tail of the V-cycle (Sec. 3.1) in one launch: every level of at
// most TAIL_POINTS points, the coarsest direct solve and the way back up, one
// 1024-thread workgroup per right-hand side, passes separated by workgroup
// barriers.  On these levels a pass is a few points per thread, so the cost
// of a cycle there is set by dependent steps, not bytes: one launch replaces
// about six per level.  Smoothing is omega-Jacobi (Sec. 3.2.1) or one GMRES(3)
// step (Sec. 3.2.2) with the minimiser from the Gram matrix of the scaled
// power basis, reduced inside the workgroup.

#include "mg_kcommon.hpp"

namespace mg {

using namespace kc;

namespace {

constexpr int NTT = 1024;
constexpr int PPT = TAIL_POINTS / NTT;   // points per thread on a tail level

// out[p] = fn(p) for the level's points: every value first, then every store,
// so that the loads of all of a thread's points are in flight together.
template <typename T, typename F>
__device__ __forceinline__ void map_store(int N, cx<T>* out, F fn) {
    cx<T> v[PPT];
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
        const int p = threadIdx.x + i * NTT;
        v[i] = p < N ? fn(p) : mk<T>(0, 0);
    }
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
        const int p = threadIdx.x + i * NTT;
        if (p < N) out[p] = v[i];
    }
}

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
    const long long sx = Lc.n[0], sxy = (long long)Lc.n[0] * Lc.n[1];
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
        const long long zb = (D == 3) ? (long long)(2 * cz + 1 + oz) * nx * ny : 0;
#pragma unroll
        for (int oy = -1; oy <= 1; ++oy) {
            const T wy = wz * (oy == 0 ? T(0.5) : T(0.25));
            const cx<T>* row = r + zb + (long long)(2 * cy + 1 + oy) * nx + 2 * cx_ + 1;
#pragma unroll
            for (int ox = -1; ox <= 1; ++ox) acc = acc + (wy * (ox == 0 ? T(0.5) : T(0.25))) * row[ox];
        }
    }
    return acc;
}

// Workgroup Gram matrix of (q0, q1, q2, q3 = (A/s) q2) and the coefficient
// solve; the coefficients land in sc[0..2] for every thread.
template <int D, typename T>
__device__ void tail_gram(const LevelView<T>& L, const cx<T>* q0, const cx<T>* q1, const cx<T>* q2, double brk,
                          cx<double>* sred, cx<double>* sc) {
    const int nx = L.n[0], ny = L.n[1];
    const int N = (int)L.N;
    cx<double> g[NUM_GRAM];
#pragma unroll
    for (int v = 0; v < NUM_GRAM; ++v) g[v] = mk(0.0, 0.0);
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
        const int p = threadIdx.x + i * NTT;
        if (p >= N) continue;
        int gx, gy, gz;
        pos3<D>(p, nx, ny, gx, gy, gz);
        const cx<double> v0 = cvt<double>(q0[p]), v1 = cvt<double>(q1[p]), v2 = cvt<double>(q2[p]);
        const cx<double> v3 = cvt<double>(L.sinv * stencil_at<D, T, T>(L, q2, T(1), p, gx, gy, gz));
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

template <int D, typename T, bool GM>
__global__ void __launch_bounds__(NTT) k_tail(const TailArgs a) {
    __shared__ cx<double> sred[(NTT / 64 + 1) * NUM_GRAM];
    __shared__ cx<double> sc[4];
    __shared__ cx<double> b[MAX_COARSE];
    const TailSlot& ts = a.s[blockIdx.x];
    if (gated_off(ts.gate)) return;
    const LevelView<T>* Lv = static_cast<const LevelView<T>*>(ts.lv);
    const SmoothBufs* SB = ts.sb;
    const int last = ts.nlev - 1;

    for (int k = 0; k < last; ++k) {
        const LevelView<T> L = Lv[k];
        const SmoothBufs B = SB[k];
        const int nx = L.n[0], ny = L.n[1], N = (int)L.N;
        const cx<T>* f = static_cast<const cx<T>*>(B.f);
        cx<T>* u1 = static_cast<cx<T>*>(B.u1);
        cx<T>* q1 = static_cast<cx<T>*>(B.q[1]);
        if constexpr (GM) {
            cx<T>* q2 = static_cast<cx<T>*>(B.q[2]);
            map_store<T>(N, q1, [&](int p) {
                int gx, gy, gz;
                pos3<D>(p, nx, ny, gx, gy, gz);
                return L.sinv * stencil_at<D, T, T>(L, f, T(1), p, gx, gy, gz);
            });
            __syncthreads();
            map_store<T>(N, q2, [&](int p) {
                int gx, gy, gz;
                pos3<D>(p, nx, ny, gx, gy, gz);
                return L.sinv * stencil_at<D, T, T>(L, q1, T(1), p, gx, gy, gz);
            });
            __syncthreads();
            tail_gram<D, T>(L, f, q1, q2, a.brk, sred, sc);
            const cx<T> c1 = cvt<T>(sc[0]), c2 = cvt<T>(sc[1]), c3 = cvt<T>(sc[2]);
            // u1 and the new residual (into q1, pointwise in place)
            cx<T> ru[PPT], rr[PPT];
#pragma unroll
            for (int i = 0; i < PPT; ++i) {
                const int p = threadIdx.x + i * NTT;
                ru[i] = rr[i] = mk<T>(0, 0);
                if (p < N) {
                    int gx, gy, gz;
                    pos3<D>(p, nx, ny, gx, gy, gz);
                    const cx<T> q0 = f[p], v1 = q1[p], v2 = q2[p];
                    const cx<T> v3 = L.sinv * stencil_at<D, T, T>(L, q2, T(1), p, gx, gy, gz);
                    ru[i] = mk<T>(0, 0) - L.sinv * (c1 * q0 + c2 * v1 + c3 * v2);
                    rr[i] = q0 + c1 * v1 + c2 * v2 + c3 * v3;
                }
            }
#pragma unroll
            for (int i = 0; i < PPT; ++i) {
                const int p = threadIdx.x + i * NTT;
                if (p < N) {
                    u1[p] = ru[i];
                    q1[p] = rr[i];
                }
            }
        } else {
            map_store<T>(N, u1, [&](int p) {
                int gx, gy, gz;
                pos3<D>(p, nx, ny, gx, gy, gz);
                return cdiv(L.omega * f[p], diag_at<D>(L, gx, gy, gz, L.k2[p]));
            });
            __syncthreads();
            map_store<T>(N, q1, [&](int p) {
                int gx, gy, gz;
                pos3<D>(p, nx, ny, gx, gy, gz);
                return f[p] - stencil_at<D, T, T>(L, u1, T(1), p, gx, gy, gz);
            });
        }
        __syncthreads();
        const LevelView<T> Lc = Lv[k + 1];
        cx<T>* fc = static_cast<cx<T>*>(SB[k + 1].f);
        const int Nc = (int)Lc.N;
        map_store<T>(Nc, fc, [&](int p) {
            int cx_, cy, cz;
            pos3<D>(p, Lc.n[0], Lc.n[1], cx_, cy, cz);
            return restrict_at<D, T>(L, q1, cx_, cy, cz);
        });
        __syncthreads();
    }

    // coarsest: LU forward/back substitution in FP64
    {
        const LevelView<T> C = Lv[last];
        const int n = (int)C.N;
        const cx<double>* lu = C.lu;
        const int* piv = C.piv;
        const cx<T>* f = static_cast<const cx<T>*>(SB[last].f);
        cx<T>* e = static_cast<cx<T>*>(SB[last].e);
        for (int i = threadIdx.x; i < n; i += NTT) b[i] = cvt<double>(f[i]);
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int i = 0; i < n; ++i) {
                const int p = piv[i];
                if (p != i) {
                    const cx<double> tmp = b[i];
                    b[i] = b[p];
                    b[p] = tmp;
                }
            }
        }
        __syncthreads();
        for (int k = 0; k < n; ++k) {
            const cx<double> bk = b[k];
            for (int i = k + 1 + threadIdx.x; i < n; i += NTT) b[i] = b[i] - lu[(long long)i * n + k] * bk;
            __syncthreads();
        }
        for (int k = n - 1; k >= 0; --k) {
            if (threadIdx.x == 0) b[k] = cdiv(b[k], lu[(long long)k * n + k]);
            __syncthreads();
            const cx<double> bk = b[k];
            for (int i = threadIdx.x; i < k; i += NTT) b[i] = b[i] - lu[(long long)i * n + k] * bk;
            __syncthreads();
        }
        for (int i = threadIdx.x; i < n; i += NTT) e[i] = cvt<T>(b[i]);
        __syncthreads();
    }

    for (int k = last - 1; k >= 0; --k) {
        const LevelView<T> L = Lv[k];
        const LevelView<T> Lc = Lv[k + 1];
        const SmoothBufs B = SB[k];
        const int nx = L.n[0], ny = L.n[1], N = (int)L.N;
        const cx<T>* f = static_cast<const cx<T>*>(B.f);
        cx<T>* u = static_cast<cx<T>*>(B.u1);   // u2 = u1 + P e, in place
        cx<T>* e = static_cast<cx<T>*>(B.e);
        const cx<T>* ec = static_cast<const cx<T>*>(SB[k + 1].e);
        map_store<T>(N, u, [&](int p) {
            int gx, gy, gz;
            pos3<D>(p, nx, ny, gx, gy, gz);
            return u[p] + prolong_at<D, T>(Lc, ec, gx, gy, gz);
        });
        __syncthreads();
        if constexpr (GM) {
            cx<T>* q0 = static_cast<cx<T>*>(B.q[0]);
            cx<T>* q1 = static_cast<cx<T>*>(B.q[1]);
            cx<T>* q2 = static_cast<cx<T>*>(B.q[2]);
            map_store<T>(N, q0, [&](int p) {
                int gx, gy, gz;
                pos3<D>(p, nx, ny, gx, gy, gz);
                return f[p] - stencil_at<D, T, T>(L, u, T(1), p, gx, gy, gz);
            });
            __syncthreads();
            map_store<T>(N, q1, [&](int p) {
                int gx, gy, gz;
                pos3<D>(p, nx, ny, gx, gy, gz);
                return L.sinv * stencil_at<D, T, T>(L, q0, T(1), p, gx, gy, gz);
            });
            __syncthreads();
            map_store<T>(N, q2, [&](int p) {
                int gx, gy, gz;
                pos3<D>(p, nx, ny, gx, gy, gz);
                return L.sinv * stencil_at<D, T, T>(L, q1, T(1), p, gx, gy, gz);
            });
            __syncthreads();
            tail_gram<D, T>(L, q0, q1, q2, a.brk, sred, sc);
            const cx<T> c1 = cvt<T>(sc[0]), c2 = cvt<T>(sc[1]), c3 = cvt<T>(sc[2]);
            map_store<T>(N, e, [&](int p) { return u[p] - L.sinv * (c1 * q0[p] + c2 * q1[p] + c3 * q2[p]); });
        } else {
            map_store<T>(N, e, [&](int p) {
                int gx, gy, gz;
                pos3<D>(p, nx, ny, gx, gy, gz);
                const cx<T> r = f[p] - stencil_at<D, T, T>(L, u, T(1), p, gx, gy, gz);
                return u[p] + cdiv(L.omega * r, diag_at<D>(L, gx, gy, gz, L.k2[p]));
            });
        }
        __syncthreads();
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
