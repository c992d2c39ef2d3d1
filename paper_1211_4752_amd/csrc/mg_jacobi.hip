// gfx950 omega-Jacobi cycle kernels of the level-dependent complex-shifted
// multigrid: the two fused passes of every level above the coarse tail, in
// two forms.
//
//   K_A  omega-Jacobi pre-smoothing (Sec. 3.2.1, eq. wjacobi), residual of
//        the smoothed iterate and full-weighting restriction to the next
//        level (Sec. 2.1, Sec. 3.1, eq. erreq1 with c = 1); optional
//        ||f - A u||^2 partials of the incoming iterate.
//   K_B  (bi/tri)linear interpolation of the coarse correction, v <- v + e
//        (Sec. 3.1), and omega-Jacobi post-smoothing.
//
// Tiles (k_smooth_restrict, k_prolong_smooth): one workgroup per 2D/3D tile,
// every stage through LDS with its halo; any incoming iterate.
// Plane sweeps (k_sweep_sr, k_sweep_ps), zero incoming iterate only (the
// cycle applied as a preconditioner, Sec. 4.1, and the correction equation
// of every coarser level): a workgroup owns a TX x TY column of the grid (3D;
// a TX-point row segment in 2D) and sweeps a chunk of ZC planes along the
// slowest axis.  Every input is read once per plane plus a one-point halo
// inside the plane; the planes that the operator couples along the sweep
// axis stay in registers (each thread keeps its own points of the last
// three planes), so LDS carries only the in-plane neighbours; the inputs of
// the next plane are loaded before the current plane is computed.
//
// Both forms build every value with the same operations in the same order,
// and this file is compiled without floating-point contraction, so the two
// give bit-identical results and a launch may use either on any level (a
// batch launch takes the shape of its largest grid).
//
// Level operator (Sec. 3.1, eq. cslvariant): A~ u = sum_axes (cm u_- + c0 u +
// cp u_+) - sigma k^2 u, zero Dirichlet ghosts; D = sum_axes c0 - sigma k^2.

// every multiply and add rounds on its own (no fused multiply-add), here and
// in the helpers included below
#pragma clang fp contract(off)

#include "mg_kcommon.hpp"

namespace mg {

using namespace kc;

namespace {

// Arithmetic of both forms of the kernels.  The fused multiply-adds are
// written out (contraction is off in this file), so each value comes out
// bit-identical wherever it is formed.
template <typename T>
__device__ __forceinline__ T jfma(T a, T b, T c) {
    if constexpr (sizeof(T) == 8)
        return __builtin_fma(a, b, c);
    else
        return __builtin_fmaf(a, b, c);
}
// a b
template <typename T>
__device__ __forceinline__ cx<T> jmul(cx<T> a, cx<T> b) {
    return mk<T>(jfma(a.r, b.r, -(a.i * b.i)), jfma(a.r, b.i, a.i * b.r));
}
// acc + a b
template <typename T>
__device__ __forceinline__ cx<T> jmad(cx<T> acc, cx<T> a, cx<T> b) {
    return mk<T>(jfma(a.r, b.r, jfma(-a.i, b.i, acc.r)), jfma(a.r, b.i, jfma(a.i, b.r, acc.i)));
}
// acc + w b, w real
template <typename T>
__device__ __forceinline__ cx<T> jmadr(cx<T> acc, T w, cx<T> b) {
    return mk<T>(jfma(w, b.r, acc.r), jfma(w, b.i, acc.i));
}
// w b, w real
template <typename T>
__device__ __forceinline__ cx<T> jscale(T w, cx<T> b) {
    return mk<T>(w * b.r, w * b.i);
}
// D = (c0 of the other axes, summed x first) + c0 of the last axis - sigma k^2
template <typename T>
__device__ __forceinline__ cx<T> jdiag(cx<T> c0s, cx<T> c0m, T k2, cx<T> sigma) {
    const cx<T> d = c0s + c0m;
    return mk<T>(jfma(-k2, sigma.r, d.r), jfma(-k2, sigma.i, d.i));
}
// sum of c0 over the axes before the last one
template <int D, typename T>
__device__ __forceinline__ cx<T> c0_head(const GLevel<T>& L, int gx, int gy) {
    if constexpr (D == 3)
        return L.c0[0][gx] + L.c0[1][gy];
    else
        return L.c0[0][gx];
}
// v where c holds, else 0 (componentwise, so that no select of addresses
// sends v through scratch memory)
template <typename T>
__device__ __forceinline__ cx<T> keep(bool c, cx<T> v) {
    return mk<T>(c ? v.r : T(0), c ? v.i : T(0));
}
// 1 / |d|^2
template <typename T>
__device__ __forceinline__ T jinv(cx<T> d) {
    return T(1) / jfma(d.r, d.r, d.i * d.i);
}
// a / d with inv = 1 / |d|^2
template <typename T>
__device__ __forceinline__ cx<T> jdiv(cx<T> a, cx<T> d, T inv) {
    return mk<T>(jfma(a.r, d.r, a.i * d.i) * inv, jfma(a.i, d.r, -(a.r * d.i)) * inv);
}

// ---------------------------------------------------------------------------
// Fused pre-smooth + residual + full weighting.
// Tile: fine points [x0, x0+TX) x [y0, y0+TY) (x [z0, z0+TZ)); it owns the
// coarse points whose centre 2C+1 lies in the tile.  LDS regions, relative to
// the tile origin: u on [-2, T+2], u1 on [-1, T+1], r on [0, T].
// ---------------------------------------------------------------------------
template <int D, typename T, typename TF, bool ZERO, int TX, int TY, int TZ>
__global__ void __launch_bounds__(NT) k_smooth_restrict(const CycleArgs a) {
    constexpr int TZE = (D == 3) ? TZ : 1;
    constexpr int UX = TX + 5, UY = TY + 5, UZ = (D == 3) ? TZ + 5 : 1;
    constexpr int VX = TX + 3, VY = TY + 3, VZ = (D == 3) ? TZ + 3 : 1;
    constexpr int RX = TX + 1, RY = TY + 1, RZ = (D == 3) ? TZ + 1 : 1;
    constexpr int NU = UX * UY * UZ, NV = VX * VY * VZ, NR = RX * RY * RZ;
    constexpr int NB0 = ZERO ? NR : (NU > NR ? NU : NR);
    constexpr int CX = TX / 2, CY = TY / 2, CZ = (D == 3) ? TZ / 2 : 1;
    static_assert(TX % 2 == 0 && TY % 2 == 0 && (D == 2 || TZ % 2 == 0), "even tiles");

    __shared__ cx<T> s0[NB0];   // u, later r
    __shared__ cx<T> s1[NV];    // u1
    __shared__ double sred[NT / 64];

    const int pid = xcd_remap(blockIdx.x, gridDim.x);
    const int slot = find_slot(a.st.s, a.st.n, pid);
    const CycleSlot& sl = a.st.s[slot];
    if (gated_off(sl.gate)) return;
    const int tile = pid - sl.tile0;
    const LevelView<T>* Lp = static_cast<const LevelView<T>*>(sl.lv);
    const GLevel<T> L = glevel(*Lp);
    const int nx = L.n[0], ny = L.n[1], nz = L.n[2];
    const int ntx = (nx + TX - 1) / TX, nty = (ny + TY - 1) / TY;
    const int tx = tile % ntx;
    const int rest = tile / ntx;
    const int ty = rest % nty;
    const int tz = rest / nty;
    const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZE;
    const auto f = gin(static_cast<const cx<TF>*>(sl.f));
    const T fs = (T)fscale_of(sl);
    const auto u1p = gout(static_cast<cx<T>*>(sl.u1));

    if constexpr (!ZERO) {
        const auto u = gin(static_cast<const cx<T>*>(sl.u));
        for (int idx = threadIdx.x; idx < NU; idx += NT) {
            const int lx = idx % UX;
            const int rr = idx / UX;
            const int ly = rr % UY;
            const int lz = rr / UY;
            const int gx = x0 - 2 + lx, gy = y0 - 2 + ly;
            const int gz = (D == 3) ? z0 - 2 + lz : 0;
            cx<T> v = mk<T>(0, 0);
            if (gx >= 0 && gx < nx && gy >= 0 && gy < ny && (D == 2 || (gz >= 0 && gz < nz)))
                v = u[((long long)gz * ny + gy) * nx + gx];
            s0[idx] = v;
        }
        __syncthreads();
    }

    double nrm = 0.0;
    for (int idx = threadIdx.x; idx < NV; idx += NT) {
        const int lx = idx % VX;
        const int rr = idx / VX;
        const int ly = rr % VY;
        const int lz = rr / VY;
        const int gx = x0 - 1 + lx, gy = y0 - 1 + ly;
        const int gz = (D == 3) ? z0 - 1 + lz : 0;
        cx<T> u1 = mk<T>(0, 0);
        if (gx >= 0 && gx < nx && gy >= 0 && gy < ny && (D == 2 || (gz >= 0 && gz < nz))) {
            const long long g = ((long long)gz * ny + gy) * nx + gx;
            const cx<T> fv = fs * cvt<T, TF>(f[g]);
            const cx<T> d = jdiag<T>(c0_head<D>(L, gx, gy), L.c0[D - 1][D == 3 ? gz : gy], L.k2[g], L.sigma);
            const T inv = jinv<T>(d);
            if constexpr (ZERO) {
                u1 = jdiv<T>(jmul<T>(L.omega, fv), d, inv);
            } else {
                const int c = ((D == 3 ? lz + 1 : 0) * UY + (ly + 1)) * UX + (lx + 1);
                const cx<T> uc = s0[c];
                cx<T> au = jmul<T>(d, uc);
                au = jmad<T>(au, L.cm[0][gx], s0[c - 1]);
                au = jmad<T>(au, L.cp[0][gx], s0[c + 1]);
                au = jmad<T>(au, L.cm[1][gy], s0[c - UX]);
                au = jmad<T>(au, L.cp[1][gy], s0[c + UX]);
                if constexpr (D == 3) {
                    au = jmad<T>(au, L.cm[2][gz], s0[c - UX * UY]);
                    au = jmad<T>(au, L.cp[2][gz], s0[c + UX * UY]);
                }
                const cx<T> res = fv - au;
                u1 = uc + jdiv<T>(jmul<T>(L.omega, res), d, inv);
                const bool own = lx >= 1 && lx <= TX && ly >= 1 && ly <= TY && (D == 2 || (lz >= 1 && lz <= TZ));
                if (own) {
                    nrm += (double)abs2(res);
                    if (u1p) u1p[g] = u1;
                }
            }
        }
        s1[idx] = u1;
    }
    __syncthreads();

    for (int idx = threadIdx.x; idx < NR; idx += NT) {
        const int lx = idx % RX;
        const int rr = idx / RX;
        const int ly = rr % RY;
        const int lz = rr / RY;
        const int gx = x0 + lx, gy = y0 + ly;
        const int gz = (D == 3) ? z0 + lz : 0;
        cx<T> r = mk<T>(0, 0);
        if (gx < nx && gy < ny && (D == 2 || gz < nz)) {
            const long long g = ((long long)gz * ny + gy) * nx + gx;
            const cx<T> fv = fs * cvt<T, TF>(f[g]);
            const cx<T> d = jdiag<T>(c0_head<D>(L, gx, gy), L.c0[D - 1][D == 3 ? gz : gy], L.k2[g], L.sigma);
            const int c = ((D == 3 ? lz + 1 : 0) * VY + (ly + 1)) * VX + (lx + 1);
            cx<T> au = jmul<T>(d, s1[c]);
            au = jmad<T>(au, L.cm[0][gx], s1[c - 1]);
            au = jmad<T>(au, L.cp[0][gx], s1[c + 1]);
            au = jmad<T>(au, L.cm[1][gy], s1[c - VX]);
            au = jmad<T>(au, L.cp[1][gy], s1[c + VX]);
            if constexpr (D == 3) {
                au = jmad<T>(au, L.cm[2][gz], s1[c - VX * VY]);
                au = jmad<T>(au, L.cp[2][gz], s1[c + VX * VY]);
            }
            r = fv - au;
        }
        s0[idx] = r;
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
                        acc = jmadr<T>(acc, w, s0[row + ox]);
                    }
                }
            }
            fc[((long long)Cz * ncy + Cy) * ncx + Cx] = acc;
        }
    }

    if constexpr (!ZERO) {
        if (a.norm_part) {
            const double s = block_sum(nrm, sred);
            if (threadIdx.x == 0) a.norm_part[(long long)slot * a.pstride + tile] = s;
        }
    }
}

// ---------------------------------------------------------------------------
// Fused prolongation + correction + post-smooth.
// LDS: coarse correction on [x0/2 - 1, x0/2 + TX/2], corrected iterate u2 on
// fine [-1, T] relative to the tile.
// ---------------------------------------------------------------------------
template <int D, typename T, typename TF, typename TO, bool ZERO, bool ACC, int TX, int TY, int TZ>
__global__ void __launch_bounds__(NT) k_prolong_smooth(const CycleArgs a) {
    constexpr int TZE = (D == 3) ? TZ : 1;
    constexpr int EX = TX / 2 + 2, EY = TY / 2 + 2, EZ = (D == 3) ? TZ / 2 + 2 : 1;
    constexpr int WX = TX + 2, WY = TY + 2, WZ = (D == 3) ? TZ + 2 : 1;
    constexpr int NE = EX * EY * EZ, NW = WX * WY * WZ;

    __shared__ cx<T> se[NE];
    __shared__ cx<T> s2[NW];

    const int pid = xcd_remap(blockIdx.x, gridDim.x);
    const int slot = find_slot(a.st.s, a.st.n, pid);
    const CycleSlot& sl = a.st.s[slot];
    if (gated_off(sl.gate)) return;
    const int tile = pid - sl.tile0;
    const LevelView<T>* Lp = static_cast<const LevelView<T>*>(sl.lv);
    const GLevel<T> L = glevel(*Lp);
    const int nx = L.n[0], ny = L.n[1], nz = L.n[2];
    const int ncx = Lp[1].n[0], ncy = Lp[1].n[1], ncz = Lp[1].n[2];
    const int ntx = (nx + TX - 1) / TX, nty = (ny + TY - 1) / TY;
    const int tx = tile % ntx;
    const int rest = tile / ntx;
    const int ty = rest % nty;
    const int tz = rest / nty;
    const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZE;
    const auto f = gin(static_cast<const cx<TF>*>(sl.f));
    const T fs = (T)fscale_of(sl);
    const auto ec = gin(static_cast<const cx<T>*>(sl.c));
    const auto u1in = gin(static_cast<const cx<T>*>(sl.u1));
    const int cxs = x0 / 2 - 1, cys = y0 / 2 - 1, czs = (D == 3) ? z0 / 2 - 1 : 0;

    for (int idx = threadIdx.x; idx < NE; idx += NT) {
        const int lx = idx % EX;
        const int rr = idx / EX;
        const int ly = rr % EY;
        const int lz = rr / EY;
        const int Cx = cxs + lx, Cy = cys + ly, Cz = czs + lz;
        cx<T> v = mk<T>(0, 0);
        if (Cx >= 0 && Cx < ncx && Cy >= 0 && Cy < ncy && (D == 2 || (Cz >= 0 && Cz < ncz)))
            v = ec[((long long)Cz * ncy + Cy) * ncx + Cx];
        se[idx] = v;
    }
    __syncthreads();

    for (int idx = threadIdx.x; idx < NW; idx += NT) {
        const int lx = idx % WX;
        const int rr = idx / WX;
        const int ly = rr % WY;
        const int lz = rr / WY;
        const int gx = x0 - 1 + lx, gy = y0 - 1 + ly;
        const int gz = (D == 3) ? z0 - 1 + lz : 0;
        cx<T> u2 = mk<T>(0, 0);
        if (gx >= 0 && gx < nx && gy >= 0 && gy < ny && (D == 2 || (gz >= 0 && gz < nz))) {
            const long long g = ((long long)gz * ny + gy) * nx + gx;
            cx<T> u1;
            if constexpr (ZERO) {
                const cx<T> fv = fs * cvt<T, TF>(f[g]);
                const cx<T> d = jdiag<T>(c0_head<D>(L, gx, gy), L.c0[D - 1][D == 3 ? gz : gy], L.k2[g], L.sigma);
                u1 = jdiv<T>(jmul<T>(L.omega, fv), d, jinv<T>(d));
            } else {
                u1 = u1in[g];
            }
            int ix0, ix1, iy0, iy1;
            T wx0, wx1, wy0, wy1;
            interp_1d<T>(gx, cxs, ix0, ix1, wx0, wx1);
            interp_1d<T>(gy, cys, iy0, iy1, wy0, wy1);
            cx<T> pe;
            if constexpr (D == 2) {
                pe = jscale<T>(wy0 * wx0, se[iy0 * EX + ix0]);
                pe = jmadr<T>(pe, wy0 * wx1, se[iy0 * EX + ix1]);
                pe = jmadr<T>(pe, wy1 * wx0, se[iy1 * EX + ix0]);
                pe = jmadr<T>(pe, wy1 * wx1, se[iy1 * EX + ix1]);
            } else {
                int iz0, iz1;
                T wz0, wz1;
                interp_1d<T>(gz, czs, iz0, iz1, wz0, wz1);
                const int p00 = (iz0 * EY + iy0) * EX, p01 = (iz0 * EY + iy1) * EX;
                const int p10 = (iz1 * EY + iy0) * EX, p11 = (iz1 * EY + iy1) * EX;
                pe = jscale<T>(wz0 * wy0 * wx0, se[p00 + ix0]);
                pe = jmadr<T>(pe, wz0 * wy0 * wx1, se[p00 + ix1]);
                pe = jmadr<T>(pe, wz0 * wy1 * wx0, se[p01 + ix0]);
                pe = jmadr<T>(pe, wz0 * wy1 * wx1, se[p01 + ix1]);
                pe = jmadr<T>(pe, wz1 * wy0 * wx0, se[p10 + ix0]);
                pe = jmadr<T>(pe, wz1 * wy0 * wx1, se[p10 + ix1]);
                pe = jmadr<T>(pe, wz1 * wy1 * wx0, se[p11 + ix0]);
                pe = jmadr<T>(pe, wz1 * wy1 * wx1, se[p11 + ix1]);
            }
            u2 = u1 + pe;
        }
        s2[idx] = u2;
    }
    __syncthreads();

    const auto out = gout(static_cast<cx<TO>*>(sl.out));
    for (int idx = threadIdx.x; idx < TX * TY * TZE; idx += NT) {
        const int lx = idx % TX;
        const int rr = idx / TX;
        const int ly = rr % TY;
        const int lz = rr / TY;
        const int gx = x0 + lx, gy = y0 + ly;
        const int gz = (D == 3) ? z0 + lz : 0;
        if (gx < nx && gy < ny && (D == 2 || gz < nz)) {
            const long long g = ((long long)gz * ny + gy) * nx + gx;
            const cx<T> fv = fs * cvt<T, TF>(f[g]);
            const cx<T> d = jdiag<T>(c0_head<D>(L, gx, gy), L.c0[D - 1][D == 3 ? gz : gy], L.k2[g], L.sigma);
            const int c = ((D == 3 ? lz + 1 : 0) * WY + (ly + 1)) * WX + (lx + 1);
            const cx<T> u2c = s2[c];
            cx<T> au = jmul<T>(d, u2c);
            au = jmad<T>(au, L.cm[0][gx], s2[c - 1]);
            au = jmad<T>(au, L.cp[0][gx], s2[c + 1]);
            au = jmad<T>(au, L.cm[1][gy], s2[c - WX]);
            au = jmad<T>(au, L.cp[1][gy], s2[c + WX]);
            if constexpr (D == 3) {
                au = jmad<T>(au, L.cm[2][gz], s2[c - WX * WY]);
                au = jmad<T>(au, L.cp[2][gz], s2[c + WX * WY]);
            }
            const cx<T> u3 = u2c + jdiv<T>(jmul<T>(L.omega, fv - au), d, jinv<T>(d));
            if constexpr (ACC) {
                out[g] = out[g].get() + cvt<TO>(u3);
            } else {
                out[g] = cvt<TO>(u3);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Plane sweeps
// ---------------------------------------------------------------------------
// Per-level constants of a sweep launch.  The plane's axes are x and, in 3D,
// y; the sweep axis is D - 1.
struct SweepGeo {
    int nx, nyp, nm;       // points along x, along the plane's y (1 in 2D), along the sweep axis
    int ncx, ncyp, ncm;    // the same on the next coarser level
    int x0, y0, m0;        // tile origin
};

template <int D, typename T, int TX, int TY, int ZC>
__device__ __forceinline__ SweepGeo sweep_geo(const LevelView<T>* Lp, int tile) {
    SweepGeo G;
    const LevelView<T>& L = *Lp;
    G.nx = L.n[0];
    G.nyp = (D == 3) ? L.n[1] : 1;
    G.nm = L.n[D - 1];
    G.ncx = Lp[1].n[0];
    G.ncyp = (D == 3) ? Lp[1].n[1] : 1;
    G.ncm = Lp[1].n[D - 1];
    const int ntx = (G.nx + TX - 1) / TX;
    const int nty = (D == 3) ? (G.nyp + TY - 1) / TY : 1;
    const int tx = tile % ntx;
    const int rest = tile / ntx;
    G.x0 = tx * TX;
    G.y0 = (D == 3) ? (rest % nty) * TY : 0;
    G.m0 = (rest / nty) * ZC;
    return G;
}

// Sweep-axis coefficients c0, cm, cp of planes m0 - 1 .. m0 - 1 + NZ - 1 into
// LDS (zero outside the grid), so that the sweep issues no global loads but
// the inputs it loads ahead (a wait on a later load would wait on those too).
template <int D, typename T, int NZ, int BS>
__device__ __forceinline__ void load_ztables(const GLevel<T>& L, const SweepGeo& G, cx<T>* z0, cx<T>* zm,
                                             cx<T>* zp) {
    for (int i = threadIdx.x; i < NZ; i += BS) {
        const int q = G.m0 - 1 + i;
        cx<T> a = mk<T>(0, 0), b = a, c = a;
        if (q >= 0 && q < G.nm) {
            a = L.c0[D - 1][q];
            b = L.cm[D - 1][q];
            c = L.cp[D - 1][q];
        }
        z0[i] = a;
        zm[i] = b;
        zp[i] = c;
    }
}

// f and k^2 of plane q at the points of this thread.  The loads are issued
// unconditionally (from element 0 where the point is outside the grid or the
// plane outside the level), and the caller masks what it uses: a load under
// a branch would make the compiler drain every load in flight at the next
// use of one of them.
template <typename T, typename TF, int K>
__device__ __forceinline__ void load_plane(GIn<cx<TF>> f, GIn<T> k2, const int (&gxy)[K], int q, int nm,
                                           long long plane, cx<TF> (&fo)[K], T (&ko)[K]) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const long long g = (gxy[k] >= 0 && q >= 0 && q < nm) ? q * plane + gxy[k] : 0;
        fo[k] = f[g];
        ko[k] = k2[g];
    }
}

// ---------------------------------------------------------------------------
// K_A sweep.  Regions of a plane, relative to the tile origin:
//   u1 on x in [-1, TX+1] (and y in [-1, TY+1] in 3D): UX x UY points,
//   r  on x in [0, TX]    (and y in [0, TY]):          RX x RY points,
// enumerated r region first (the thread that forms u1 at an r point also
// forms r there), then the ring of u1 halo points around it.
// ---------------------------------------------------------------------------
template <int D, int TX, int TY, int BS>
struct SrShape {
    static constexpr int UX = TX + 3, UY = (D == 3) ? TY + 3 : 1;
    static constexpr int RX = TX + 1, RY = (D == 3) ? TY + 1 : 1;
    static constexpr int HY = (D == 3) ? 1 : 0;
    static constexpr int NV = UX * UY, NR = RX * RY;
    static constexpr int CXN = TX / 2, CYN = (D == 3) ? TY / 2 : 1, NC = CXN * CYN;
    static constexpr int KV = (NV + BS - 1) / BS, KR = (NR + BS - 1) / BS, KC = (NC + BS - 1) / BS;
};

// local u1-region coordinates of enumeration index idx < NV
template <int D, int TX, int TY, int BS>
__device__ __forceinline__ void sr_local(int idx, int& lx, int& ly) {
    using S = SrShape<D, TX, TY, BS>;
    if (idx < S::NR) {
        lx = idx % S::RX + 1;
        ly = idx / S::RX + S::HY;
        return;
    }
    const int h = idx - S::NR;
    if constexpr (D == 2) {
        lx = h == 0 ? 0 : S::UX - 1;
        ly = 0;
    } else {
        if (h < S::UX) {
            lx = h;
            ly = 0;
        } else if (h < 2 * S::UX) {
            lx = h - S::UX;
            ly = S::UY - 1;
        } else if (h < 2 * S::UX + S::RY) {
            lx = 0;
            ly = h - 2 * S::UX + 1;
        } else {
            lx = S::UX - 1;
            ly = h - 2 * S::UX - S::RY + 1;
        }
    }
}

// acc += the in-plane full-weighting terms of one fine plane with sweep-axis
// weight wz, around the coarse point (cxl, cyl) of the tile; same terms and
// order as the tiled kernel
template <int D, typename T, int RX>
__device__ __forceinline__ void fw_plane(cx<T>& acc, const cx<T>* r, T wz, int cxl, int cyl) {
#pragma unroll
    for (int oy = (D == 3 ? -1 : 0); oy <= (D == 3 ? 1 : 0); ++oy) {
        const T wy = (D == 3) ? wz * (oy == 0 ? T(0.5) : T(0.25)) : wz;
        const int row = (D == 3) ? (2 * cyl + 1 + oy) * RX : 0;
#pragma unroll
        for (int ox = -1; ox <= 1; ++ox) {
            const T w = wy * (ox == 0 ? T(0.5) : T(0.25));
            acc = acc + w * r[row + 2 * cxl + 1 + ox];
        }
    }
}

template <int D, typename T, typename TF, int TX, int TY, int ZC, int BS, int PD>
__global__ void __launch_bounds__(BS) k_sweep_sr(const CycleArgs a) {
    using S = SrShape<D, TX, TY, BS>;
    static_assert(TX % 2 == 0 && (D == 2 || TY % 2 == 0) && ZC % 2 == 0, "even tiles");
    __shared__ cx<T> su[2 * S::NV];   // u1 of plane q in slot q & 1
    __shared__ cx<T> sr[S::NR];       // r of one plane
    // sweep-axis coefficients of planes m0 - 1 .. m0 + ZC + PD (the steps run
    // in groups of PD, past the last plane up to PD - 1 steps)
    constexpr int NZ = ZC + PD + 2;
    __shared__ cx<T> tz0[NZ], tzm[NZ], tzp[NZ];

    const int pid = xcd_remap(blockIdx.x, gridDim.x);
    const int slot = find_slot(a.st.s, a.st.n, pid);
    const CycleSlot& sl = a.st.s[slot];
    if (gated_off(sl.gate)) return;
    const LevelView<T>* Lp = static_cast<const LevelView<T>*>(sl.lv);
    const GLevel<T> L = glevel(*Lp);
    const SweepGeo G = sweep_geo<D, T, TX, TY, ZC>(Lp, pid - sl.tile0);
    const auto f = gin(static_cast<const cx<TF>*>(sl.f));
    const T fs = (T)fscale_of(sl);
    const auto fc = gout(static_cast<cx<T>*>(sl.c));
    const int t = threadIdx.x;
    const cx<T> Z = mk<T>(0, 0);

    // per point of this thread: offset in a plane of the grid (-1: outside
    // the grid or past the region) and the c0 sum of the in-plane axes
    int gxy[S::KV];
    cx<T> dxy[S::KV];
#pragma unroll
    for (int k = 0; k < S::KV; ++k) {
        const int idx = t + k * BS;
        gxy[k] = -1;
        dxy[k] = Z;
        if (idx < S::NV) {
            int lx, ly;
            sr_local<D, TX, TY, BS>(idx, lx, ly);
            const int gx = G.x0 - 1 + lx, gy = (D == 3) ? G.y0 - 1 + ly : 0;
            if (gx >= 0 && gx < G.nx && gy >= 0 && gy < G.nyp) {
                gxy[k] = gy * G.nx + gx;
                dxy[k] = c0_head<D>(L, gx, gy);
            }
        }
    }
    // per r point: in-plane couplings
    cx<T> cxm[S::KR], cxp[S::KR], cym[S::KR], cyp[S::KR];
    unsigned rin = 0;
#pragma unroll
    for (int k = 0; k < S::KR; ++k) {
        const int idx = t + k * BS;
        cxm[k] = cxp[k] = cym[k] = cyp[k] = Z;
        if (idx < S::NR) {
            const int gx = G.x0 + idx % S::RX, gy = (D == 3) ? G.y0 + idx / S::RX : 0;
            if (gx < G.nx && gy < G.nyp) {
                rin |= 1u << k;
                cxm[k] = L.cm[0][gx];
                cxp[k] = L.cp[0][gx];
                if constexpr (D == 3) {
                    cym[k] = L.cm[1][gy];
                    cyp[k] = L.cp[1][gy];
                }
            }
        }
    }
    const long long plane = (long long)G.nyp * G.nx;
    const long long cplane = (long long)G.ncyp * G.ncx;
    const int plast = G.m0 + ZC < G.nm - 1 ? G.m0 + ZC : G.nm - 1;   // last plane of r this chunk needs
    load_ztables<D, T, NZ, BS>(L, G, tz0, tzm, tzp);

    // f and k^2 of planes q .. q + PD - 1 (loads issued PD planes ahead)
    cx<TF> pf[PD][S::KV];
    T pk[PD][S::KV];
    // at the r points: u1 of planes q - 2, q - 1, q; f and D of planes q - 1, q
    cx<T> ua[S::KR], ub[S::KR], uc[S::KR], fvp[S::KR], dp[S::KR], fvc[S::KR], dc[S::KR];
    cx<T> acc[S::KC];
#pragma unroll
    for (int k = 0; k < S::KR; ++k) ua[k] = ub[k] = uc[k] = fvp[k] = dp[k] = fvc[k] = dc[k] = Z;
#pragma unroll
    for (int k = 0; k < S::KC; ++k) acc[k] = Z;
#pragma unroll
    for (int i = 0; i < PD; ++i) load_plane(f, L.k2, gxy, G.m0 - 1 + i, G.nm, plane, pf[i], pk[i]);
    __syncthreads();   // sweep-axis tables

    // plane q = q0 + i uses register set i, which then takes plane q + PD (the
    // loop over i is unrolled, so the sets are never copied, and it has no
    // early exit, so the compiler keeps the loads in flight); steps past the
    // last plane only form u1
    const int qend = plast + 1;
    for (int q0 = G.m0 - 1; q0 <= qend; q0 += PD) {
#pragma unroll
        for (int i = 0; i < PD; ++i) {
            const int q = q0 + i;
            // u1 on plane q (zero outside the grid)
            cx<T>* U = su + (q & 1) * S::NV;
            const bool qin = q >= 0 && q < G.nm;
            const cx<T> dz = tz0[q - G.m0 + 1];
#pragma unroll
            for (int k = 0; k < S::KV; ++k) {
                const int idx = t + k * BS;
                if (idx >= S::NV) continue;
                int lx, ly;
                sr_local<D, TX, TY, BS>(idx, lx, ly);
                cx<T> u1 = Z, fv = Z, d = Z;
                if (gxy[k] >= 0 && qin) {
                    fv = fs * cvt<T>(pf[i][k]);
                    d = jdiag<T>(dxy[k], dz, pk[i][k], L.sigma);
                    u1 = jdiv<T>(jmul<T>(L.omega, fv), d, jinv<T>(d));
                }
                U[ly * S::UX + lx] = u1;
                if (k < S::KR) {
                    ua[k] = ub[k];
                    ub[k] = uc[k];
                    uc[k] = u1;
                    fvp[k] = fvc[k];
                    dp[k] = dc[k];
                    fvc[k] = fv;
                    dc[k] = d;
                }
            }
            load_plane(f, L.k2, gxy, q + PD, G.nm, plane, pf[i], pk[i]);
            __syncthreads();

            // r on plane p = q - 1 (u1 of planes p - 1, p, p + 1 in ua, ub,
            // uc), then the full-weighting terms of that plane
            const int p = q - 1;
            if (p < G.m0 || p > plast) continue;
            const cx<T>* U0 = su + (p & 1) * S::NV;
            const cx<T> cmz = tzm[p - G.m0 + 1], cpz = tzp[p - G.m0 + 1];
#pragma unroll
            for (int k = 0; k < S::KR; ++k) {
                const int idx = t + k * BS;
                if (idx >= S::NR) continue;
                cx<T> r = Z;
                if ((rin >> k) & 1u) {
                    const int c = (idx / S::RX + S::HY) * S::UX + idx % S::RX + 1;
                    cx<T> au = jmul<T>(dp[k], ub[k]);
                    au = jmad<T>(au, cxm[k], U0[c - 1]);
                    au = jmad<T>(au, cxp[k], U0[c + 1]);
                    if constexpr (D == 3) {
                        au = jmad<T>(au, cym[k], U0[c - S::UX]);
                        au = jmad<T>(au, cyp[k], U0[c + S::UX]);
                    }
                    au = jmad<T>(au, cmz, ua[k]);
                    au = jmad<T>(au, cpz, uc[k]);
                    r = fvp[k] - au;
                }
                sr[idx] = r;
            }
            __syncthreads();
            // plane p is 2C + 1 + oz of coarse plane C: oz = 0 for odd p; for
            // even p the last plane (oz = 1) of C = p/2 - 1 and the first
            // (oz = -1) of C = p/2
#pragma unroll
            for (int k = 0; k < S::KC; ++k) {
                const int j = t + k * BS;
                if (j >= S::NC) continue;
                const int cxl = j % S::CXN, cyl = j / S::CXN;
                if (p & 1) {
                    fw_plane<D, T, S::RX>(acc[k], sr, T(0.5), cxl, cyl);
                } else {
                    const int Cm = p / 2 - 1;
                    if (p >= G.m0 + 2) {
                        fw_plane<D, T, S::RX>(acc[k], sr, T(0.25), cxl, cyl);
                        const int Cx = G.x0 / 2 + cxl, Cy = (D == 3) ? G.y0 / 2 + cyl : 0;
                        if (Cx < G.ncx && Cy < G.ncyp && Cm < G.ncm)
                            fc[Cm * cplane + (long long)Cy * G.ncx + Cx] = acc[k];
                    }
                    acc[k] = Z;
                    fw_plane<D, T, S::RX>(acc[k], sr, T(0.25), cxl, cyl);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// K_B sweep.  Regions of a plane, relative to the tile origin:
//   u2 on x in [-1, TX] (and y in [-1, TY] in 3D): WX x WY points,
//   the tile itself TX x TY (TX in 2D), enumerated first, then the halo ring;
//   coarse correction on x in [x0/2 - 1, x0/2 + TX/2] (and likewise in y):
//   EX x EY points per coarse plane, two coarse planes in LDS.
// ---------------------------------------------------------------------------
template <int D, int TX, int TY, int BS>
struct PsShape {
    static constexpr int WX = TX + 2, WY = (D == 3) ? TY + 2 : 1;
    static constexpr int PY = (D == 3) ? TY : 1, HY = (D == 3) ? 1 : 0;
    static constexpr int NW = WX * WY, NI = TX * PY;
    static constexpr int EX = TX / 2 + 2, EY = (D == 3) ? TY / 2 + 2 : 1, NE = EX * EY;
    static constexpr int KW = (NW + BS - 1) / BS, KI = (NI + BS - 1) / BS, KE = (NE + BS - 1) / BS;
};

template <int D, int TX, int TY, int BS>
__device__ __forceinline__ void ps_local(int idx, int& lx, int& ly) {
    using S = PsShape<D, TX, TY, BS>;
    if (idx < S::NI) {
        lx = idx % TX + 1;
        ly = idx / TX + S::HY;
        return;
    }
    const int h = idx - S::NI;
    if constexpr (D == 2) {
        lx = h == 0 ? 0 : S::WX - 1;
        ly = 0;
    } else {
        if (h < S::WX) {
            lx = h;
            ly = 0;
        } else if (h < 2 * S::WX) {
            lx = h - S::WX;
            ly = S::WY - 1;
        } else if (h < 2 * S::WX + TY) {
            lx = 0;
            ly = h - 2 * S::WX + 1;
        } else {
            lx = S::WX - 1;
            ly = h - 2 * S::WX - TY + 1;
        }
    }
}

template <int D, typename T, typename TF, typename TO, bool ACC, int TX, int TY, int ZC, int BS, int PD>
__global__ void __launch_bounds__(BS) k_sweep_ps(const CycleArgs a) {
    using S = PsShape<D, TX, TY, BS>;
    static_assert(TX % 2 == 0 && (D == 2 || TY % 2 == 0) && ZC % 2 == 0, "even tiles");
    static_assert(PD % 2 == 0, "the coarse planes advance every second plane");
    constexpr int PC = PD / 2;        // coarse planes loaded ahead
    __shared__ cx<T> su[3 * S::NW];   // u2 of plane q in slot (q + 1) % 3
    __shared__ cx<T> se[2 * S::NE];   // coarse correction, coarse plane J in slot (J + 1) % 2
    // sweep-axis coefficients of planes m0 - 1 .. m0 + ZC + PD - 1 (the steps
    // run in groups of PD, past the last plane up to PD - 1 steps)
    constexpr int NZ = ZC + PD + 1;
    __shared__ cx<T> tz0[NZ], tzm[NZ], tzp[NZ];

    const int pid = xcd_remap(blockIdx.x, gridDim.x);
    const int slot = find_slot(a.st.s, a.st.n, pid);
    const CycleSlot& sl = a.st.s[slot];
    if (gated_off(sl.gate)) return;
    const LevelView<T>* Lp = static_cast<const LevelView<T>*>(sl.lv);
    const GLevel<T> L = glevel(*Lp);
    const SweepGeo G = sweep_geo<D, T, TX, TY, ZC>(Lp, pid - sl.tile0);
    const auto f = gin(static_cast<const cx<TF>*>(sl.f));
    const T fs = (T)fscale_of(sl);
    const auto ec = gin(static_cast<const cx<T>*>(sl.c));
    const auto out = gout(static_cast<cx<TO>*>(sl.out));
    const int t = threadIdx.x;
    const cx<T> Z = mk<T>(0, 0);
    const int cxs = G.x0 / 2 - 1, cys = (D == 3) ? G.y0 / 2 - 1 : 0;
    const long long plane = (long long)G.nyp * G.nx;
    const long long cplane = (long long)G.ncyp * G.ncx;

    int gxy[S::KW];
    cx<T> dxy[S::KW];
#pragma unroll
    for (int k = 0; k < S::KW; ++k) {
        const int idx = t + k * BS;
        gxy[k] = -1;
        dxy[k] = Z;
        if (idx < S::NW) {
            int lx, ly;
            ps_local<D, TX, TY, BS>(idx, lx, ly);
            const int gx = G.x0 - 1 + lx, gy = (D == 3) ? G.y0 - 1 + ly : 0;
            if (gx >= 0 && gx < G.nx && gy >= 0 && gy < G.nyp) {
                gxy[k] = gy * G.nx + gx;
                dxy[k] = c0_head<D>(L, gx, gy);
            }
        }
    }
    cx<T> cxm[S::KI], cxp[S::KI], cym[S::KI], cyp[S::KI];
    unsigned iin = 0;
#pragma unroll
    for (int k = 0; k < S::KI; ++k) {
        const int idx = t + k * BS;
        cxm[k] = cxp[k] = cym[k] = cyp[k] = Z;
        if (idx < S::NI) {
            const int gx = G.x0 + idx % TX, gy = (D == 3) ? G.y0 + idx / TX : 0;
            if (gx < G.nx && gy < G.nyp) {
                iin |= 1u << k;
                cxm[k] = L.cm[0][gx];
                cxp[k] = L.cp[0][gx];
                if constexpr (D == 3) {
                    cym[k] = L.cm[1][gy];
                    cyp[k] = L.cp[1][gy];
                }
            }
        }
    }
    // offset of each coarse point of this thread in a coarse plane (-1: outside)
    int cxy[S::KE];
#pragma unroll
    for (int k = 0; k < S::KE; ++k) {
        const int idx = t + k * BS;
        cxy[k] = -1;
        if (idx < S::NE) {
            const int Cx = cxs + idx % S::EX, Cy = cys + idx / S::EX;
            if (Cx >= 0 && Cx < G.ncx && Cy >= 0 && Cy < G.ncyp) cxy[k] = Cy * G.ncx + Cx;
        }
    }
    // coarse plane J at the points of this thread (loaded unconditionally,
    // like load_plane; the LDS store masks)
#define MG_LOAD_COARSE(J, V)                                                                   \
    for (int k = 0; k < S::KE; ++k)                                                            \
        V[k] = ec[(cxy[k] >= 0 && (J) >= 0 && (J) < G.ncm) ? (long long)(J) * cplane + cxy[k] : 0];
#define MG_STORE_COARSE(J, V)                                                                  \
    for (int k = 0; k < S::KE; ++k)                                                            \
        if (t + k * BS < S::NE)                                                                \
            se[(((J) + 1) & 1) * S::NE + t + k * BS] = keep(cxy[k] >= 0 && (J) >= 0 && (J) < G.ncm, V[k]);

    cx<TF> pf[PD][S::KW];
    T pk[PD][S::KW];
    cx<T> pc[PC][S::KE];   // coarse planes J1 .. J1 + PC - 1, J1 the next one to enter LDS
    // at the tile points: u2 of planes q - 2, q - 1, q; f, D and 1/|D|^2 of planes q - 1, q
    cx<T> ua[S::KI], ub[S::KI], uc[S::KI], fvp[S::KI], dp[S::KI], fvc[S::KI], dc[S::KI];
    T ivp[S::KI], ivc[S::KI];
#pragma unroll
    for (int k = 0; k < S::KI; ++k) {
        ua[k] = ub[k] = uc[k] = fvp[k] = dp[k] = fvc[k] = dc[k] = Z;
        ivp[k] = ivc[k] = T(0);
    }
    const int pend = G.m0 + ZC < G.nm ? G.m0 + ZC : G.nm;   // planes [m0, pend) of the result
    load_ztables<D, T, NZ, BS>(L, G, tz0, tzm, tzp);

    {
        cx<T> v[S::KE];
        const int J = G.m0 / 2 - 1;
#pragma unroll
        MG_LOAD_COARSE(J, v)
#pragma unroll
        MG_STORE_COARSE(J, v)
    }
    // coarse sets first, then the plane sets: the same order of loads in
    // flight as in the loop, so the first pass waits no longer than the rest
#pragma unroll
    for (int i = 0; i < PC; ++i) {
        const int J = G.m0 / 2 + i;
#pragma unroll
        MG_LOAD_COARSE(J, pc[i])
    }
#pragma unroll
    for (int i = 0; i < PD; ++i) load_plane(f, L.k2, gxy, G.m0 - 1 + i, G.nm, plane, pf[i], pk[i]);
    __syncthreads();
    // plane q = q0 + i uses register set i, which then takes plane q + PD;
    // q0 is odd, so the coarse plane J0 + i/2 (J0 = (q0 + 1) / 2) enters LDS
    // at even i from coarse set i/2, which then takes plane J0 + i/2 + PC
    // (no early exit from the unrolled loop; steps past the last plane only
    // form u2)
    for (int q0 = G.m0 - 1; q0 <= pend; q0 += PD) {
        const int J0 = (q0 + 1) / 2;
#pragma unroll
        for (int i = 0; i < PD; ++i) {
            const int q = q0 + i;
            if (i % 2 == 0) {
                const int J = J0 + i / 2;
#pragma unroll
                MG_STORE_COARSE(J, pc[i / 2])
                const int Jn = J + PC;
#pragma unroll
                MG_LOAD_COARSE(Jn, pc[i / 2])
            }
            // u2 on plane q; coarse planes Ja and Ja + 1 (Ja alone, weight 1, for odd q)
            cx<T>* U = su + ((q + 1) % 3) * S::NW;
            const bool qin = q >= 0 && q < G.nm;
            const cx<T> dz = tz0[q - G.m0 + 1];
            const bool odd = (i % 2 == 0);   // q0 is odd
            const int Ja = odd ? (q - 1) / 2 : q / 2 - 1;
            const cx<T>* Ea = se + ((Ja + 1) & 1) * S::NE;
            const cx<T>* Eb = odd ? Ea : se + (Ja & 1) * S::NE;
            const T wa = odd ? T(1) : T(0.5), wb = odd ? T(0) : T(0.5);
#pragma unroll
            for (int k = 0; k < S::KW; ++k) {
                const int idx = t + k * BS;
                if (idx >= S::NW) continue;
                int lx, ly;
                ps_local<D, TX, TY, BS>(idx, lx, ly);
                cx<T> u2 = Z, fv = Z, d = Z;
                T iv = T(0);
                if (gxy[k] >= 0 && qin) {
                    fv = fs * cvt<T>(pf[i][k]);
                    d = jdiag<T>(dxy[k], dz, pk[i][k], L.sigma);
                    iv = jinv<T>(d);
                    const cx<T> u1 = jdiv<T>(jmul<T>(L.omega, fv), d, iv);
                    int ix0, ix1;
                    T wx0, wx1;
                    interp_1d<T>(G.x0 - 1 + lx, cxs, ix0, ix1, wx0, wx1);
                    cx<T> pe;
                    if constexpr (D == 3) {
                        int iy0, iy1;
                        T wy0, wy1;
                        interp_1d<T>(G.y0 - 1 + ly, cys, iy0, iy1, wy0, wy1);
                        const int p0 = iy0 * S::EX, p1 = iy1 * S::EX;
                        pe = jscale<T>(wa * wy0 * wx0, Ea[p0 + ix0]);
                        pe = jmadr<T>(pe, wa * wy0 * wx1, Ea[p0 + ix1]);
                        pe = jmadr<T>(pe, wa * wy1 * wx0, Ea[p1 + ix0]);
                        pe = jmadr<T>(pe, wa * wy1 * wx1, Ea[p1 + ix1]);
                        pe = jmadr<T>(pe, wb * wy0 * wx0, Eb[p0 + ix0]);
                        pe = jmadr<T>(pe, wb * wy0 * wx1, Eb[p0 + ix1]);
                        pe = jmadr<T>(pe, wb * wy1 * wx0, Eb[p1 + ix0]);
                        pe = jmadr<T>(pe, wb * wy1 * wx1, Eb[p1 + ix1]);
                    } else {
                        pe = jscale<T>(wa * wx0, Ea[ix0]);
                        pe = jmadr<T>(pe, wa * wx1, Ea[ix1]);
                        pe = jmadr<T>(pe, wb * wx0, Eb[ix0]);
                        pe = jmadr<T>(pe, wb * wx1, Eb[ix1]);
                    }
                    u2 = u1 + pe;
                }
                U[ly * S::WX + lx] = u2;
                if (k < S::KI) {
                    ua[k] = ub[k];
                    ub[k] = uc[k];
                    uc[k] = u2;
                    fvp[k] = fvc[k];
                    dp[k] = dc[k];
                    ivp[k] = ivc[k];
                    fvc[k] = fv;
                    dc[k] = d;
                    ivc[k] = iv;
                }
            }
            load_plane(f, L.k2, gxy, q + PD, G.nm, plane, pf[i], pk[i]);
            __syncthreads();

            // result on plane p = q - 1 (u2 of planes p - 1, p, p + 1 in ua, ub, uc)
            const int p = q - 1;
            if (p < G.m0 || p >= pend) continue;
            const cx<T>* U0 = su + ((p + 1) % 3) * S::NW;
            const cx<T> cmz = tzm[p - G.m0 + 1], cpz = tzp[p - G.m0 + 1];
#pragma unroll
            for (int k = 0; k < S::KI; ++k) {
                const int idx = t + k * BS;
                if (idx >= S::NI || !((iin >> k) & 1u)) continue;
                const int ix = idx % TX, iy = (D == 3) ? idx / TX : 0;
                const int c = (iy + S::HY) * S::WX + ix + 1;
                cx<T> au = jmul<T>(dp[k], ub[k]);
                au = jmad<T>(au, cxm[k], U0[c - 1]);
                au = jmad<T>(au, cxp[k], U0[c + 1]);
                if constexpr (D == 3) {
                    au = jmad<T>(au, cym[k], U0[c - S::WX]);
                    au = jmad<T>(au, cyp[k], U0[c + S::WX]);
                }
                au = jmad<T>(au, cmz, ua[k]);
                au = jmad<T>(au, cpz, uc[k]);
                const cx<T> u3 = ub[k] + jdiv<T>(jmul<T>(L.omega, fvp[k] - au), dp[k], ivp[k]);
                const long long g = p * plane + (long long)(G.y0 + iy) * G.nx + G.x0 + ix;
                if constexpr (ACC) {
                    out[g] = out[g].get() + cvt<TO>(u3);
                } else {
                    out[g] = cvt<TO>(u3);
                }
            }
        }
    }
}

#undef MG_LOAD_COARSE
#undef MG_STORE_COARSE

// Sweep configurations (tile x, tile y, planes per chunk, threads), ids 0,
// 1, 2.  The thread counts cover the u1 region of a plane in one pass where
// the registers allow it (2D row segments of 256 (512) points need 259 (515)
// u1 values per row; a 3D 64 x 8 column needs 67 x 11).  The inputs are
// loaded SWEEP_AHEAD planes ahead: with one or two workgroups per CU that
// keeps some 60 KB of loads in flight per CU.
constexpr int SWEEP_AHEAD = 4;
constexpr int SWEEPS_2D[NUM_SWEEP_SHAPES][4] = {{256, 1, 16, 320}, {512, 1, 16, 576}, {256, 1, 32, 320}};
constexpr int SWEEPS_3D[NUM_SWEEP_SHAPES][4] = {{64, 8, 16, 768}, {32, 8, 16, 448}, {64, 4, 16, 384}};

#define MG_SWEEP_SWITCH(LAUNCH)                          \
    if (dim == 2) {                                      \
        switch (sweep) {                                 \
            case 1: LAUNCH(2, 512, 1, 16, 576); break;   \
            case 2: LAUNCH(2, 256, 1, 32, 320); break;   \
            default: LAUNCH(2, 256, 1, 16, 320); break;  \
        }                                                \
    } else {                                             \
        switch (sweep) {                                 \
            case 1: LAUNCH(3, 32, 8, 16, 448); break;    \
            case 2: LAUNCH(3, 64, 4, 16, 384); break;    \
            default: LAUNCH(3, 64, 8, 16, 768); break;   \
        }                                                \
    }

template <typename T, typename TF>
hipError_t sweep_sr(int dim, int sweep, const CycleArgs& a, hipStream_t s) {
#define SW(D, X, Y, Z, B) \
    hipLaunchKernelGGL((k_sweep_sr<D, T, TF, X, Y, Z, B, SWEEP_AHEAD>), dim3(a.st.ntiles), dim3(B), 0, s, a);
    MG_SWEEP_SWITCH(SW)
#undef SW
    return hipGetLastError();
}

template <typename T, typename TF, typename TO, bool ACC>
hipError_t sweep_ps(int dim, int sweep, const CycleArgs& a, hipStream_t s) {
#define SW(D, X, Y, Z, B) \
    hipLaunchKernelGGL((k_sweep_ps<D, T, TF, TO, ACC, X, Y, Z, B, SWEEP_AHEAD>), dim3(a.st.ntiles), dim3(B), 0, s, a);
    MG_SWEEP_SWITCH(SW)
#undef SW
    return hipGetLastError();
}

template <typename T, typename TF, bool ZERO>
hipError_t sr_launch(int dim, int shape, const CycleArgs& a, hipStream_t s) {
    dim3 grid(a.st.ntiles);
#define SR(D, X, Y, Z) hipLaunchKernelGGL((k_smooth_restrict<D, T, TF, ZERO, X, Y, Z>), grid, dim3(NT), 0, s, a);
    MG_SHAPE_SWITCH(SR)
#undef SR
    return hipGetLastError();
}

template <typename T, typename TF, typename TO, bool ZERO, bool ACC>
hipError_t ps_launch(int dim, int shape, const CycleArgs& a, hipStream_t s) {
    dim3 grid(a.st.ntiles);
#define PS(D, X, Y, Z) \
    hipLaunchKernelGGL((k_prolong_smooth<D, T, TF, TO, ZERO, ACC, X, Y, Z>), grid, dim3(NT), 0, s, a);
    MG_SHAPE_SWITCH(PS)
#undef PS
    return hipGetLastError();
}

}  // namespace

hipError_t launch_smooth_restrict(int dim, bool f32, bool level0, bool zero, int shape, const CycleArgs& a,
                                  hipStream_t s) {
    if (a.st.n <= 0) return hipSuccess;
    if (!f32) {
        return zero ? sr_launch<double, double, true>(dim, shape, a, s)
                    : sr_launch<double, double, false>(dim, shape, a, s);
    }
    if (!zero) return hipErrorInvalidValue;   // the complex64 cycle always starts from zero
    return level0 ? sr_launch<float, double, true>(dim, shape, a, s) : sr_launch<float, float, true>(dim, shape, a, s);
}

hipError_t launch_prolong_smooth(int dim, bool f32, bool level0, bool zero, bool acc, int shape,
                                 const CycleArgs& a, hipStream_t s) {
    if (a.st.n <= 0) return hipSuccess;
    if (!f32) {
        if (zero)
            return acc ? ps_launch<double, double, double, true, true>(dim, shape, a, s)
                       : ps_launch<double, double, double, true, false>(dim, shape, a, s);
        return acc ? ps_launch<double, double, double, false, true>(dim, shape, a, s)
                   : ps_launch<double, double, double, false, false>(dim, shape, a, s);
    }
    if (!zero) return hipErrorInvalidValue;
    if (!level0) return ps_launch<float, float, float, true, false>(dim, shape, a, s);
    return acc ? ps_launch<float, double, double, true, true>(dim, shape, a, s)
               : ps_launch<float, double, double, true, false>(dim, shape, a, s);
}

void sweep_counts(int dim, int sweep, const int n[3], int nt[3]) {
    if (sweep < 0 || sweep >= NUM_SWEEP_SHAPES) sweep = 0;
    const int* c = dim == 2 ? SWEEPS_2D[sweep] : SWEEPS_3D[sweep];
    nt[0] = (n[0] + c[0] - 1) / c[0];
    nt[1] = dim == 3 ? (n[1] + c[1] - 1) / c[1] : 1;
    nt[2] = (n[dim - 1] + c[2] - 1) / c[2];
}

hipError_t launch_sweep_sr(int dim, bool f32, bool level0, int sweep, const CycleArgs& a, hipStream_t s) {
    if (a.st.n <= 0) return hipSuccess;
    if (!f32) return sweep_sr<double, double>(dim, sweep, a, s);
    return level0 ? sweep_sr<float, double>(dim, sweep, a, s) : sweep_sr<float, float>(dim, sweep, a, s);
}

hipError_t launch_sweep_ps(int dim, bool f32, bool level0, bool accumulate, int sweep, const CycleArgs& a,
                           hipStream_t s) {
    if (a.st.n <= 0) return hipSuccess;
    if (!f32)
        return accumulate ? sweep_ps<double, double, double, true>(dim, sweep, a, s)
                          : sweep_ps<double, double, double, false>(dim, sweep, a, s);
    if (!level0) return sweep_ps<float, float, float, false>(dim, sweep, a, s);
    return accumulate ? sweep_ps<float, double, double, true>(dim, sweep, a, s)
                      : sweep_ps<float, double, double, false>(dim, sweep, a, s);
}

}  // namespace mg
