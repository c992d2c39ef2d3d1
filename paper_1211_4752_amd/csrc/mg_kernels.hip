// gfx950 kernels of the level-dependent complex-shifted multigrid cycle.
//
// Hot kernels (bandwidth-bound, no dense contraction anywhere, so no MFMA):
//   k_smooth_restrict  omega-Jacobi pre-smoothing (Sec. 3.2.1, eq. wjacobi),
//                      residual of the smoothed iterate and full-weighting
//                      restriction to the next level (Sec. 2.1, Sec. 3.1,
//                      eq. erreq1 with c = 1), fused through LDS tiles with
//                      a two-point halo; optional ||f - A u||^2 partials of
//                      the incoming iterate.
//   k_prolong_smooth   (bi/tri)linear interpolation of the coarse correction,
//                      v <- v + e (Sec. 3.1), and omega-Jacobi
//                      post-smoothing, fused through LDS tiles.
//   k_matvec_dot / k_update_dot / k_update_norm
//                      the GMRES Arnoldi step (Sec. 4.1: one cycle per outer
//                      step) as three passes of classical Gram-Schmidt with
//                      re-orthogonalisation, each fused with its dot products.
// Reductions are two-stage and deterministic: per-workgroup partials in a
// fixed tree, then a fixed-order sum per value.
//
// Level operator (Sec. 3.1, eq. cslvariant): A~ u = sum_axes (cm u_- + c0 u +
// cp u_+) - sigma k^2 u, zero Dirichlet ghosts; D = sum_axes c0 - sigma k^2.

#include "mg_device.hpp"

namespace mg {

namespace {

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

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
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

template <int D, typename T>
__device__ __forceinline__ cx<T> diag_at(const LevelView<T>& L, int gx, int gy, int gz, T k2) {
    cx<T> d = L.c0[0][gx] + L.c0[1][gy];
    if constexpr (D == 3) d = d + L.c0[2][gz];
    return d - k2 * L.sigma;
}

// ---------------------------------------------------------------------------
// Fused pre-smooth + residual + full weighting.
// Tile: fine points [x0, x0+TX) x [y0, y0+TY) (x [z0, z0+TZ)); it owns the
// coarse points whose centre 2C+1 lies in the tile.  LDS regions, relative to
// the tile origin: u on [-2, T+2], u1 on [-1, T+1], r on [0, T].
// ---------------------------------------------------------------------------
template <int D, typename T, typename TF, bool ZERO, int TX, int TY, int TZ>
__global__ void __launch_bounds__(NT) k_smooth_restrict(const SmoothRestrictArgs<T, TF> a) {
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

    const LevelView<T>& L = a.lv;
    const int nx = L.n[0], ny = L.n[1], nz = L.n[2];
    const int ntile = a.ntiles[0] * a.ntiles[1] * a.ntiles[2];
    const int pid = xcd_remap(blockIdx.x, gridDim.x);
    const int slot = pid / ntile;
    int t = pid - slot * ntile;
    const int tile = t;
    const int tx = t % a.ntiles[0];
    t /= a.ntiles[0];
    const int ty = t % a.ntiles[1];
    const int tz = t / a.ntiles[1];
    const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZE;
    const Slot sl = a.st.s[slot];
    const cx<TF>* f = a.f + (a.f_by_slot ? (long long)sl.buf * L.N : sl.in_off);
    const T fs = a.f_by_slot ? T(1) : (T)sl.in_scale;

    if constexpr (!ZERO) {
        const cx<T>* u = a.u + (long long)sl.rhs * L.N;
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
            const cx<T> fv = fs * cvt<T>(f[g]);
            const cx<T> d = diag_at<D>(L, gx, gy, gz, L.k2[g]);
            if constexpr (ZERO) {
                u1 = cdiv(L.omega * fv, d);
            } else {
                const int c = ((D == 3 ? lz + 1 : 0) * UY + (ly + 1)) * UX + (lx + 1);
                const cx<T> uc = s0[c];
                cx<T> au = d * uc + L.cm[0][gx] * s0[c - 1] + L.cp[0][gx] * s0[c + 1] +
                           L.cm[1][gy] * s0[c - UX] + L.cp[1][gy] * s0[c + UX];
                if constexpr (D == 3) au = au + L.cm[2][gz] * s0[c - UX * UY] + L.cp[2][gz] * s0[c + UX * UY];
                const cx<T> res = fv - au;
                u1 = uc + cdiv(L.omega * res, d);
                const bool own = lx >= 1 && lx <= TX && ly >= 1 && ly <= TY && (D == 2 || (lz >= 1 && lz <= TZ));
                if (own) {
                    nrm += (double)abs2(res);
                    if (a.u1) a.u1[(long long)sl.buf * L.N + g] = u1;
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
            const cx<T> fv = fs * cvt<T>(f[g]);
            const cx<T> d = diag_at<D>(L, gx, gy, gz, L.k2[g]);
            const int c = ((D == 3 ? lz + 1 : 0) * VY + (ly + 1)) * VX + (lx + 1);
            cx<T> au = d * s1[c] + L.cm[0][gx] * s1[c - 1] + L.cp[0][gx] * s1[c + 1] +
                       L.cm[1][gy] * s1[c - VX] + L.cp[1][gy] * s1[c + VX];
            if constexpr (D == 3) au = au + L.cm[2][gz] * s1[c - VX * VY] + L.cp[2][gz] * s1[c + VX * VY];
            r = fv - au;
        }
        s0[idx] = r;
    }
    __syncthreads();

    const int ncx = a.nc[0], ncy = a.nc[1], ncz = a.nc[2];
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
                        acc = acc + w * s0[row + ox];
                    }
                }
            }
            a.fc[(long long)sl.buf * a.Nc + ((long long)Cz * ncy + Cy) * ncx + Cx] = acc;
        }
    }

    if constexpr (!ZERO) {
        if (a.norm_part) {
            const double s = block_sum(nrm, sred);
            if (threadIdx.x == 0) a.norm_part[(long long)slot * ntile + tile] = s;
        }
    }
}

// ---------------------------------------------------------------------------
// Fused prolongation + correction + post-smooth.
// LDS: coarse correction on [x0/2 - 1, x0/2 + TX/2], corrected iterate u2 on
// fine [-1, T] relative to the tile.
// ---------------------------------------------------------------------------
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

template <int D, typename T, typename TF, typename TO, bool ZERO, bool ACC, int TX, int TY, int TZ>
__global__ void __launch_bounds__(NT) k_prolong_smooth(const ProlongSmoothArgs<T, TF, TO> a) {
    constexpr int TZE = (D == 3) ? TZ : 1;
    constexpr int EX = TX / 2 + 2, EY = TY / 2 + 2, EZ = (D == 3) ? TZ / 2 + 2 : 1;
    constexpr int WX = TX + 2, WY = TY + 2, WZ = (D == 3) ? TZ + 2 : 1;
    constexpr int NE = EX * EY * EZ, NW = WX * WY * WZ;

    __shared__ cx<T> se[NE];
    __shared__ cx<T> s2[NW];

    const LevelView<T>& L = a.lv;
    const int nx = L.n[0], ny = L.n[1], nz = L.n[2];
    const int ncx = a.nc[0], ncy = a.nc[1], ncz = a.nc[2];
    const int ntile = a.ntiles[0] * a.ntiles[1] * a.ntiles[2];
    const int pid = xcd_remap(blockIdx.x, gridDim.x);
    const int slot = pid / ntile;
    int t = pid - slot * ntile;
    const int tx = t % a.ntiles[0];
    t /= a.ntiles[0];
    const int ty = t % a.ntiles[1];
    const int tz = t / a.ntiles[1];
    const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZE;
    const Slot sl = a.st.s[slot];
    const cx<TF>* f = a.f + (a.f_by_slot ? (long long)sl.buf * L.N : sl.in_off);
    const T fs = a.f_by_slot ? T(1) : (T)sl.in_scale;
    const cx<T>* ec = a.ec + (long long)sl.buf * a.Nc;
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
                const cx<T> fv = fs * cvt<T>(f[g]);
                u1 = cdiv(L.omega * fv, diag_at<D>(L, gx, gy, gz, L.k2[g]));
            } else {
                u1 = a.u1[(long long)sl.buf * L.N + g];
            }
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
            u2 = u1 + pe;
        }
        s2[idx] = u2;
    }
    __syncthreads();

    cx<TO>* out = a.out + (a.out_by_slot ? (long long)sl.buf * L.N : sl.out_off);
    for (int idx = threadIdx.x; idx < TX * TY * TZE; idx += NT) {
        const int lx = idx % TX;
        const int rr = idx / TX;
        const int ly = rr % TY;
        const int lz = rr / TY;
        const int gx = x0 + lx, gy = y0 + ly;
        const int gz = (D == 3) ? z0 + lz : 0;
        if (gx < nx && gy < ny && (D == 2 || gz < nz)) {
            const long long g = ((long long)gz * ny + gy) * nx + gx;
            const cx<T> fv = fs * cvt<T>(f[g]);
            const cx<T> d = diag_at<D>(L, gx, gy, gz, L.k2[g]);
            const int c = ((D == 3 ? lz + 1 : 0) * WY + (ly + 1)) * WX + (lx + 1);
            const cx<T> u2c = s2[c];
            cx<T> au = d * u2c + L.cm[0][gx] * s2[c - 1] + L.cp[0][gx] * s2[c + 1] +
                       L.cm[1][gy] * s2[c - WX] + L.cp[1][gy] * s2[c + WX];
            if constexpr (D == 3) au = au + L.cm[2][gz] * s2[c - WX * WY] + L.cp[2][gz] * s2[c + WX * WY];
            const cx<T> u3 = u2c + cdiv(L.omega * (fv - au), d);
            if constexpr (ACC) {
                out[g] = out[g] + cvt<TO>(u3);
            } else {
                out[g] = cvt<TO>(u3);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Coarsest level: LU forward/back substitution, one workgroup per slot, in
// FP64 whatever the cycle precision.  lu: row-major n x n, unit-lower L below
// the diagonal, U on and above; piv: row interchanges in elimination order.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(NT) k_coarse_solve(const cx<double>* lu, const int* piv, int n,
                                                      const SlotTable st, const cx<T>* f, cx<T>* e) {
    __shared__ cx<double> b[MAX_COARSE];
    const long long base = (long long)st.s[blockIdx.x].buf * n;
    for (int i = threadIdx.x; i < n; i += NT) b[i] = cvt<double>(f[base + i]);
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
        for (int i = k + 1 + threadIdx.x; i < n; i += NT) b[i] = b[i] - lu[(long long)i * n + k] * bk;
        __syncthreads();
    }
    for (int k = n - 1; k >= 0; --k) {
        if (threadIdx.x == 0) b[k] = cdiv(b[k], lu[(long long)k * n + k]);
        __syncthreads();
        const cx<double> bk = b[k];
        for (int i = threadIdx.x; i < k; i += NT) b[i] = b[i] - lu[(long long)i * n + k] * bk;
        __syncthreads();
    }
    for (int i = threadIdx.x; i < n; i += NT) e[base + i] = cvt<T>(b[i]);
}

// ---------------------------------------------------------------------------
// Residual / operator application, one point per thread, contiguous chunk
// per workgroup.
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ cx<double> apply_at(const LevelView<double>& L, const cx<double>* x, int p,
                                               int gx, int gy, int gz) {
    const int nx = L.n[0], ny = L.n[1], nz = L.n[2];
    cx<double> ax = diag_at<D>(L, gx, gy, gz, L.k2[p]) * x[p];
    if (gx > 0) ax = ax + L.cm[0][gx] * x[p - 1];
    if (gx < nx - 1) ax = ax + L.cp[0][gx] * x[p + 1];
    if (gy > 0) ax = ax + L.cm[1][gy] * x[p - nx];
    if (gy < ny - 1) ax = ax + L.cp[1][gy] * x[p + nx];
    if constexpr (D == 3) {
        const int sz = nx * ny;
        if (gz > 0) ax = ax + L.cm[2][gz] * x[p - sz];
        if (gz < nz - 1) ax = ax + L.cp[2][gz] * x[p + sz];
    }
    return ax;
}

__device__ __forceinline__ void chunk_range(long long N, int nblocks, int b, int& lo, int& hi) {
    const long long per = (N + nblocks - 1) / nblocks;
    long long l = per * b, h = l + per;
    if (l > N) l = N;
    if (h > N) h = N;
    lo = (int)l;
    hi = (int)h;
}

template <int D>
__global__ void __launch_bounds__(NT) k_residual(const ResidualArgs a) {
    __shared__ double sred[NT / 64];
    const LevelView<double>& L = a.lv;
    const int slot = blockIdx.y;
    const Slot sl = a.st.s[slot];
    const long long N = L.N;
    const cx<double>* x = a.x + (long long)sl.rhs * N;
    const cx<double>* f = a.f ? a.f + (long long)sl.rhs * N : nullptr;
    cx<double>* y = a.y + sl.out_off;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    int lo, hi;
    chunk_range(N, gridDim.x, b, lo, hi);
    double nrm = 0.0;
    const int nx = L.n[0], ny = L.n[1];
    for (int p = lo + (int)threadIdx.x; p < hi; p += NT) {
        const int gx = p % nx;
        const int rr = p / nx;
        const int gy = rr % ny;
        const int gz = rr / ny;
        cx<double> v = apply_at<D>(L, x, p, gx, gy, gz);
        if (f) v = f[p] - v;
        y[p] = v;
        nrm += abs2(v);
    }
    if (a.norm_part) {
        const double s = block_sum(nrm, sred);
        if (threadIdx.x == 0) a.norm_part[(long long)slot * gridDim.x + b] = s;
    }
}

__global__ void __launch_bounds__(NT) k_norm(const SlotTable st, const cx<double>* x, bool by_buf,
                                             long long N, double* part) {
    __shared__ double sred[NT / 64];
    const int slot = blockIdx.y;
    const Slot sl = st.s[slot];
    const cx<double>* v = x + (by_buf ? (long long)sl.buf : (long long)sl.rhs) * N;
    int lo, hi;
    chunk_range(N, gridDim.x, blockIdx.x, lo, hi);
    double nrm = 0.0;
    for (int p = lo + (int)threadIdx.x; p < hi; p += NT) nrm += abs2(v[p]);
    const double s = block_sum(nrm, sred);
    if (threadIdx.x == 0) part[(long long)slot * gridDim.x + blockIdx.x] = s;
}

// ---------------------------------------------------------------------------
// GMRES passes.  Each slot has basis vectors V_0..V_j (j = slot.j) stored
// unnormalised with v_i = scale_i V_i.
// ---------------------------------------------------------------------------
template <int MAXJ>
__device__ __forceinline__ void block_sum_vec(cx<double> (&acc)[MAXJ], int nv, cx<double>* sm,
                                              cx<double>* dst, int nblocks, int b) {
    // sm: (NT/64) * MAXJ complex
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < MAXJ; ++i) {
        if (i < nv) {
            const double r = wave_sum(acc[i].r);
            const double im = wave_sum(acc[i].i);
            if (lane == 0) sm[wave * MAXJ + i] = mk(r, im);
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < nv) {
        cx<double> s = mk(0.0, 0.0);
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) s = s + sm[w * MAXJ + threadIdx.x];
        dst[(long long)threadIdx.x * nblocks + b] = s;
    }
}

template <int D, int MAXJ>
__global__ void __launch_bounds__(NT) k_matvec_dot(const OrthoArgs a) {
    __shared__ cx<double> sm[(NT / 64) * MAXJ];
    const LevelView<double>& L = a.lv;
    const int slot = blockIdx.y;
    const Slot sl = a.st.s[slot];
    const int nv = sl.j + 1;
    const long long N = a.N;
    const cx<double>* z = a.z + (long long)sl.buf * N;
    cx<double>* w = a.w + (long long)sl.buf * N;
    const cx<double>* V = a.Vb + (long long)sl.rhs * a.vstride * N;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    int lo, hi;
    chunk_range(N, gridDim.x, b, lo, hi);
    cx<double> acc[MAXJ];
#pragma unroll
    for (int i = 0; i < MAXJ; ++i) acc[i] = mk(0.0, 0.0);
    const int nx = L.n[0], ny = L.n[1];
    for (int p = lo + (int)threadIdx.x; p < hi; p += NT) {
        const int gx = p % nx;
        const int rr = p / nx;
        const int gy = rr % ny;
        const int gz = rr / ny;
        const cx<double> wv = apply_at<D>(L, z, p, gx, gy, gz);
        w[p] = wv;
#pragma unroll
        for (int i = 0; i < MAXJ; ++i)
            if (i < nv) acc[i] = acc[i] + cmulc(V[(long long)i * N + p], wv);
    }
    const double* sc = a.scale + (long long)sl.rhs * a.sstride;
#pragma unroll
    for (int i = 0; i < MAXJ; ++i)
        if (i < nv) acc[i] = sc[i] * acc[i];
    block_sum_vec<MAXJ>(acc, nv, sm, a.part + (long long)slot * a.pstride * a.nblocks, a.nblocks, b);
}

template <int MAXJ>
__global__ void __launch_bounds__(NT) k_update_dot(const OrthoArgs a) {
    __shared__ cx<double> sm[(NT / 64) * MAXJ];
    const int slot = blockIdx.y;
    const Slot sl = a.st.s[slot];
    const int nv = sl.j + 1;
    const long long N = a.N;
    cx<double>* w = a.w + (long long)sl.buf * N;
    const cx<double>* V = a.Vb + (long long)sl.rhs * a.vstride * N;
    const double* sc = a.scale + (long long)sl.rhs * a.sstride;
    const cx<double>* h = a.hin + (long long)slot * a.hstride;
    cx<double> coef[MAXJ];
#pragma unroll
    for (int i = 0; i < MAXJ; ++i) coef[i] = (i < nv) ? sc[i] * h[i] : mk(0.0, 0.0);
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    int lo, hi;
    chunk_range(N, gridDim.x, b, lo, hi);
    cx<double> acc[MAXJ];
#pragma unroll
    for (int i = 0; i < MAXJ; ++i) acc[i] = mk(0.0, 0.0);
    for (int p = lo + (int)threadIdx.x; p < hi; p += NT) {
        cx<double> vv[MAXJ];
#pragma unroll
        for (int i = 0; i < MAXJ; ++i) vv[i] = (i < nv) ? V[(long long)i * N + p] : mk(0.0, 0.0);
        cx<double> wv = w[p];
#pragma unroll
        for (int i = 0; i < MAXJ; ++i) wv = wv - coef[i] * vv[i];
        w[p] = wv;
#pragma unroll
        for (int i = 0; i < MAXJ; ++i) acc[i] = acc[i] + cmulc(vv[i], wv);
    }
#pragma unroll
    for (int i = 0; i < MAXJ; ++i)
        if (i < nv) acc[i] = sc[i] * acc[i];
    block_sum_vec<MAXJ>(acc, nv, sm, a.part + (long long)slot * a.pstride * a.nblocks, a.nblocks, b);
}

template <int MAXJ>
__global__ void __launch_bounds__(NT) k_update_norm(const OrthoArgs a) {
    __shared__ double sred[NT / 64];
    const int slot = blockIdx.y;
    const Slot sl = a.st.s[slot];
    const int nv = sl.j + 1;
    const long long N = a.N;
    const cx<double>* w = a.w + (long long)sl.buf * N;
    cx<double>* V = a.Vb + (long long)sl.rhs * a.vstride * N;
    const double* sc = a.scale + (long long)sl.rhs * a.sstride;
    const cx<double>* h = a.hin + (long long)slot * a.hstride;
    cx<double> coef[MAXJ];
#pragma unroll
    for (int i = 0; i < MAXJ; ++i) coef[i] = (i < nv) ? sc[i] * h[i] : mk(0.0, 0.0);
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    int lo, hi;
    chunk_range(N, gridDim.x, b, lo, hi);
    cx<double>* vout = V + (long long)nv * N;
    double nrm = 0.0;
    for (int p = lo + (int)threadIdx.x; p < hi; p += NT) {
        cx<double> wv = w[p];
#pragma unroll
        for (int i = 0; i < MAXJ; ++i)
            if (i < nv) wv = wv - coef[i] * V[(long long)i * N + p];
        vout[p] = wv;
        nrm += abs2(wv);
    }
    const double s = block_sum(nrm, sred);
    if (threadIdx.x == 0) a.part[(long long)slot * a.pstride * a.nblocks + b] = mk(s, 0.0);
}

template <int MAXJ>
__global__ void __launch_bounds__(NT) k_combine(const CombineArgs a) {
    const int slot = blockIdx.y;
    const Slot sl = a.st.s[slot];
    const int nv = sl.j + 1;
    const long long N = a.N;
    const cx<double>* V = a.Vb + (long long)sl.rhs * a.vstride * N;
    const cx<double>* c = a.coef + (long long)sl.rhs * a.sstride;
    cx<double> coef[MAXJ];
#pragma unroll
    for (int i = 0; i < MAXJ; ++i) coef[i] = (i < nv) ? c[i] : mk(0.0, 0.0);
    cx<double>* t = a.t + (long long)sl.buf * N;
    int lo, hi;
    chunk_range(N, gridDim.x, xcd_remap(blockIdx.x, gridDim.x), lo, hi);
    for (int p = lo + (int)threadIdx.x; p < hi; p += NT) {
        cx<double> s = mk(0.0, 0.0);
#pragma unroll
        for (int i = 0; i < MAXJ; ++i)
            if (i < nv) s = s + coef[i] * V[(long long)i * N + p];
        t[p] = s;
    }
}

// ---------------------------------------------------------------------------
// Second reduction stage, fixed order.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(NT) k_reduce_complex(const cx<double>* part, int vstride, int nblocks,
                                                       cx<double>* out, int ostride) {
    __shared__ double sr[NT / 64], si[NT / 64];
    const int v = blockIdx.x, slot = blockIdx.y;
    const cx<double>* p = part + ((long long)slot * vstride + v) * nblocks;
    double r = 0.0, im = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += NT) {
        r += p[b].r;
        im += p[b].i;
    }
    r = block_sum(r, sr);
    im = block_sum(im, si);
    if (threadIdx.x == 0) out[(long long)slot * ostride + v] = mk(r, im);
}

__global__ void __launch_bounds__(NT) k_reduce_real(const double* part, int nblocks, double* out) {
    __shared__ double sr[NT / 64];
    const int slot = blockIdx.x;
    const double* p = part + (long long)slot * nblocks;
    double r = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += NT) r += p[b];
    r = block_sum(r, sr);
    if (threadIdx.x == 0) out[slot] = r;
}

// ---------------------------------------------------------------------------
// Set-up and small helpers.
// ---------------------------------------------------------------------------
__global__ void k_inject_k2(const double* fine, int nfx, int nfy, double* coarse, int ncx, int ncy,
                            long long Nc, int dim) {
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= Nc) return;
    const int x = (int)(p % ncx);
    const long long rr = p / ncx;
    const int y = (int)(rr % ncy);
    const int z = (int)(rr / ncy);
    const long long fz = (dim == 3) ? 2LL * z + 1 : 0;
    coarse[p] = fine[(fz * nfy + 2LL * y + 1) * nfx + 2LL * x + 1];
}

__global__ void k_to_f32(const double* src, float* dst, long long n) {
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) dst[p] = (float)src[p];
}

__global__ void k_grad_k2(const cx<double>* u, const cx<double>* lam, int nrhs, long long N, double* grad) {
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    double g = 0.0;
    for (int r = 0; r < nrhs; ++r) {
        const cx<double> a = lam[(long long)r * N + p];
        const cx<double> b = u[(long long)r * N + p];
        g += a.r * b.r + a.i * b.i;
    }
    grad[p] += g;
}

__global__ void k_fill_zero(uint4* p, long long n16) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n16) p[i] = make_uint4(0u, 0u, 0u, 0u);
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
namespace {
// tile shapes (x, y, z) of the fused kernels
constexpr int T2X = 64, T2Y = 16;
constexpr int T3X = 16, T3Y = 8, T3Z = 4;

inline int cdivi(int a, int b) { return (a + b - 1) / b; }
}  // namespace

void tile_counts(int dim, bool /*f32*/, const int n[3], int ntiles[3]) {
    if (dim == 2) {
        ntiles[0] = cdivi(n[0], T2X);
        ntiles[1] = cdivi(n[1], T2Y);
        ntiles[2] = 1;
    } else {
        ntiles[0] = cdivi(n[0], T3X);
        ntiles[1] = cdivi(n[1], T3Y);
        ntiles[2] = cdivi(n[2], T3Z);
    }
}

template <int D, typename T, typename TF, bool ZERO>
static hipError_t sr_launch(const SmoothRestrictArgs<T, TF>& a, int* nb, hipStream_t s) {
    const int ntile = a.ntiles[0] * a.ntiles[1] * a.ntiles[2];
    if (nb) *nb = ntile;
    dim3 grid(ntile * a.st.n);
    if (D == 2)
        hipLaunchKernelGGL((k_smooth_restrict<2, T, TF, ZERO, T2X, T2Y, 1>), grid, dim3(NT), 0, s, a);
    else
        hipLaunchKernelGGL((k_smooth_restrict<3, T, TF, ZERO, T3X, T3Y, T3Z>), grid, dim3(NT), 0, s, a);
    return hipGetLastError();
}

template <int D, typename T, typename TF, typename TO, bool ZERO, bool ACC>
static hipError_t ps_launch(const ProlongSmoothArgs<T, TF, TO>& a, hipStream_t s) {
    const int ntile = a.ntiles[0] * a.ntiles[1] * a.ntiles[2];
    dim3 grid(ntile * a.st.n);
    if (D == 2)
        hipLaunchKernelGGL((k_prolong_smooth<2, T, TF, TO, ZERO, ACC, T2X, T2Y, 1>), grid, dim3(NT), 0, s, a);
    else
        hipLaunchKernelGGL((k_prolong_smooth<3, T, TF, TO, ZERO, ACC, T3X, T3Y, T3Z>), grid, dim3(NT), 0, s,
                           a);
    return hipGetLastError();
}

hipError_t launch_smooth_restrict_f64(int dim, bool zero, const SmoothRestrictArgs<double, double>& a,
                                      int* nb, hipStream_t s) {
    if (dim == 2) return zero ? sr_launch<2, double, double, true>(a, nb, s) : sr_launch<2, double, double, false>(a, nb, s);
    return zero ? sr_launch<3, double, double, true>(a, nb, s) : sr_launch<3, double, double, false>(a, nb, s);
}

hipError_t launch_smooth_restrict_f32(int dim, bool level0, const SmoothRestrictArgs<float, double>& a0,
                                      const SmoothRestrictArgs<float, float>& ac, int* nb, hipStream_t s) {
    if (dim == 2) return level0 ? sr_launch<2, float, double, true>(a0, nb, s) : sr_launch<2, float, float, true>(ac, nb, s);
    return level0 ? sr_launch<3, float, double, true>(a0, nb, s) : sr_launch<3, float, float, true>(ac, nb, s);
}

hipError_t launch_prolong_smooth_f64(int dim, bool zero, bool acc,
                                     const ProlongSmoothArgs<double, double, double>& a, hipStream_t s) {
    if (dim == 2) {
        if (zero) return acc ? ps_launch<2, double, double, double, true, true>(a, s)
                             : ps_launch<2, double, double, double, true, false>(a, s);
        return acc ? ps_launch<2, double, double, double, false, true>(a, s)
                   : ps_launch<2, double, double, double, false, false>(a, s);
    }
    if (zero) return acc ? ps_launch<3, double, double, double, true, true>(a, s)
                         : ps_launch<3, double, double, double, true, false>(a, s);
    return acc ? ps_launch<3, double, double, double, false, true>(a, s)
               : ps_launch<3, double, double, double, false, false>(a, s);
}

hipError_t launch_prolong_smooth_f32(int dim, bool level0, bool acc,
                                     const ProlongSmoothArgs<float, double, double>& a0,
                                     const ProlongSmoothArgs<float, float, float>& ac, hipStream_t s) {
    if (dim == 2) {
        if (!level0) return ps_launch<2, float, float, float, true, false>(ac, s);
        return acc ? ps_launch<2, float, double, double, true, true>(a0, s)
                   : ps_launch<2, float, double, double, true, false>(a0, s);
    }
    if (!level0) return ps_launch<3, float, float, float, true, false>(ac, s);
    return acc ? ps_launch<3, float, double, double, true, true>(a0, s)
               : ps_launch<3, float, double, double, true, false>(a0, s);
}

hipError_t launch_coarse_solve_f64(const cx<double>* lu, const int* piv, int n, const SlotTable& st,
                                   const cx<double>* f, cx<double>* e, hipStream_t s) {
    hipLaunchKernelGGL((k_coarse_solve<double>), dim3(st.n), dim3(NT), 0, s, lu, piv, n,
                       st, f, e);
    return hipGetLastError();
}

hipError_t launch_coarse_solve_f32(const cx<double>* lu, const int* piv, int n, const SlotTable& st,
                                   const cx<float>* f, cx<float>* e, hipStream_t s) {
    hipLaunchKernelGGL((k_coarse_solve<float>), dim3(st.n), dim3(NT), 0, s, lu, piv, n,
                       st, f, e);
    return hipGetLastError();
}

int residual_blocks(long long N) {
    long long b = (N + NT * 4 - 1) / (NT * 4);
    if (b > 1024) b = 1024;
    if (b < 1) b = 1;
    return (int)b;
}

hipError_t launch_residual(int dim, const ResidualArgs& a, hipStream_t s) {
    dim3 grid(a.nblocks, a.st.n);
    if (dim == 2)
        hipLaunchKernelGGL((k_residual<2>), grid, dim3(NT), 0, s, a);
    else
        hipLaunchKernelGGL((k_residual<3>), grid, dim3(NT), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_norm(const SlotTable& st, const cx<double>* x, bool by_buf, long long N, double* part,
                       int nblocks, hipStream_t s) {
    hipLaunchKernelGGL(k_norm, dim3(nblocks, st.n), dim3(NT), 0, s, st, x, by_buf, N, part);
    return hipGetLastError();
}

int ortho_blocks(long long N) {
    long long b = (N + NT * 8 - 1) / (NT * 8);
    if (b > 1024) b = 1024;
    if (b < 1) b = 1;
    return (int)b;
}

static int jbucket(int jmax) {
    return jmax <= 4 ? 4 : jmax <= 8 ? 8 : jmax <= 16 ? 16 : jmax <= 24 ? 24 : 33;
}

// MAXJ buckets of the GMRES pass kernels (registers scale with MAXJ)
#define MG_JSWITCH(CASE) \
    switch (jbucket(jmax)) { \
        case 4: CASE(4) break; \
        case 8: CASE(8) break; \
        case 16: CASE(16) break; \
        case 24: CASE(24) break; \
        default: CASE(33) break; \
    }

hipError_t launch_matvec_dot(int dim, int jmax, const OrthoArgs& a, hipStream_t s) {
    dim3 grid(a.nblocks, a.st.n);
#define MV(J)                                                                  \
    if (dim == 2)                                                              \
        hipLaunchKernelGGL((k_matvec_dot<2, J>), grid, dim3(NT), 0, s, a);     \
    else                                                                       \
        hipLaunchKernelGGL((k_matvec_dot<3, J>), grid, dim3(NT), 0, s, a);
    MG_JSWITCH(MV)
#undef MV
    return hipGetLastError();
}

hipError_t launch_update_dot(int jmax, const OrthoArgs& a, hipStream_t s) {
    dim3 grid(a.nblocks, a.st.n);
#define UD(J) hipLaunchKernelGGL((k_update_dot<J>), grid, dim3(NT), 0, s, a);
    MG_JSWITCH(UD)
#undef UD
    return hipGetLastError();
}

hipError_t launch_update_norm(int jmax, const OrthoArgs& a, hipStream_t s) {
    dim3 grid(a.nblocks, a.st.n);
#define UN(J) hipLaunchKernelGGL((k_update_norm<J>), grid, dim3(NT), 0, s, a);
    MG_JSWITCH(UN)
#undef UN
    return hipGetLastError();
}

hipError_t launch_combine(int jmax, const CombineArgs& a, hipStream_t s) {
    dim3 grid(ortho_blocks(a.N), a.st.n);
#define CB(J) hipLaunchKernelGGL((k_combine<J>), grid, dim3(NT), 0, s, a);
    MG_JSWITCH(CB)
#undef CB
    return hipGetLastError();
}

hipError_t launch_reduce_complex(const cx<double>* part, int nvals, int vstride, int nblocks, int nslots,
                                 cx<double>* out, int ostride, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_complex, dim3(nvals, nslots), dim3(NT), 0, s, part, vstride, nblocks, out,
                       ostride);
    return hipGetLastError();
}

hipError_t launch_reduce_real(const double* part, int nblocks, int nslots, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_real, dim3(nslots), dim3(NT), 0, s, part, nblocks, out);
    return hipGetLastError();
}

hipError_t launch_inject_k2(int dim, const double* fine, const int nf[3], double* coarse, const int nc[3],
                            hipStream_t s) {
    const long long Nc = (long long)nc[0] * nc[1] * (dim == 3 ? nc[2] : 1);
    hipLaunchKernelGGL(k_inject_k2, dim3((unsigned)((Nc + NT - 1) / NT)), dim3(NT), 0, s, fine, nf[0], nf[1],
                       coarse, nc[0], nc[1], Nc, dim);
    return hipGetLastError();
}

hipError_t launch_to_f32(const double* src, float* dst, long long n, hipStream_t s) {
    hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, s, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_grad_k2(const cx<double>* u, const cx<double>* lam, int nrhs, long long N, double* grad,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_grad_k2, dim3((unsigned)((N + NT - 1) / NT)), dim3(NT), 0, s, u, lam, nrhs, N, grad);
    return hipGetLastError();
}

hipError_t launch_fill_zero(void* p, long long bytes, hipStream_t s) {
    const long long n16 = bytes / 16;
    if (n16 > 0)
        hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((n16 + NT - 1) / NT)), dim3(NT), 0, s, (uint4*)p, n16);
    return hipGetLastError();
}

}  // namespace mg
