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
//   k_matvec_dot / k_update_gram
//                      the GMRES Arnoldi step (Sec. 4.1: one cycle per outer
//                      step) as two passes: w = A z fused with h1 = V^H w,
//                      then v = w - V h fused with V^H v and ||v||^2, where h
//                      is h1 plus the second Gram-Schmidt projection formed
//                      from the Gram matrix of the stored basis.
// Reductions are two-stage and deterministic: per-workgroup partials in a
// fixed tree, then a fixed-order sum per value.
//
// Level operator (Sec. 3.1, eq. cslvariant): A~ u = sum_axes (cm u_- + c0 u +
// cp u_+) - sigma k^2 u, zero Dirichlet ghosts; D = sum_axes c0 - sigma k^2.

#include "mg_kcommon.hpp"

namespace mg {

using namespace kc;

namespace {

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
    const LevelView<T> L = *Lp;
    const int nx = L.n[0], ny = L.n[1], nz = L.n[2];
    const int ntx = (nx + TX - 1) / TX, nty = (ny + TY - 1) / TY;
    const int tx = tile % ntx;
    const int rest = tile / ntx;
    const int ty = rest % nty;
    const int tz = rest / nty;
    const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZE;
    const cx<TF>* f = static_cast<const cx<TF>*>(sl.f);
    const T fs = (T)fscale_of(sl);
    cx<T>* u1p = static_cast<cx<T>*>(sl.u1);

    if constexpr (!ZERO) {
        const cx<T>* u = static_cast<const cx<T>*>(sl.u);
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

    const int ncx = Lp[1].n[0], ncy = Lp[1].n[1], ncz = Lp[1].n[2];
    cx<T>* fc = static_cast<cx<T>*>(sl.c);
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
    const LevelView<T> L = *Lp;
    const int nx = L.n[0], ny = L.n[1], nz = L.n[2];
    const int ncx = Lp[1].n[0], ncy = Lp[1].n[1], ncz = Lp[1].n[2];
    const int ntx = (nx + TX - 1) / TX, nty = (ny + TY - 1) / TY;
    const int tx = tile % ntx;
    const int rest = tile / ntx;
    const int ty = rest % nty;
    const int tz = rest / nty;
    const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZE;
    const cx<TF>* f = static_cast<const cx<TF>*>(sl.f);
    const T fs = (T)fscale_of(sl);
    const cx<T>* ec = static_cast<const cx<T>*>(sl.c);
    const cx<T>* u1in = static_cast<const cx<T>*>(sl.u1);
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
                u1 = u1in[g];
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

    cx<TO>* out = static_cast<cx<TO>*>(sl.out);
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
// Vector kernels: one point per thread, a contiguous chunk of the slot's
// vector per workgroup.
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

// y = f - A x (f null: y = A x); ||y||^2 partials in rpart.
template <int D>
__global__ void __launch_bounds__(NT) k_residual(const VecArgs a) {
    __shared__ double sred[NT / 64];
    VecPos q = vec_pos(a.st);
    const VecSlot& sl = a.st.s[q.slot];
    if (gated_off(sl.gate)) return;
    const LevelView<double> L = *static_cast<const LevelView<double>*>(sl.lv);
    chunk_range(L.N, q.nb, q.b, q.lo, q.hi);
    double nrm = 0.0;
    const int nx = L.n[0], ny = L.n[1];
    for (int p = q.lo + (int)threadIdx.x; p < q.hi; p += NT) {
        const int gx = p % nx;
        const int rr = p / nx;
        const int gy = rr % ny;
        const int gz = rr / ny;
        cx<double> v = apply_at<D>(L, sl.x, p, gx, gy, gz);
        if (sl.f) v = sl.f[p] - v;
        sl.y[p] = v;
        nrm += abs2(v);
    }
    if (a.rpart) {
        const double s = block_sum(nrm, sred);
        if (threadIdx.x == 0) a.rpart[(long long)q.slot * a.bstride + q.b] = s;
    }
}

// ||x||^2 partials.
__global__ void __launch_bounds__(NT) k_norm(const VecArgs a) {
    __shared__ double sred[NT / 64];
    VecPos q = vec_pos(a.st);
    const VecSlot& sl = a.st.s[q.slot];
    if (gated_off(sl.gate)) return;
    const long long N = static_cast<const LevelView<double>*>(sl.lv)->N;
    chunk_range(N, q.nb, q.b, q.lo, q.hi);
    double nrm = 0.0;
    for (int p = q.lo + (int)threadIdx.x; p < q.hi; p += NT) nrm += abs2(sl.x[p]);
    const double s = block_sum(nrm, sred);
    if (threadIdx.x == 0) a.rpart[(long long)q.slot * a.bstride + q.b] = s;
}

// ---------------------------------------------------------------------------
// GMRES passes.  Each slot has basis vectors V_0..V_j (j = slot.j) stored
// unnormalised with v_i = scale_i V_i.
// ---------------------------------------------------------------------------
template <int MAXJ>
__device__ __forceinline__ void block_sum_vec(cx<double> (&acc)[MAXJ], int nv, cx<double>* sm,
                                              cx<double>* dst, long long bstride, int b) {
    // sm: (NT/64) * MAXJ complex; dst[i * bstride + b] for i < nv
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
        dst[(long long)threadIdx.x * bstride + b] = s;
    }
}

// w = A z, h_i = <v_i, w>.
template <int D, int MAXJ>
__global__ void __launch_bounds__(NT) k_matvec_dot(const VecArgs a) {
    __shared__ cx<double> sm[(NT / 64) * MAXJ];
    VecPos q = vec_pos(a.st);
    const VecSlot& sl = a.st.s[q.slot];
    if (gated_off(sl.gate)) return;
    const LevelView<double> L = *static_cast<const LevelView<double>*>(sl.lv);
    const long long N = L.N;
    const int nv = sl.j + 1;
    const cx<double>* z = sl.x;
    cx<double>* w = sl.y;
    const cx<double>* V = sl.V;
    chunk_range(N, q.nb, q.b, q.lo, q.hi);
    cx<double> acc[MAXJ];
#pragma unroll
    for (int i = 0; i < MAXJ; ++i) acc[i] = mk(0.0, 0.0);
    const int nx = L.n[0], ny = L.n[1];
    if constexpr (D == 2) {
        // Column marching: workgroup b owns NT consecutive columns of a strip
        // of rows (b = row strip * ncb + column block); each thread walks
        // down its column keeping the rows above, at and below in registers,
        // so every z value is fetched once.  The host sizes the launch with
        // mv_blocks(), i.e. nb = ncb * (number of row strips).
        const int ncb = (nx + NT - 1) / NT;
        const int nrs = q.nb / ncb;
        const int rows = (ny + nrs - 1) / nrs;
        const int gx = (q.b % ncb) * NT + (int)threadIdx.x;
        const int y0 = (q.b / ncb) * rows;
        const int y1 = y0 + rows < ny ? y0 + rows : ny;
        if (gx < nx && y0 < y1) {
            const cx<double> zero = mk(0.0, 0.0);
            cx<double> zm = y0 > 0 ? z[(y0 - 1) * nx + gx] : zero;
            cx<double> zc = z[y0 * nx + gx];
            for (int gy = y0; gy < y1; ++gy) {
                const int p = gy * nx + gx;
                cx<double> vv[MAXJ];
#pragma unroll
                for (int i = 0; i < MAXJ; ++i) vv[i] = (i < nv) ? V[(long long)i * N + p] : zero;
                const cx<double> zp = gy + 1 < ny ? z[p + nx] : zero;
                // same terms in the same order as apply_at<2>
                cx<double> wv = diag_at<2>(L, gx, gy, 0, L.k2[p]) * zc;
                if (gx > 0) wv = wv + L.cm[0][gx] * z[p - 1];
                if (gx < nx - 1) wv = wv + L.cp[0][gx] * z[p + 1];
                if (gy > 0) wv = wv + L.cm[1][gy] * zm;
                if (gy < ny - 1) wv = wv + L.cp[1][gy] * zp;
                w[p] = wv;
#pragma unroll
                for (int i = 0; i < MAXJ; ++i) acc[i] = acc[i] + cmulc(vv[i], wv);
                zm = zc;
                zc = zp;
            }
        }
#pragma unroll
        for (int i = 0; i < MAXJ; ++i)
            if (i < nv) acc[i] = sl.scale[i] * acc[i];
        block_sum_vec<MAXJ>(acc, nv, sm, a.part + (long long)q.slot * a.pstride * a.bstride, a.bstride, q.b);
        return;
    }
    // grid coordinates of p, carried forward by NT points per iteration
    int p = q.lo + (int)threadIdx.x;
    int gx = p % nx, gy = (p / nx) % ny, gz = p / nx / ny;
    for (; p < q.hi; p += NT) {
        // the basis loads do not depend on the stencil: issue them first
        cx<double> vv[MAXJ];
#pragma unroll
        for (int i = 0; i < MAXJ; ++i) vv[i] = (i < nv) ? V[(long long)i * N + p] : mk(0.0, 0.0);
        const cx<double> wv = apply_at<D>(L, z, p, gx, gy, gz);
        w[p] = wv;
#pragma unroll
        for (int i = 0; i < MAXJ; ++i) acc[i] = acc[i] + cmulc(vv[i], wv);
        gx += NT;
        while (gx >= nx) {
            gx -= nx;
            if (++gy == ny) {
                gy = 0;
                ++gz;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < MAXJ; ++i)
        if (i < nv) acc[i] = sl.scale[i] * acc[i];
    block_sum_vec<MAXJ>(acc, nv, sm, a.part + (long long)q.slot * a.pstride * a.bstride, a.bstride, q.b);
}

// Second pass of the Arnoldi step (classical Gram-Schmidt applied twice
// with one reduction per pass): V_{j+1} = w - sum_i h_i v_i, where h already
// contains the second projection (formed on the device from the Gram
// matrix of the stored basis), fused with the partials of <v_i, V_{j+1}>
// (i <= j; the next column of that Gram matrix) and of ||V_{j+1}||^2 (value
// j + 1).  The coefficients scale_i h_i are staged in LDS.
template <int MAXJ>
__global__ void __launch_bounds__(NT) k_update_gram(const VecArgs a) {
    __shared__ cx<double> sm[(NT / 64) * (MAXJ + 1)];
    __shared__ cx<double> sc[MAXJ];
    VecPos q = vec_pos(a.st);
    const VecSlot& sl = a.st.s[q.slot];
    if (gated_off(sl.gate)) return;
    const long long N = static_cast<const LevelView<double>*>(sl.lv)->N;
    const int nv = sl.j + 1;
    const cx<double>* w = sl.y;
    const cx<double>* V = sl.V;
    if ((int)threadIdx.x < MAXJ) sc[threadIdx.x] = ((int)threadIdx.x < nv) ? sl.scale[threadIdx.x] * sl.hin[threadIdx.x]
                                                                          : mk(0.0, 0.0);
    __syncthreads();
    chunk_range(N, q.nb, q.b, q.lo, q.hi);
    cx<double>* vout = sl.V + (long long)nv * N;
    cx<double> acc[MAXJ + 1];
#pragma unroll
    for (int i = 0; i <= MAXJ; ++i) acc[i] = mk(0.0, 0.0);
    for (int p = q.lo + (int)threadIdx.x; p < q.hi; p += NT) {
        cx<double> vv[MAXJ];
#pragma unroll
        for (int i = 0; i < MAXJ; ++i) vv[i] = (i < nv) ? V[(long long)i * N + p] : mk(0.0, 0.0);
        cx<double> wv = w[p];
#pragma unroll
        for (int i = 0; i < MAXJ; ++i) wv = wv - sc[i] * vv[i];
        vout[p] = wv;
#pragma unroll
        for (int i = 0; i < MAXJ; ++i) acc[i] = acc[i] + cmulc(vv[i], wv);
        acc[MAXJ].r += abs2(wv);
    }
#pragma unroll
    for (int i = 0; i < MAXJ; ++i)
        if (i < nv) acc[i] = sl.scale[i] * acc[i];
    // value nv carries the norm
    cx<double> out[MAXJ + 1];
#pragma unroll
    for (int i = 0; i <= MAXJ; ++i) out[i] = (i < nv) ? acc[i] : (i == nv ? acc[MAXJ] : mk(0.0, 0.0));
    block_sum_vec<MAXJ + 1>(out, nv + 1, sm, a.part + (long long)q.slot * a.pstride * a.bstride, a.bstride, q.b);
}

// y = 0 (gated).
__global__ void __launch_bounds__(NT) k_vzero(const VecArgs a) {
    VecPos q = vec_pos(a.st);
    const VecSlot& sl = a.st.s[q.slot];
    if (gated_off(sl.gate)) return;
    const long long N = static_cast<const LevelView<double>*>(sl.lv)->N;
    chunk_range(N, q.nb, q.b, q.lo, q.hi);
    for (int p = q.lo + (int)threadIdx.x; p < q.hi; p += NT) sl.y[p] = mk(0.0, 0.0);
}

// t = sum_i coef_i V_i (ACC: t += ...).
template <int MAXJ, bool ACC>
__global__ void __launch_bounds__(NT) k_combine(const VecArgs a) {
    VecPos q = vec_pos(a.st);
    const VecSlot& sl = a.st.s[q.slot];
    if (gated_off(sl.gate)) return;
    const long long N = static_cast<const LevelView<double>*>(sl.lv)->N;
    const int nv = (sl.jp ? *sl.jp : sl.j) + 1;
    const cx<double>* V = sl.V;
    cx<double> coef[MAXJ];
#pragma unroll
    for (int i = 0; i < MAXJ; ++i) coef[i] = (i < nv) ? sl.coef[i] : mk(0.0, 0.0);
    cx<double>* t = sl.y;
    chunk_range(N, q.nb, q.b, q.lo, q.hi);
    for (int p = q.lo + (int)threadIdx.x; p < q.hi; p += NT) {
        cx<double> s = mk(0.0, 0.0);
#pragma unroll
        for (int i = 0; i < MAXJ; ++i)
            if (i < nv) s = s + coef[i] * V[(long long)i * N + p];
        if constexpr (ACC)
            t[p] = t[p] + s;
        else
            t[p] = s;
    }
}

// ---------------------------------------------------------------------------
// Second reduction stage, fixed order.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(NT) k_reduce_complex(const ReduceArgs a) {
    __shared__ double sr[NT / 64], si[NT / 64];
    const int v = blockIdx.x, slot = blockIdx.y;
    const cx<double>* p = a.part + ((long long)slot * a.pstride + v) * a.bstride;
    const int cnt = a.cnt[slot];
    double r = 0.0, im = 0.0;
    for (int b = threadIdx.x; b < cnt; b += NT) {
        r += p[b].r;
        im += p[b].i;
    }
    r = block_sum(r, sr);
    im = block_sum(im, si);
    if (threadIdx.x == 0) a.out[(long long)slot * a.ostride + v] = mk(r, im);
}

__global__ void __launch_bounds__(NT) k_reduce_real(const ReduceArgs a) {
    __shared__ double sr[NT / 64];
    const int slot = blockIdx.y;
    const double* p = a.rpart + (long long)slot * a.bstride;
    const int cnt = a.cnt[slot];
    double r = 0.0;
    for (int b = threadIdx.x; b < cnt; b += NT) r += p[b];
    r = block_sum(r, sr);
    if (threadIdx.x == 0) a.rout[slot] = r;
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
// tile shapes (x, y, z) of the fused kernels; LDS per workgroup stays under
// 64 KB for the complex-double iterate variant
constexpr int SHAPES_2D[NUM_TILE_SHAPES][2] = {{64, 16}, {64, 8}, {128, 8}};
constexpr int SHAPES_3D[NUM_TILE_SHAPES][3] = {{16, 8, 4}, {32, 4, 2}, {16, 4, 4}};

inline int cdivi(int a, int b) { return (a + b - 1) / b; }
}  // namespace

void tile_shape(int dim, int shape, int t[3]) {
    if (shape < 0 || shape >= NUM_TILE_SHAPES) shape = 0;
    if (dim == 2) {
        t[0] = SHAPES_2D[shape][0];
        t[1] = SHAPES_2D[shape][1];
        t[2] = 1;
    } else {
        t[0] = SHAPES_3D[shape][0];
        t[1] = SHAPES_3D[shape][1];
        t[2] = SHAPES_3D[shape][2];
    }
}

void tile_counts(int dim, int shape, const int n[3], int ntiles[3]) {
    int t[3];
    tile_shape(dim, shape, t);
    ntiles[0] = cdivi(n[0], t[0]);
    ntiles[1] = cdivi(n[1], t[1]);
    ntiles[2] = dim == 3 ? cdivi(n[2], t[2]) : 1;
}

template <typename T, typename TF, bool ZERO>
static hipError_t sr_launch(int dim, int shape, const CycleArgs& a, hipStream_t s) {
    dim3 grid(a.st.ntiles);
#define SR(D, X, Y, Z) hipLaunchKernelGGL((k_smooth_restrict<D, T, TF, ZERO, X, Y, Z>), grid, dim3(NT), 0, s, a);
    MG_SHAPE_SWITCH(SR)
#undef SR
    return hipGetLastError();
}

template <typename T, typename TF, typename TO, bool ZERO, bool ACC>
static hipError_t ps_launch(int dim, int shape, const CycleArgs& a, hipStream_t s) {
    dim3 grid(a.st.ntiles);
#define PS(D, X, Y, Z) \
    hipLaunchKernelGGL((k_prolong_smooth<D, T, TF, TO, ZERO, ACC, X, Y, Z>), grid, dim3(NT), 0, s, a);
    MG_SHAPE_SWITCH(PS)
#undef PS
    return hipGetLastError();
}

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

int mv_blocks(int dim, const int n[3], int per) {
    if (dim != 2) return vec_blocks((long long)n[0] * n[1] * n[2], per);
    const int ncb = (n[0] + NT - 1) / NT;
    return ncb * ((n[1] + per - 1) / per);
}

int vec_blocks(long long N, int per) {
    long long b = (N + (long long)NT * per - 1) / ((long long)NT * per);
    if (b > 1024) b = 1024;
    if (b < 1) b = 1;
    return (int)b;
}

hipError_t launch_residual(int dim, const VecArgs& a, hipStream_t s) {
    if (a.st.n <= 0) return hipSuccess;
    if (dim == 2)
        hipLaunchKernelGGL((k_residual<2>), dim3(a.st.nblocks), dim3(NT), 0, s, a);
    else
        hipLaunchKernelGGL((k_residual<3>), dim3(a.st.nblocks), dim3(NT), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_norm(const VecArgs& a, hipStream_t s) {
    if (a.st.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_norm, dim3(a.st.nblocks), dim3(NT), 0, s, a);
    return hipGetLastError();
}

static int jbucket(int jmax) {
    return jmax <= 4 ? 4 : jmax <= 8 ? 8 : jmax <= 16 ? 16 : jmax <= 24 ? 24 : 32;
}

// MAXJ buckets of the GMRES pass kernels (registers scale with MAXJ)
#define MG_JSWITCH(CASE)         \
    switch (jbucket(jmax)) {     \
        case 4: CASE(4) break;   \
        case 8: CASE(8) break;   \
        case 16: CASE(16) break; \
        case 24: CASE(24) break; \
        default: CASE(32) break; \
    }

hipError_t launch_matvec_dot(int dim, int jmax, const VecArgs& a, hipStream_t s) {
    if (a.st.n <= 0) return hipSuccess;
    dim3 grid(a.st.nblocks);
#define MV(J)                                                                  \
    if (dim == 2)                                                              \
        hipLaunchKernelGGL((k_matvec_dot<2, J>), grid, dim3(NT), 0, s, a);     \
    else                                                                       \
        hipLaunchKernelGGL((k_matvec_dot<3, J>), grid, dim3(NT), 0, s, a);
    MG_JSWITCH(MV)
#undef MV
    return hipGetLastError();
}

hipError_t launch_update_gram(int jmax, const VecArgs& a, hipStream_t s) {
    if (a.st.n <= 0) return hipSuccess;
    dim3 grid(a.st.nblocks);
#define UG(J) hipLaunchKernelGGL((k_update_gram<J>), grid, dim3(NT), 0, s, a);
    MG_JSWITCH(UG)
#undef UG
    return hipGetLastError();
}

hipError_t launch_vzero(const VecArgs& a, hipStream_t s) {
    if (a.st.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_vzero, dim3(a.st.nblocks), dim3(NT), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_combine(int jmax, bool accumulate, const VecArgs& a, hipStream_t s) {
    if (a.st.n <= 0) return hipSuccess;
    dim3 grid(a.st.nblocks);
#define CB(J)                                                                \
    if (accumulate)                                                          \
        hipLaunchKernelGGL((k_combine<J, true>), grid, dim3(NT), 0, s, a);   \
    else                                                                     \
        hipLaunchKernelGGL((k_combine<J, false>), grid, dim3(NT), 0, s, a);
    MG_JSWITCH(CB)
#undef CB
    return hipGetLastError();
}

hipError_t launch_reduce(const ReduceArgs& a, int nslots, bool real, hipStream_t s) {
    if (nslots <= 0) return hipSuccess;
    if (real)
        hipLaunchKernelGGL(k_reduce_real, dim3(1, nslots), dim3(NT), 0, s, a);
    else
        hipLaunchKernelGGL(k_reduce_complex, dim3(a.nvals, nslots), dim3(NT), 0, s, a);
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
