// gfx950 vector kernels of the level-dependent complex-shifted multigrid:
// level-0 residual and norms, the GMRES Arnoldi passes and the set-up
// helpers (the fused omega-Jacobi cycle kernels are in mg_jacobi.hip).
//
// Hot kernels (bandwidth-bound, no dense contraction anywhere, so no MFMA):
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
// Vector kernels: one point per thread, a contiguous chunk of the slot's
// vector per workgroup.
// ---------------------------------------------------------------------------
// (loads unconditional, missing neighbours masked to exact zeros, as in
// stencil_at)
template <int D, typename PX>
__device__ __forceinline__ cx<double> apply_at(const GLevel<double>& L, const PX& x, int p, int gx, int gy,
                                               int gz) {
    return stencil_at<D, double, double>(L, x, 1.0, p, gx, gy, gz);
}

// y = f - A x (f null: y = A x); ||y||^2 partials in rpart.
template <int D>
__global__ void __launch_bounds__(NT) k_residual(const VecArgs a) {
    __shared__ double sred[NT / 64];
    VecPos q = vec_pos(a.st);
    const VecSlot sl = a.st.s[q.slot];
    if (gated_off(sl.gate)) return;
    const GLevel<double> L = glevel(*static_cast<const LevelView<double>*>(sl.lv));
    chunk_range(L.N, q.nb, q.b, q.lo, q.hi);
    double nrm = 0.0;
    const int nx = L.n[0], ny = L.n[1];
    const auto x = gin(sl.x);
    const auto fr = gin(sl.f);
    const auto y = gout(sl.y);
    for (int p = q.lo + (int)threadIdx.x; p < q.hi; p += NT) {
        const int gx = p % nx;
        const int rr = p / nx;
        const int gy = rr % ny;
        const int gz = rr / ny;
        cx<double> v = apply_at<D>(L, x, p, gx, gy, gz);
        if (sl.f) v = fr[p] - v;
        y[p] = v;
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
    const VecSlot sl = a.st.s[q.slot];
    if (gated_off(sl.gate)) return;
    const long long N = static_cast<const LevelView<double>*>(sl.lv)->N;
    chunk_range(N, q.nb, q.b, q.lo, q.hi);
    double nrm = 0.0;
    const auto x = gin(sl.x);
    for (int p = q.lo + (int)threadIdx.x; p < q.hi; p += NT) nrm += abs2(x[p]);
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
    __syncthreads();   // sm may be written again
}

// ---------------------------------------------------------------------------
// Live-chunk schedule of the Arnoldi passes (see ARN_SPLIT).
// ---------------------------------------------------------------------------
struct ChunkItem {
    int slot, c;   // chunk c of slot
};

// Inclusive prefix sum of v over the workgroup; tot = the workgroup's sum.
__device__ __forceinline__ int block_scan(int v, int* sh, int& tot) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) sh[wave] = x;
    __syncthreads();
    int off = 0;
    tot = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
        const int t = sh[w];
        if (w < wave) off += t;
        tot += t;
    }
    __syncthreads();
    return x + off;
}

__device__ __forceinline__ int live_chunks_of(const VecSlots& st, int s) {
    return (s < st.n && !gated_off(st.s[s].gate)) ? st.s[s].nc : 0;
}

// This workgroup's share of the live chunks, at most ARN_SPLIT items in
// item[] (every thread gets the same count).  The live chunks, slot by
// slot, are numbered 0 .. L - 1 and workgroup g takes [g L / G, (g + 1) L /
// G); as G >= L / ARN_SPLIT that is at most ARN_SPLIT chunks.
__device__ int live_items(const VecSlots& st, ChunkItem* item, int* sh, int* nitem) {
    int L = 0;
    for (int g = 0; g < st.n; g += NT) {
        int tot;
        block_scan(live_chunks_of(st, g + (int)threadIdx.x), sh, tot);
        L += tot;
    }
    if (L == 0) return 0;
    const long long pid = xcd_remap(blockIdx.x, gridDim.x);
    const long long k0 = (long long)L * pid / gridDim.x, k1 = (long long)L * (pid + 1) / gridDim.x;
    if (threadIdx.x == 0) *nitem = 0;
    __syncthreads();
    long long carry = 0;
    for (int g = 0; g < st.n; g += NT) {
        const int s = g + (int)threadIdx.x;
        const int c = live_chunks_of(st, s);
        int tot;
        const int inc = block_scan(c, sh, tot);
        const long long lo = carry + inc - c, hi = carry + inc;
        const long long a = lo > k0 ? lo : k0, b = hi < k1 ? hi : k1;
        if (a < b) {
            const int m = (int)(b - a);
            const int r = atomicAdd(nitem, m);
            for (int q = 0; q < m; ++q)
                if (r + q < ARN_SPLIT) item[r + q] = ChunkItem{s, (int)(a - lo) + q};
        }
        carry += tot;
    }
    __syncthreads();
    const int n = __builtin_amdgcn_readfirstlane(*nitem);
    return n < ARN_SPLIT ? n : ARN_SPLIT;
}

// item k, read back as wave-uniform values (so the slot's fields are loaded
// into scalar registers)
__device__ __forceinline__ ChunkItem item_at(const ChunkItem* item, int k) {
    const ChunkItem x = item[k];
    return ChunkItem{__builtin_amdgcn_readfirstlane(x.slot), __builtin_amdgcn_readfirstlane(x.c)};
}

__device__ __forceinline__ int clampi3(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// w = A z, h_i = <v_i, w>: one partial per chunk.
template <int D, int MAXJ>
__global__ void __launch_bounds__(NT) k_matvec_dot(const VecArgs a) {
    static_assert(D == 2 || PZX * PZY == NT, "one point of a 3D column per thread");
    __shared__ cx<double> sm[(NT / 64) * MAXJ];
    __shared__ cx<double> P[D == 3 ? 2 * PZW * PZH : 1];   // 3D: a plane and its ring, two buffers
    __shared__ double ssc[MAXJ];   // scale_i, read at the end from LDS
    __shared__ ChunkItem item[ARN_SPLIT];
    __shared__ int sh[NT / 64], nitem;
    const int ni = live_items(a.st, item, sh, &nitem);
    for (int k = 0; k < ni; ++k) {
        const ChunkItem cr = item_at(item, k);
        const int c = cr.c;
        const VecSlot sl = a.st.s[cr.slot];
        const GLevel<double> L = glevel(*static_cast<const LevelView<double>*>(sl.lv));
        const long long N = L.N;
        const int nv = sl.j + 1;
        if (k == 0 || cr.slot != item_at(item, k - 1).slot) {   // stage the slot's scales
            __syncthreads();   // the previous chunk's readers of ssc are done
            if ((int)threadIdx.x < MAXJ) ssc[threadIdx.x] = (int)threadIdx.x < nv ? sl.scale[threadIdx.x] : 0.0;
            __syncthreads();
        }
        const auto z = gin(sl.x);
        const auto w = gout(sl.y);
        const auto V = gstream(sl.V);
        cx<double>* dst = a.part + (long long)cr.slot * a.pstride * a.bstride;
        const int nx = L.n[0], ny = L.n[1];
        cx<double> acc[MAXJ];
#pragma unroll
        for (int i = 0; i < MAXJ; ++i) acc[i] = mk(0.0, 0.0);
        if constexpr (D == 2) {
            // Column marching: chunk c owns NT consecutive columns of a
            // strip of rows (c = column block * nrs + strip); each thread
            // walks down its column keeping the rows above, at and below
            // in registers, so every z value is fetched once.
            const int ncb = (nx + NT - 1) / NT;
            const int nrs = sl.nc / ncb;
            const int rows = (ny + nrs - 1) / nrs;
            const int gx = (c / nrs) * NT + (int)threadIdx.x;
            const int y0 = (c % nrs) * rows;
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
        } else {
            // 3D: chunk c is a column of PZX x PZY points through up to PZC
            // planes; plane zz with its one-point ring goes through LDS, the
            // planes zz +- 1 of each point stay in registers, and the next
            // plane's inputs are requested first (the terms of apply_at, in
            // its order)
            int ntx, nty, ntz;
            pz_counts(L.n, ntx, nty, ntz);
            const int nz = L.n[2];
            const long long nxy = (long long)nx * ny;
            const int tx = c % ntx, ty = (c / ntx) % nty, tz = c / (ntx * nty);
            const int x0 = tx * PZX, y0 = ty * PZY, z0 = tz * PZC;
            const int z1 = z0 + PZC < nz ? z0 + PZC : nz;
            const int t = (int)threadIdx.x;
            const int lx = t % PZX, ly = t / PZX;
            const int gx = x0 + lx, gy = y0 + ly;
            const bool own = gx < nx && gy < ny;
            const int cgx = gx < nx ? gx : nx - 1, cgy = gy < ny ? gy : ny - 1;
            const long long pxy = (long long)cgy * nx + cgx;
            const bool ring = t < PZR;
            int rlx = 0, rly = 0;
            pz_ring(ring ? t : 0, rlx, rly);
            const int rgx = clampi3(x0 + rlx - 1, 0, nx - 1), rgy = clampi3(y0 + rly - 1, 0, ny - 1);
            const long long rxy = (long long)rgy * nx + rgx;
            auto plane = [&](int q) { return (long long)clampi3(q, 0, nz - 1) * nxy; };
            const cx<double> cmx = L.cm[0][cgx], cpx = L.cp[0][cgx], c0x = L.c0[0][cgx];
            const cx<double> cmy = L.cm[1][cgy], cpy = L.cp[1][cgy], c0y = L.c0[1][cgy];
            const bool bxm = gx > 0, bxp = gx < nx - 1, bym = gy > 0, byp = gy < ny - 1;
            const int ci = (ly + 1) * PZW + lx + 1;
            cx<double> xm = z[plane(z0 - 1) + pxy], xc = z[plane(z0) + pxy], xp = z[plane(z0 + 1) + pxy];
            cx<double> rc = z[plane(z0) + rxy];
            double k2c = L.k2[plane(z0) + pxy];
            for (int zz = z0; zz < z1; ++zz) {
                const long long p = (long long)zz * nxy + pxy;
                // the basis loads do not depend on the stencil: issue them first
                cx<double> vv[MAXJ];
#pragma unroll
                for (int i = 0; i < MAXJ; ++i) vv[i] = (i < nv) ? V[(long long)i * N + p] : mk(0.0, 0.0);
                const cx<double> xn = z[plane(zz + 2) + pxy];
                const cx<double> rn = z[plane(zz + 1) + rxy];
                const double k2n = L.k2[plane(zz + 1) + pxy];
                const cx<double> cmz = L.cm[2][zz], cpz = L.cp[2][zz], c0z = L.c0[2][zz];
                cx<double>* Pb = P + (zz & 1) * (PZW * PZH);
                Pb[ci] = xc;
                if (ring) Pb[rly * PZW + rlx] = rc;
                __syncthreads();
                const bool bzm = zz > 0, bzp = zz < nz - 1;
                cx<double> d = c0x + c0y;
                d = d + c0z;
                d = d - k2c * L.sigma;
                cx<double> ax = d * xc;
                ax = ax + masked(bxm, cmx) * Pb[ci - 1];
                ax = ax + masked(bxp, cpx) * Pb[ci + 1];
                ax = ax + masked(bym, cmy) * Pb[ci - PZW];
                ax = ax + masked(byp, cpy) * Pb[ci + PZW];
                ax = ax + masked(bzm, cmz) * xm;
                ax = ax + masked(bzp, cpz) * xp;
                const cx<double> wv = 1.0 * ax;
                if (own) {
                    w[p] = wv;
#pragma unroll
                    for (int i = 0; i < MAXJ; ++i) acc[i] = acc[i] + cmulc(vv[i], wv);
                }
                xm = xc;
                xc = xp;
                xp = xn;
                rc = rn;
                k2c = k2n;
            }
        }
#pragma unroll
        for (int i = 0; i < MAXJ; ++i)
            if (i < nv) acc[i] = ssc[i] * acc[i];
        block_sum_vec<MAXJ>(acc, nv, sm, dst, a.bstride, c);
    }
}

// Second pass of the Arnoldi step (classical Gram-Schmidt applied twice
// with one reduction per pass): V_{j+1} = w - sum_i h_i v_i, where h already
// contains the second projection (formed on the device from the Gram
// matrix of the stored basis), fused with the partials of <v_i, V_{j+1}>
// (i <= j; the next column of that Gram matrix) and of ||V_{j+1}||^2 (value
// j + 1), one partial per chunk.  The coefficients scale_i h_i are staged
// in LDS.
template <int MAXJ>
__global__ void __launch_bounds__(NT) k_update_gram(const VecArgs a) {
    __shared__ cx<double> sm[(NT / 64) * (MAXJ + 1)];
    __shared__ cx<double> sc[MAXJ];
    __shared__ double ssc[MAXJ];   // scale_i, read at the end from LDS
    __shared__ ChunkItem item[ARN_SPLIT];
    __shared__ int sh[NT / 64], nitem;
    const int ni = live_items(a.st, item, sh, &nitem);
    for (int k = 0; k < ni; ++k) {
        const ChunkItem cr = item_at(item, k);
        const int c = cr.c;
        const VecSlot sl = a.st.s[cr.slot];
        const long long N = static_cast<const LevelView<double>*>(sl.lv)->N;
        const int nv = sl.j + 1;
        const auto w = gin(sl.y);
        const auto V = gstream(sl.V);
        if (k == 0 || cr.slot != item_at(item, k - 1).slot) {   // stage the slot's coefficients
            __syncthreads();   // the previous chunk's readers of sc, ssc are done
            if ((int)threadIdx.x < MAXJ) {
                const double sv = (int)threadIdx.x < nv ? sl.scale[threadIdx.x] : 0.0;
                ssc[threadIdx.x] = sv;
                sc[threadIdx.x] = (int)threadIdx.x < nv ? sv * sl.hin[threadIdx.x] : mk(0.0, 0.0);
            }
            __syncthreads();
        }
        const auto vout = gout(sl.V + (long long)nv * N);
        cx<double>* dst = a.part + (long long)cr.slot * a.pstride * a.bstride;
        int lo, hi;
        chunk_range(N, sl.nc, c, lo, hi);
        cx<double> acc[MAXJ + 1];
#pragma unroll
        for (int i = 0; i <= MAXJ; ++i) acc[i] = mk(0.0, 0.0);
        for (int p = lo + (int)threadIdx.x; p < hi; p += NT) {
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
            if (i < nv) acc[i] = ssc[i] * acc[i];
        // value nv carries the norm
        cx<double> out[MAXJ + 1];
#pragma unroll
        for (int i = 0; i <= MAXJ; ++i) out[i] = (i < nv) ? acc[i] : (i == nv ? acc[MAXJ] : mk(0.0, 0.0));
        block_sum_vec<MAXJ + 1>(out, nv + 1, sm, dst, a.bstride, c);
    }
}

// y = 0 (gated).
__global__ void __launch_bounds__(NT) k_vzero(const VecArgs a) {
    VecPos q = vec_pos(a.st);
    const VecSlot sl = a.st.s[q.slot];
    if (gated_off(sl.gate)) return;
    const long long N = static_cast<const LevelView<double>*>(sl.lv)->N;
    chunk_range(N, q.nb, q.b, q.lo, q.hi);
    const auto y = gout(sl.y);
    for (int p = q.lo + (int)threadIdx.x; p < q.hi; p += NT) y[p] = mk(0.0, 0.0);
}

// t = sum_i coef_i V_i (ACC: t += ...).
template <int MAXJ, bool ACC>
__global__ void __launch_bounds__(NT) k_combine(const VecArgs a) {
    VecPos q = vec_pos(a.st);
    const VecSlot sl = a.st.s[q.slot];
    if (gated_off(sl.gate)) return;
    const long long N = static_cast<const LevelView<double>*>(sl.lv)->N;
    const int nv = (sl.jp ? *sl.jp : sl.j) + 1;
    const auto V = gstream(sl.V);
    cx<double> coef[MAXJ];
#pragma unroll
    for (int i = 0; i < MAXJ; ++i) coef[i] = (i < nv) ? sl.coef[i] : mk(0.0, 0.0);
    const auto t = gout(sl.y);
    chunk_range(N, q.nb, q.b, q.lo, q.hi);
    for (int p = q.lo + (int)threadIdx.x; p < q.hi; p += NT) {
        // every vector's load issued before the first use (past nv a load
        // re-reads the last vector, whose coefficient is 0): a load under a
        // branch would be waited for one at a time
        cx<double> vv[MAXJ];
#pragma unroll
        for (int k = 0; k < MAXJ; ++k) vv[k] = V[(long long)(k < nv ? k : nv - 1) * N + p];
        cx<double> s = mk(0.0, 0.0);
#pragma unroll
        for (int k = 0; k < MAXJ; ++k) s = s + coef[k] * vv[k];
        if constexpr (ACC)
            t[p] = t[p].get() + s;
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

int arnoldi_chunks(bool mv, int dim, const int n[3], long long N, int per) {
    if (mv && dim == 3) return power_z_tiles(n);
    if (per < 1) per = 1;
    if (mv && dim == 2) {
        const int ncb = (n[0] + NT - 1) / NT;
        return ncb * ((n[1] + per - 1) / per);
    }
    long long c = (N + (long long)NT * per - 1) / ((long long)NT * per);
    if (c > 1024LL * ARN_SPLIT) c = 1024LL * ARN_SPLIT;
    if (c < 1) c = 1;
    return (int)c;
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
