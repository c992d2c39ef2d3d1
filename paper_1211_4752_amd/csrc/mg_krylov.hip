// Krylov control on the device (gfx950): the small dense work of restarted,
// right-preconditioned (F)GMRES(m) -- one V-cycle per outer step (Sec. 4.1;
// flexible when the cycle changes from step to step, Sec. 3.2.2) -- and the
// stop tests of the standalone iteration (Sec. 4.1, LVL-MG).  With them a
// whole restart cycle of every right-hand side of a batch is a fixed
// sequence of launches, captured once as a HIP graph; the host reads a few
// flags per restart cycle instead of synchronising every step.
//
// Arnoldi step j (all right-hand sides of a launch are at the same j):
//   k_matvec_dot   w = A z_j,           partials of h1 = V^H w
//   gm_h           h = h1 + (h1 - G h1), G the Gram matrix of the stored
//                  (normalised) basis: the second classical Gram-Schmidt
//                  projection V^H (w - V h1) written through G, so the
//                  basis is read twice per step instead of three times
//   k_update_gram  V_{j+1} = w - V h,   partials of V^H V_{j+1} and ||V_{j+1}||^2
//   gm_col         H(:, j) = (h, ||V_{j+1}||), the next column of G, complex
//                  Givens rotation, residual estimate |g_{j+1}| / ||f||, stop
//                  tests; at the end of a restart cycle y = R^{-1} g
// Every sum over partials runs in a fixed order (deterministic results).

#include "mg_kcommon.hpp"

namespace mg {

using namespace kc;

namespace {

__device__ __forceinline__ double cabs_(cx<double> z) { return hypot(z.r, z.i); }
__device__ __forceinline__ cx<double> conj_(cx<double> z) { return mk(z.r, -z.i); }
__device__ __forceinline__ cx<double> cdivd(cx<double> a, cx<double> b) { return cdiv(a, b); }

// out[v] = sum_b part[(slot * pstride + v) * bstride + b], v < nv, in a fixed
// order: wave w of the NTH threads takes the values v = w, w + NTH / 64,
// ...; lane l adds b = l, l + 64, ... in turn, then a fixed butterfly.  Ends
// with a barrier.
template <int NTH>
__device__ void wg_sum_cx(const cx<double>* part, int slot, int pstride, int bstride, int nv, int cnt,
                          cx<double>* out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int v = wave; v < nv; v += NTH / 64) {
        const cx<double>* p = part + ((long long)slot * pstride + v) * bstride;
        double r = 0.0, i = 0.0;
        int b = lane;
        // four loads in flight, added in the same order as one at a time
        for (; b + 192 < cnt; b += 256) {
            const cx<double> x0 = p[b], x1 = p[b + 64], x2 = p[b + 128], x3 = p[b + 192];
            r += x0.r;
            i += x0.i;
            r += x1.r;
            i += x1.i;
            r += x2.r;
            i += x2.i;
            r += x3.r;
            i += x3.i;
        }
        for (; b < cnt; b += 64) {
            r += p[b].r;
            i += p[b].i;
        }
        r = wave_sum(r);
        i = wave_sum(i);
        if (lane == 0) out[v] = mk(r, i);
    }
    __syncthreads();
}

__device__ double wg_sum_real(const double* p, int cnt, double* sm) {
    double s = 0.0;
    for (int b = threadIdx.x; b < cnt; b += NT) s += p[b];
    s = block_sum(s, sm);
    __syncthreads();
    if (threadIdx.x == 0) sm[0] = s;
    __syncthreads();
    return sm[0];
}

__device__ __forceinline__ void push_hist(GmFlags* fl, double* hist, int maxit, double v) {
    if (fl->hlen <= maxit) hist[fl->hlen] = v;
    fl->hlen++;
}

// <v_i, v_k> from the stored upper triangle G[k][i] (i <= k).
__device__ __forceinline__ cx<double> gram(const GmState* st, int i, int k) {
    return i <= k ? st->G[k][i] : conj_(st->G[i][k]);
}

__global__ void __launch_bounds__(NT) k_gm_init(const GmArgs a, int standalone) {
    __shared__ double sm[NT / 64];
    const GmItem it = a.it[blockIdx.x];
    const GmParams P = *a.prm;
    double* hist = P.hist + (long long)blockIdx.x * P.hstride;
    const double nf2 = wg_sum_real(a.rpart + (long long)it.slot * a.bstride, it.cnt, sm);
    for (int i = threadIdx.x; i < P.hstride; i += NT) hist[i] = -1.0;
    __syncthreads();
    if (threadIdx.x != 0) return;
    GmFlags* fl = it.fl;
    const double nf = sqrt(nf2);
    it.st->nf = nf;
    fl->its = 0;
    fl->j = 0;
    fl->kk = 0;
    fl->live = 0;
    fl->fin = 0;
    fl->zero = 0;
    fl->hlen = 0;
    if (nf == 0.0) {   // f = 0: the solution is 0
        fl->zero = 1;
        fl->state = 1;
        hist[0] = 0.0;
        fl->hlen = 1;
    } else if (standalone) {
        fl->state = P.maxit > 0 ? 0 : 2;
        fl->live = P.maxit > 0 ? 1 : 0;
    } else {
        fl->state = 0;
        fl->fin = 1;   // run the restart residual
    }
}

// Start of a restart cycle from the residual r = f - A x stored in V_0.
__global__ void __launch_bounds__(NT) k_gm_restart(const GmArgs a) {
    __shared__ double sm[NT / 64];
    const GmItem it = a.it[blockIdx.x];
    if (gated_off(&it.fl->fin)) return;
    const GmParams P = *a.prm;
    double* hist = P.hist + (long long)blockIdx.x * P.hstride;
    const double beta2 = wg_sum_real(a.rpart + (long long)it.slot * a.bstride, it.cnt, sm);
    if (threadIdx.x != 0) return;
    GmFlags* fl = it.fl;
    GmState* st = it.st;
    const double beta = sqrt(beta2);
    const double ratio = beta / st->nf;
    if (fl->hlen == 0) push_hist(fl, hist, P.maxit, ratio);
    fl->fin = 0;
    fl->live = 0;
    if (ratio <= P.rtol) {
        fl->state = 1;
    } else if (!isfinite(ratio)) {
        fl->state = 3;
    } else if (fl->its >= P.maxit) {
        fl->state = 2;
    } else {
        fl->state = 0;
        fl->j = 0;
        for (int i = 0; i <= P.m; ++i) st->g[i] = mk(0.0, 0.0);
        st->g[0] = mk(beta, 0.0);
        const double s0 = 1.0 / beta;
        it.scale[0] = s0;
        st->G[0][0] = mk(beta2 * s0 * s0, 0.0);
        fl->live = 1;
    }
}

// The per-step reductions take NTG threads: one or two values per wave.
constexpr int NTG = 1024;

// h = 2 h1 - G h1 for step j.
__global__ void __launch_bounds__(NTG) k_gm_h(const GmArgs a) {
    __shared__ cx<double> h1[HSTRIDE];
    const GmItem it = a.it[blockIdx.x];
    if (gated_off(&it.fl->live)) return;
    const int nv = a.j + 1;
    wg_sum_cx<NTG>(a.part, it.slot, a.pstride, a.bstride, nv, it.cnt, h1);
    const int i = threadIdx.x;
    if (i < nv) {
        const GmState* st = it.st;
        cx<double> s = mk(0.0, 0.0);
        for (int k = 0; k < nv; ++k) s = s + gram(st, i, k) * h1[k];
        it.st->h[i] = mk(2.0 * h1[i].r - s.r, 2.0 * h1[i].i - s.i);
    }
}

// Hessenberg column, Givens rotation, estimate and stop tests of step j.
__global__ void __launch_bounds__(NTG) k_gm_col(const GmArgs a) {
    __shared__ cx<double> vals[HSTRIDE + 1];
    const GmItem it = a.it[blockIdx.x];
    if (gated_off(&it.fl->live)) return;
    const int j = a.j, nv = j + 1;
    wg_sum_cx<NTG>(a.part, it.slot, a.pstride, a.bstride, nv + 1, it.cnt, vals);
    if (threadIdx.x != 0) return;
    const GmParams P = *a.prm;
    double* hist = P.hist + (long long)blockIdx.x * P.hstride;
    GmFlags* fl = it.fl;
    GmState* st = it.st;
    const double r = vals[nv].r > 0.0 ? vals[nv].r : 0.0;
    const double hn = sqrt(r);
    cx<double>* col = st->H[j];
    for (int i = 0; i <= j; ++i) col[i] = st->h[i];
    col[j + 1] = mk(hn, 0.0);
    for (int i = 0; i < j; ++i) {
        const cx<double> x = col[i], y = col[i + 1];
        const cx<double> sn = st->sn[i];
        const double c = st->cs[i];
        col[i] = c * x + sn * y;
        col[i + 1] = c * y - conj_(sn) * x;
    }
    // rotation j zeroing col[j + 1] below col[j]
    const cx<double> x = col[j], y = col[j + 1];
    double cj;
    cx<double> sj;
    if (y.r == 0.0 && y.i == 0.0) {
        cj = 1.0;
        sj = mk(0.0, 0.0);
    } else if (x.r == 0.0 && x.i == 0.0) {
        cj = 0.0;
        sj = (1.0 / cabs_(y)) * conj_(y);
    } else {
        const double ax = cabs_(x), t = hypot(ax, cabs_(y));
        cj = ax / t;
        sj = (1.0 / t) * (((1.0 / ax) * x) * conj_(y));
    }
    st->cs[j] = cj;
    st->sn[j] = sj;
    col[j] = cj * x + sj * y;
    col[j + 1] = mk(0.0, 0.0);
    const cx<double> gj = st->g[j];
    st->g[j + 1] = mk(0.0, 0.0) - conj_(sj) * gj;
    st->g[j] = cj * gj;
    fl->its++;
    const double est = cabs_(st->g[j + 1]) / st->nf;
    push_hist(fl, hist, P.maxit, est);
    if (!isfinite(est)) {
        fl->state = 3;
        fl->live = 0;
        return;
    }
    if (hn != 0.0) {
        const double s1 = 1.0 / hn;
        it.scale[j + 1] = s1;
        for (int i = 0; i <= j; ++i) st->G[j + 1][i] = s1 * vals[i];
        st->G[j + 1][j + 1] = mk(r * s1 * s1, 0.0);
    }
    if (est <= P.rtol || fl->its >= P.maxit || j + 1 == P.m || hn == 0.0) {
        // y = R^{-1} g on the first j + 1 rotated columns
        const int kk = j + 1;
        cx<double> y[MAX_RESTART];
        for (int i = kk - 1; i >= 0; --i) {
            cx<double> s = st->g[i];
            for (int l = i + 1; l < kk; ++l) s = s - st->H[l][i] * y[l];
            y[i] = cdivd(s, st->H[i][i]);
        }
        for (int i = 0; i < kk; ++i) it.coef[i] = P.flexible ? y[i] : it.scale[i] * y[i];
        fl->kk = kk - 1;
        fl->fin = 1;
        fl->live = 0;
    } else {
        fl->j = j + 1;
    }
}

// Standalone: ratio of the iterate that entered this cycle.
__global__ void __launch_bounds__(NT) k_sa_step(const GmArgs a) {
    __shared__ double sm[NT / 64];
    const GmItem it = a.it[blockIdx.x];
    if (gated_off(&it.fl->live)) return;
    const double rho = wg_sum_real(a.rpart + (long long)it.slot * a.bstride, it.cnt, sm);
    if (threadIdx.x != 0) return;
    const GmParams P = *a.prm;
    double* hist = P.hist + (long long)blockIdx.x * P.hstride;
    GmFlags* fl = it.fl;
    const double ratio = sqrt(rho) / it.st->nf;
    const int cyc = fl->j;
    hist[cyc] = ratio;
    fl->its = cyc;
    if (ratio <= P.rtol) {
        fl->state = 1;
        fl->live = 0;
    } else if (!isfinite(ratio) || ratio > 1e8) {
        fl->state = 3;
        fl->live = 0;
    } else {
        fl->its = cyc + 1;
        fl->j = cyc + 1;
        if (cyc + 1 >= P.maxit) {
            fl->state = 2;
            fl->live = 0;
        }
    }
}

}  // namespace

hipError_t launch_gm(int which, int nitems, const GmArgs& a, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    const dim3 grid(nitems), blk(NT);
    switch (which) {
        case GM_INIT: hipLaunchKernelGGL(k_gm_init, grid, blk, 0, s, a, 0); break;
        case SA_INIT: hipLaunchKernelGGL(k_gm_init, grid, blk, 0, s, a, 1); break;
        case GM_RESTART: hipLaunchKernelGGL(k_gm_restart, grid, blk, 0, s, a); break;
        case GM_H: hipLaunchKernelGGL(k_gm_h, grid, dim3(NTG), 0, s, a); break;
        case GM_COL: hipLaunchKernelGGL(k_gm_col, grid, dim3(NTG), 0, s, a); break;
        case SA_STEP: hipLaunchKernelGGL(k_sa_step, grid, blk, 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mg
