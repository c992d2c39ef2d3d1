// Host runtime of the level-dependent multigrid: hierarchy set-up, the
// V-cycle driver, the standalone and GMRES solvers, the adjoint, and the C ABI
// declared in include/mg.h.
//
// Paper: Cools, Reps, Vanroose, "A new level-dependent coarse grid correction
// scheme for indefinite Helmholtz problems" (NLAA 2013).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "mg.h"
#include "mg_device.hpp"

using cd = std::complex<double>;
using mg::cx;
using mg::Slot;
using mg::SlotTable;

namespace {

constexpr int MAX_RESTART = 32;
constexpr int HSTRIDE = MAX_RESTART + 1;     // per-slot stride of dot results
constexpr double DIVERGE = 1e8;

#define CK(expr)                                        \
    do {                                                \
        if ((expr) != hipSuccess) return MG_E_DEVICE;   \
    } while (0)
#define CKS(expr)                                       \
    do {                                                \
        mg_status st_ = (expr);                         \
        if (st_ != MG_OK) return st_;                   \
    } while (0)

inline cx<double> tocx(cd z) { return mg::mk(z.real(), z.imag()); }

// ---------------------------------------------------------------------------
// Discretisation on the host (set-up only)
// ---------------------------------------------------------------------------

// 3-point coefficients of -d^2/dz^2 on the ECS-mapped nodes z_j = Z(j h),
// j = 0..n+1 (Sec. 2.4): Z(x) = x on [a, b], rotated by e^{i phi} outside.
void axis_coefficients(int n, double h, double a, double b, double phi, std::vector<cd>& cm,
                       std::vector<cd>& c0, std::vector<cd>& cp) {
    std::vector<cd> z(n + 2);
    const cd rot = std::polar(1.0, phi);
    for (int j = 0; j < n + 2; ++j) {
        const double x = j * h;
        if (x < a)
            z[j] = a + (x - a) * rot;
        else if (x > b)
            z[j] = b + (x - b) * rot;
        else
            z[j] = x;
    }
    cm.resize(n);
    c0.resize(n);
    cp.resize(n);
    for (int j = 1; j <= n; ++j) {
        const cd hm = z[j] - z[j - 1];
        const cd hp = z[j + 1] - z[j];
        cm[j - 1] = -2.0 / ((hm + hp) * hm);
        cp[j - 1] = -2.0 / ((hm + hp) * hp);
        c0[j - 1] = -(cm[j - 1] + cp[j - 1]);
    }
}

// Dense LU with partial pivoting, row-major, in place; piv[k] = row swapped
// with row k at step k.  Returns false when a pivot is zero.
bool lu_factor(std::vector<cd>& A, std::vector<int>& piv, int n) {
    piv.assign(n, 0);
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = std::abs(A[(size_t)k * n + k]);
        for (int i = k + 1; i < n; ++i) {
            const double v = std::abs(A[(size_t)i * n + k]);
            if (v > best) {
                best = v;
                p = i;
            }
        }
        piv[k] = p;
        if (best == 0.0) return false;
        if (p != k)
            for (int j = 0; j < n; ++j) std::swap(A[(size_t)k * n + j], A[(size_t)p * n + j]);
        const cd inv = 1.0 / A[(size_t)k * n + k];
        for (int i = k + 1; i < n; ++i) {
            const cd l = A[(size_t)i * n + k] * inv;
            A[(size_t)i * n + k] = l;
            if (l != 0.0)
                for (int j = k + 1; j < n; ++j) A[(size_t)i * n + j] -= l * A[(size_t)k * n + j];
        }
    }
    return true;
}

struct Level {
    int n[3] = {1, 1, 1};
    long long N = 0;
    double h[3] = {0, 0, 0};
    cd sigma = 1.0;
    int ntiles[3] = {1, 1, 1};
    // per direction (0 forward, 1 conjugate transpose): per axis cm | c0 | cp
    std::vector<cd> coef_host[2];
    cx<double>* coef_d[2] = {nullptr, nullptr};
    cx<float>* coef_f[2] = {nullptr, nullptr};
    double* k2 = nullptr;
    float* k2f = nullptr;
    void* F = nullptr;    // right-hand sides on levels >= 1, by buf
    void* E = nullptr;    // corrections on levels >= 1, by buf
};

struct Prof {
    bool on = false;
    std::vector<hipEvent_t> pool;
    std::vector<int> cls;
    std::vector<double> bytes;
    size_t used = 0;
};

}  // namespace

struct mg_ctx {
    mg_params p{};
    int dim = 2;
    int L = 0;
    bool mixed = false;
    int nrhs = 1;
    hipStream_t stream = nullptr;
    std::vector<Level> lv;
    // coarsest LU, per direction
    int ncoarse = 0;
    cx<double>* lu[2] = {nullptr, nullptr};
    int* piv[2] = {nullptr, nullptr};
    // level-0 work vectors, by buf
    cx<double>* U1 = nullptr;
    cx<double>* Z = nullptr;
    cx<double>* W = nullptr;
    // GMRES basis, by rhs: V + (rhs * vstride + i) * N0
    cx<double>* V = nullptr;
    int vstride = 0;
    double* scale_d = nullptr;     // [rhs * HSTRIDE + i]
    double* scale_h = nullptr;     // pinned
    cx<double>* coef_d = nullptr;  // [rhs * HSTRIDE + i]
    cx<double>* coef_h = nullptr;  // pinned
    // reductions
    cx<double>* part = nullptr;
    double* rpart = nullptr;
    long long part_blocks = 0;     // blocks per slot the partial buffers hold
    cx<double>* tot = nullptr;     // [slot * TOT + v]
    double* rtot = nullptr;        // [slot]
    cx<double>* tot_h = nullptr;   // pinned [rhs * TOT + v]
    double* rtot_h = nullptr;      // pinned [rhs]
    Prof prof;
};

namespace {

constexpr int TOT = 3 * HSTRIDE;   // H1 | H2 | norm

// ---------------------------------------------------------------------------
// Small utilities
// ---------------------------------------------------------------------------
template <typename P>
mg_status dalloc(P** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) return MG_OK;
    if (hipMalloc((void**)p, bytes) != hipSuccess) {
        *p = nullptr;
        return MG_E_NOMEM;
    }
    return MG_OK;
}
template <typename P>
mg_status halloc(P** p, size_t bytes) {
    *p = nullptr;
    if (hipHostMalloc((void**)p, bytes, hipHostMallocDefault) != hipSuccess) {
        *p = nullptr;
        return MG_E_NOMEM;
    }
    std::memset((void*)*p, 0, bytes);
    return MG_OK;
}
template <typename P>
void dfree(P*& p) {
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}
template <typename P>
void hfree(P*& p) {
    if (p) (void)hipHostFree((void*)p);
    p = nullptr;
}

// bytes: algorithmic (compulsory) traffic of the launch
int prof_begin(mg_ctx* c, int cls, double bytes = 0.0) {
    if (!c->prof.on) return -1;
    Prof& P = c->prof;
    while (P.pool.size() < 2 * (P.used + 1)) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return -1;
        P.pool.push_back(e);
    }
    const int idx = (int)P.used++;
    if ((int)P.cls.size() <= idx) {
        P.cls.resize(idx + 1);
        P.bytes.resize(idx + 1);
    }
    P.cls[idx] = cls;
    P.bytes[idx] = bytes;
    (void)hipEventRecord(P.pool[2 * idx], c->stream);
    return idx;
}
void prof_end(mg_ctx* c, int idx) {
    if (idx >= 0) (void)hipEventRecord(c->prof.pool[2 * idx + 1], c->stream);
}

template <typename T>
mg::LevelView<T> view(const mg_ctx* c, int l, int dir);

template <>
mg::LevelView<double> view<double>(const mg_ctx* c, int l, int dir) {
    const Level& L = c->lv[l];
    mg::LevelView<double> v{};
    long long off = 0;
    for (int a = 0; a < 3; ++a) {
        const int aa = a < c->dim ? a : 0;
        long long o = 0;
        for (int b = 0; b < aa; ++b) o += 3LL * L.n[b];
        v.n[a] = a < c->dim ? L.n[a] : 1;
        v.cm[a] = L.coef_d[dir] + o;
        v.c0[a] = L.coef_d[dir] + o + L.n[aa];
        v.cp[a] = L.coef_d[dir] + o + 2LL * L.n[aa];
        (void)off;
    }
    v.N = L.N;
    v.k2 = L.k2;
    const cd s = dir ? std::conj(L.sigma) : L.sigma;
    v.sigma = tocx(s);
    v.omega = mg::mk(c->p.omega[0], c->p.omega[1]);
    return v;
}

template <>
mg::LevelView<float> view<float>(const mg_ctx* c, int l, int dir) {
    const Level& L = c->lv[l];
    mg::LevelView<float> v{};
    for (int a = 0; a < 3; ++a) {
        const int aa = a < c->dim ? a : 0;
        long long o = 0;
        for (int b = 0; b < aa; ++b) o += 3LL * L.n[b];
        v.n[a] = a < c->dim ? L.n[a] : 1;
        v.cm[a] = L.coef_f[dir] + o;
        v.c0[a] = L.coef_f[dir] + o + L.n[aa];
        v.cp[a] = L.coef_f[dir] + o + 2LL * L.n[aa];
    }
    v.N = L.N;
    v.k2 = L.k2f;
    const cd s = dir ? std::conj(L.sigma) : L.sigma;
    v.sigma = mg::mk((float)s.real(), (float)s.imag());
    v.omega = mg::mk((float)c->p.omega[0], (float)c->p.omega[1]);
    return v;
}

// Split a list of slots into launch groups of at most MAX_SLOTS.
std::vector<SlotTable> groups(const std::vector<Slot>& slots) {
    std::vector<SlotTable> g;
    for (size_t i = 0; i < slots.size(); i += mg::MAX_SLOTS) {
        SlotTable t{};
        t.n = (int)std::min<size_t>(mg::MAX_SLOTS, slots.size() - i);
        for (int k = 0; k < t.n; ++k) t.s[k] = slots[i + k];
        g.push_back(t);
    }
    return g;
}

// ---------------------------------------------------------------------------
// V-cycle (Sec. 3.1): one group of at most MAX_SLOTS right-hand sides.
//   u0   level-0 incoming iterate by rhs (nullptr: zero initial guess)
//   f0   level-0 right-hand side, slot.in_off / slot.in_scale
//   out0 level-0 result, slot.out_off; acc: out0 += result
//   norm level-0 ||f - A u0||^2 partials per (local slot, tile), or nullptr
// ---------------------------------------------------------------------------
mg_status vcycle(mg_ctx* c, int dir, const SlotTable& st, const cx<double>* u0, const cx<double>* f0,
                 cx<double>* out0, bool acc, double* norm) {
    const int L = c->L;
    hipStream_t s = c->stream;
    if (c->mixed && u0) return MG_E_STATE;
    // algorithmic bytes per point: complex of the cycle precision, of the
    // level-0 input/output (FP64) and the real k^2
    const double ct = c->mixed ? 8.0 : 16.0, sk = c->mixed ? 4.0 : 8.0, c0b = 16.0;
    const double ns = st.n;
    for (int l = 0; l + 1 < L; ++l) {
        const Level& A = c->lv[l];
        const Level& B = c->lv[l + 1];
        // read f, k^2 (and u), write the coarse right-hand side (and u1)
        double by = ns * (A.N * ((l == 0 ? c0b : ct) + sk) + B.N * ct);
        if (l == 0 && u0) by += ns * A.N * 2.0 * ct;
        const int pi = prof_begin(c, l == 0 ? MG_K_SMOOTH_RESTRICT_FINE : MG_K_COARSE_LEVELS, by);
        if (!c->mixed) {
            mg::SmoothRestrictArgs<double, double> a{};
            a.lv = view<double>(c, l, dir);
            for (int k = 0; k < 3; ++k) a.nc[k] = k < c->dim ? B.n[k] : 1, a.ntiles[k] = A.ntiles[k];
            a.Nc = B.N;
            a.st = st;
            a.u = l == 0 ? u0 : nullptr;
            a.f = l == 0 ? f0 : (const cx<double>*)A.F;
            a.f_by_slot = l != 0;
            a.u1 = (l == 0 && u0) ? c->U1 : nullptr;
            a.fc = (cx<double>*)B.F;
            a.norm_part = (l == 0 && u0) ? norm : nullptr;
            CK(mg::launch_smooth_restrict_f64(c->dim, !(l == 0 && u0), a, nullptr, s));
        } else {
            mg::SmoothRestrictArgs<float, double> a0{};
            mg::SmoothRestrictArgs<float, float> ac{};
            auto fill = [&](auto& a) {
                a.lv = view<float>(c, l, dir);
                for (int k = 0; k < 3; ++k) a.nc[k] = k < c->dim ? B.n[k] : 1, a.ntiles[k] = A.ntiles[k];
                a.Nc = B.N;
                a.st = st;
                a.u = nullptr;
                a.u1 = nullptr;
                a.fc = (cx<float>*)B.F;
                a.norm_part = nullptr;
            };
            fill(a0);
            fill(ac);
            a0.f = f0;
            a0.f_by_slot = false;
            ac.f = (const cx<float>*)A.F;
            ac.f_by_slot = true;
            CK(mg::launch_smooth_restrict_f32(c->dim, l == 0, a0, ac, nullptr, s));
        }
        prof_end(c, pi);
    }
    {
        const Level& C = c->lv[L - 1];
        const int pi = prof_begin(c, MG_K_COARSEST_SOLVE, ns * C.N * 2.0 * ct);
        if (!c->mixed)
            CK(mg::launch_coarse_solve_f64(c->lu[dir], c->piv[dir], c->ncoarse, st, (const cx<double>*)C.F,
                                           (cx<double>*)C.E, s));
        else
            CK(mg::launch_coarse_solve_f32(c->lu[dir], c->piv[dir], c->ncoarse, st, (const cx<float>*)C.F,
                                           (cx<float>*)C.E, s));
        prof_end(c, pi);
    }
    for (int l = L - 2; l >= 0; --l) {
        const Level& A = c->lv[l];
        const Level& B = c->lv[l + 1];
        // read f, k^2, the coarse correction (and u1, and out when accumulating), write out
        const double cf = l == 0 ? c0b : ct;
        double by = ns * (A.N * (cf + sk + cf) + B.N * ct);
        if (l == 0 && u0) by += ns * A.N * ct;
        if (l == 0 && acc) by += ns * A.N * c0b;
        const int pi = prof_begin(c, l == 0 ? MG_K_PROLONG_SMOOTH_FINE : MG_K_COARSE_LEVELS, by);
        if (!c->mixed) {
            mg::ProlongSmoothArgs<double, double, double> a{};
            a.lv = view<double>(c, l, dir);
            for (int k = 0; k < 3; ++k) a.nc[k] = k < c->dim ? B.n[k] : 1, a.ntiles[k] = A.ntiles[k];
            a.Nc = B.N;
            a.st = st;
            a.u1 = (l == 0 && u0) ? c->U1 : nullptr;
            a.f = l == 0 ? f0 : (const cx<double>*)A.F;
            a.f_by_slot = l != 0;
            a.ec = (const cx<double>*)B.E;
            a.out = l == 0 ? out0 : (cx<double>*)A.E;
            a.out_by_slot = l != 0;
            CK(mg::launch_prolong_smooth_f64(c->dim, !(l == 0 && u0), l == 0 && acc, a, s));
        } else {
            mg::ProlongSmoothArgs<float, double, double> a0{};
            mg::ProlongSmoothArgs<float, float, float> ac{};
            auto fill = [&](auto& a) {
                a.lv = view<float>(c, l, dir);
                for (int k = 0; k < 3; ++k) a.nc[k] = k < c->dim ? B.n[k] : 1, a.ntiles[k] = A.ntiles[k];
                a.Nc = B.N;
                a.st = st;
                a.u1 = nullptr;
                a.ec = (const cx<float>*)B.E;
            };
            fill(a0);
            fill(ac);
            a0.f = f0;
            a0.f_by_slot = false;
            a0.out = out0;
            a0.out_by_slot = false;
            ac.f = (const cx<float>*)A.F;
            ac.f_by_slot = true;
            ac.out = (cx<float>*)A.E;
            ac.out_by_slot = true;
            CK(mg::launch_prolong_smooth_f32(c->dim, l == 0, acc, a0, ac, s));
        }
        prof_end(c, pi);
    }
    return MG_OK;
}

// ||.||^2 of the partials rpart[local slot][nblocks] -> rtot_h[rhs] (async D2H).
mg_status reduce_norms_to_host(mg_ctx* c, const SlotTable& st, int nblocks) {
    const int pi = prof_begin(c, MG_K_REDUCE);
    CK(mg::launch_reduce_real(c->rpart, nblocks, st.n, c->rtot, c->stream));
    prof_end(c, pi);
    // rtot[local] -> rtot_h[rhs]: copy contiguous block, scatter on the host later
    CK(hipMemcpyAsync(c->rtot_h + mg::MAX_SLOTS * 0, c->rtot, st.n * sizeof(double), hipMemcpyDeviceToHost,
                      c->stream));
    return MG_OK;
}

// Per-rhs ||v||^2 of a vector indexed by rhs (synchronises).
mg_status norms_by_rhs(mg_ctx* c, const std::vector<Slot>& slots, const cx<double>* x, std::vector<double>& out) {
    const long long N = c->lv[0].N;
    const int nb = mg::residual_blocks(N);
    for (const SlotTable& st : groups(slots)) {
        CK(mg::launch_norm(st, x, false, N, c->rpart, nb, c->stream));
        CK(mg::launch_reduce_real(c->rpart, nb, st.n, c->rtot, c->stream));
        CK(hipMemcpyAsync(c->rtot_h, c->rtot, st.n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        CK(hipStreamSynchronize(c->stream));
        for (int k = 0; k < st.n; ++k) out[st.s[k].rhs] = c->rtot_h[k];
    }
    return MG_OK;
}

// y = f - A x (f == nullptr: y = A x) for the slots, y at slot.out_off, with
// ||y||^2 per rhs into nrm (nullptr: skip; synchronises otherwise).
mg_status residual(mg_ctx* c, int l, int dir, const std::vector<Slot>& slots, const cx<double>* x,
                   const cx<double>* f, cx<double>* y, std::vector<double>* nrm) {
    const long long N = c->lv[l].N;
    const int nb = mg::residual_blocks(N);
    for (const SlotTable& st : groups(slots)) {
        mg::ResidualArgs a{};
        a.lv = view<double>(c, l, dir);
        a.st = st;
        a.x = x;
        a.f = f;
        a.y = y;
        a.norm_part = nrm ? c->rpart : nullptr;
        a.nblocks = nb;
        // read x, k^2 (and f), write y
        const int pi = prof_begin(c, MG_K_RESIDUAL, (double)st.n * N * (16.0 + 8.0 + 16.0 + (f ? 16.0 : 0.0)));
        CK(mg::launch_residual(c->dim, a, c->stream));
        prof_end(c, pi);
        if (nrm) {
            CKS(reduce_norms_to_host(c, st, nb));
            CK(hipStreamSynchronize(c->stream));
            for (int k = 0; k < st.n; ++k) (*nrm)[st.s[k].rhs] = c->rtot_h[k];
        }
    }
    return MG_OK;
}

mg_status ensure_basis(mg_ctx* c, int restart) {
    if (c->V && c->vstride >= restart + 1) return MG_OK;
    dfree(c->V);
    c->vstride = 0;
    const size_t bytes = (size_t)c->nrhs * (restart + 1) * c->lv[0].N * sizeof(cx<double>);
    CKS(dalloc(&c->V, bytes));
    c->vstride = restart + 1;
    return MG_OK;
}

// ---------------------------------------------------------------------------
// Standalone iteration (Sec. 4.1, LVL-MG): repeated cycles; the residual of
// the incoming iterate is formed inside the first fused kernel of each cycle
// (FP64) or by the FP64 residual of the refinement step (mixed).
// ---------------------------------------------------------------------------
mg_status solve_standalone(mg_ctx* c, int dir, double* u, const double* f, double rtol, int maxit,
                           int* iters, double* hist) {
    const long long N = c->lv[0].N;
    cx<double>* U = (cx<double>*)u;
    const cx<double>* F = (const cx<double>*)f;
    std::vector<Slot> all(c->nrhs);
    for (int r = 0; r < c->nrhs; ++r) {
        all[r] = Slot{};
        all[r].rhs = r;
        all[r].buf = r;
        all[r].in_off = (long long)r * N;
        all[r].out_off = (long long)r * N;
        all[r].in_scale = 1.0;
    }
    std::vector<double> nf(c->nrhs);
    CKS(norms_by_rhs(c, all, F, nf));
    std::vector<int> state(c->nrhs, 0);   // 0 running, 1 converged, 2 maxit, 3 diverged
    std::vector<int> its(c->nrhs, 0);
    std::vector<Slot> active;
    for (int r = 0; r < c->nrhs; ++r) {
        if (nf[r] == 0.0) {   // f = 0: the solution is 0
            CK(mg::launch_fill_zero(U + (long long)r * N, N * sizeof(cx<double>), c->stream));
            state[r] = 1;
            if (hist) hist[(size_t)r * (maxit + 1)] = 0.0;
        } else {
            active.push_back(all[r]);
        }
    }
    const int ntile0 = c->lv[0].ntiles[0] * c->lv[0].ntiles[1] * c->lv[0].ntiles[2];
    for (int k = 0; k < maxit && !active.empty(); ++k) {
        std::vector<double> rho(c->nrhs, 0.0);
        for (const SlotTable& st : groups(active)) {
            if (!c->mixed) {
                CKS(vcycle(c, dir, st, U, F, U, false, c->rpart));
                CKS(reduce_norms_to_host(c, st, ntile0));
                CK(hipStreamSynchronize(c->stream));
                for (int q = 0; q < st.n; ++q) rho[st.s[q].rhs] = c->rtot_h[q];
            } else {
                // iterative refinement form: r = f - A u (FP64), u += M r
                std::vector<Slot> v(st.s, st.s + st.n);
                for (Slot& x : v) x.out_off = (long long)x.buf * N;
                std::vector<double> nr(c->nrhs);
                CKS(residual(c, 0, dir, v, U, F, c->W, &nr));
                for (int q = 0; q < st.n; ++q) rho[st.s[q].rhs] = nr[st.s[q].rhs];
                SlotTable s2 = st;
                for (int q = 0; q < s2.n; ++q) s2.s[q].in_off = (long long)s2.s[q].buf * N;
                CKS(vcycle(c, dir, s2, nullptr, c->W, U, true, nullptr));
            }
        }
        std::vector<Slot> next;
        for (const Slot& sl : active) {
            const int r = sl.rhs;
            const double ratio = std::sqrt(rho[r]) / std::sqrt(nf[r]);
            if (hist) hist[(size_t)r * (maxit + 1) + k] = ratio;
            its[r] = k;
            if (ratio <= rtol) {
                state[r] = 1;
            } else if (!std::isfinite(ratio) || ratio > DIVERGE) {
                state[r] = 3;
            } else {
                its[r] = k + 1;
                next.push_back(sl);
            }
        }
        active.swap(next);
    }
    CK(hipStreamSynchronize(c->stream));
    mg_status ret = MG_OK;
    for (int r = 0; r < c->nrhs; ++r) {
        if (state[r] == 0) state[r] = 2;
        if (iters) iters[r] = its[r];
        if (state[r] == 3) ret = MG_E_DIVERGED;
        else if (state[r] == 2 && ret == MG_OK) ret = MG_NOT_CONVERGED;
    }
    return ret;
}

// ---------------------------------------------------------------------------
// Restarted right-preconditioned GMRES(m) (Sec. 4.1: one V(1,1) cycle from a
// zero guess per outer step).  Arnoldi by classical Gram-Schmidt with one
// re-orthogonalisation pass; Hessenberg least squares by complex Givens
// rotations on the host; x += M (V y) at the end of each restart cycle (the
// cycle is a fixed linear map).
// ---------------------------------------------------------------------------
struct GmresState {
    int j = 0;                  // basis vectors V_0..V_j exist
    int its = 0;
    int state = 0;              // 0 arnoldi, 1 converged, 2 maxit, 3 diverged
    bool finish = false;        // restart cycle ends after this step
    double nf = 0.0;
    std::vector<cd> H;          // (m+1) x m, column-major
    std::vector<double> cs;
    std::vector<cd> sn;
    std::vector<cd> g;
};

mg_status solve_gmres(mg_ctx* c, int dir, double* x, const double* f, double rtol, int maxit, int m,
                      int* iters, double* hist) {
    const long long N = c->lv[0].N;
    cx<double>* X = (cx<double>*)x;
    const cx<double>* F = (const cx<double>*)f;
    CKS(ensure_basis(c, m));
    const int vs = c->vstride;
    std::vector<GmresState> gs(c->nrhs);
    std::vector<Slot> all(c->nrhs);
    for (int r = 0; r < c->nrhs; ++r) {
        all[r] = Slot{};
        all[r].rhs = r;
        all[r].buf = r;
        all[r].in_scale = 1.0;
        gs[r].H.assign((size_t)(m + 1) * m, 0.0);
        gs[r].cs.assign(m, 0.0);
        gs[r].sn.assign(m, 0.0);
        gs[r].g.assign(m + 1, 0.0);
    }
    std::vector<double> nf(c->nrhs);
    CKS(norms_by_rhs(c, all, F, nf));
    std::vector<int> hist_len(c->nrhs, 0);
    auto push_hist = [&](int r, double v) {
        if (hist && hist_len[r] <= maxit) hist[(size_t)r * (maxit + 1) + hist_len[r]] = v;
        hist_len[r]++;
    };

    // (Re)start: r = f - A x into V_0, beta = ||r||; decide per rhs.
    auto restart = [&](std::vector<int>& who) -> mg_status {
        std::vector<Slot> sl;
        for (int r : who) {
            Slot s = all[r];
            s.out_off = (long long)r * vs * N;
            sl.push_back(s);
        }
        std::vector<double> beta2(c->nrhs, 0.0);
        CKS(residual(c, 0, dir, sl, X, F, c->V, &beta2));
        for (int r : who) {
            GmresState& G = gs[r];
            const double beta = std::sqrt(beta2[r]);
            const double ratio = beta / G.nf;
            if (hist_len[r] == 0) push_hist(r, ratio);
            if (ratio <= rtol) {
                G.state = 1;
            } else if (!std::isfinite(ratio)) {
                G.state = 3;
            } else if (G.its >= maxit) {
                G.state = 2;
            } else {
                G.j = 0;
                G.finish = false;
                std::fill(G.g.begin(), G.g.end(), cd(0.0));
                G.g[0] = beta;
                c->scale_h[(size_t)r * HSTRIDE + 0] = 1.0 / beta;
            }
        }
        return MG_OK;
    };

    std::vector<int> who;
    for (int r = 0; r < c->nrhs; ++r) {
        gs[r].nf = std::sqrt(nf[r]);
        if (nf[r] == 0.0) {
            CK(mg::launch_fill_zero(X + (long long)r * N, N * sizeof(cx<double>), c->stream));
            gs[r].state = 1;
            push_hist(r, 0.0);
        } else {
            who.push_back(r);
        }
    }
    CKS(restart(who));

    for (;;) {
        std::vector<Slot> act;
        int jmax = 0;
        for (int r = 0; r < c->nrhs; ++r) {
            if (gs[r].state != 0) continue;
            Slot s = all[r];
            s.j = gs[r].j;
            s.in_off = ((long long)r * vs + gs[r].j) * N;
            s.in_scale = c->scale_h[(size_t)r * HSTRIDE + gs[r].j];
            s.out_off = (long long)r * N;
            act.push_back(s);
            jmax = std::max(jmax, gs[r].j + 1);
        }
        if (act.empty()) break;
        // scales of every active basis to the device
        CK(hipMemcpyAsync(c->scale_d, c->scale_h, (size_t)c->nrhs * HSTRIDE * sizeof(double),
                          hipMemcpyHostToDevice, c->stream));
        const int nb = mg::ortho_blocks(N);
        int gbase = 0;
        for (const SlotTable& st : groups(act)) {
            // z = M v_j
            CKS(vcycle(c, dir, st, nullptr, c->V, c->Z, false, nullptr));
            mg::OrthoArgs o{};
            o.lv = view<double>(c, 0, dir);
            o.st = st;
            o.N = N;
            o.z = c->Z;
            o.w = c->W;
            o.Vb = c->V;
            o.vstride = vs;
            o.scale = c->scale_d;
            o.sstride = HSTRIDE;
            o.hstride = TOT;
            o.part = c->part;
            o.pstride = HSTRIDE;
            o.nblocks = nb;
            // basis vectors read per pass: sum over slots of (j + 1)
            double nvsum = 0.0;
            for (int q = 0; q < st.n; ++q) nvsum += st.s[q].j + 1;
            const double vb = 16.0 * N;
            // pass 1: w = A z, h1 = V^H w; reads z, k^2, V_0..V_j, writes w
            int pi = prof_begin(c, MG_K_MATVEC_DOT, vb * (nvsum + 2.0 * st.n) + 8.0 * N * st.n);
            CK(mg::launch_matvec_dot(c->dim, jmax, o, c->stream));
            prof_end(c, pi);
            pi = prof_begin(c, MG_K_REDUCE);
            CK(mg::launch_reduce_complex(c->part, jmax, HSTRIDE, nb, st.n, c->tot, TOT, c->stream));
            prof_end(c, pi);
            // pass 2: w -= V h1, h2 = V^H w
            o.hin = c->tot;
            pi = prof_begin(c, MG_K_UPDATE_DOT, vb * (nvsum + 2.0 * st.n));
            CK(mg::launch_update_dot(jmax, o, c->stream));
            prof_end(c, pi);
            pi = prof_begin(c, MG_K_REDUCE);
            CK(mg::launch_reduce_complex(c->part, jmax, HSTRIDE, nb, st.n, c->tot + HSTRIDE, TOT, c->stream));
            prof_end(c, pi);
            // pass 3: V_{j+1} = w - V h2, ||V_{j+1}||^2
            o.hin = c->tot + HSTRIDE;
            pi = prof_begin(c, MG_K_UPDATE_NORM, vb * (nvsum + 2.0 * st.n));
            CK(mg::launch_update_norm(jmax, o, c->stream));
            prof_end(c, pi);
            pi = prof_begin(c, MG_K_REDUCE);
            CK(mg::launch_reduce_complex(c->part, 1, HSTRIDE, nb, st.n, c->tot + 2 * HSTRIDE, TOT, c->stream));
            prof_end(c, pi);
            CK(hipMemcpyAsync(c->tot_h + (size_t)gbase * TOT, c->tot, (size_t)st.n * TOT * sizeof(cx<double>),
                              hipMemcpyDeviceToHost, c->stream));
            gbase += st.n;
        }
        CK(hipStreamSynchronize(c->stream));

        std::vector<int> fin;
        for (size_t q = 0; q < act.size(); ++q) {
            const int r = act[q].rhs;
            GmresState& G = gs[r];
            const cx<double>* T = c->tot_h + q * TOT;
            const int j = G.j;
            cd* col = &G.H[(size_t)j * (m + 1)];
            for (int i = 0; i <= j; ++i) col[i] = cd(T[i].r, T[i].i) + cd(T[HSTRIDE + i].r, T[HSTRIDE + i].i);
            const double hn = std::sqrt(std::max(0.0, T[2 * HSTRIDE].r));
            col[j + 1] = hn;
            for (int i = 0; i < j; ++i) {
                const cd a = col[i], b = col[i + 1];
                col[i] = G.cs[i] * a + G.sn[i] * b;
                col[i + 1] = -std::conj(G.sn[i]) * a + G.cs[i] * b;
            }
            // rotation j zeroing col[j+1] below col[j]
            const cd a = col[j], b = col[j + 1];
            double cj;
            cd sj;
            if (b == 0.0) {
                cj = 1.0;
                sj = 0.0;
            } else if (a == 0.0) {
                cj = 0.0;
                sj = std::conj(b) / std::abs(b);
            } else {
                const double t = std::hypot(std::abs(a), std::abs(b));
                cj = std::abs(a) / t;
                sj = (a / std::abs(a)) * std::conj(b) / t;
            }
            G.cs[j] = cj;
            G.sn[j] = sj;
            col[j] = cj * a + sj * b;
            col[j + 1] = 0.0;
            G.g[j + 1] = -std::conj(sj) * G.g[j];
            G.g[j] = cj * G.g[j];
            G.its++;
            const double est = std::abs(G.g[j + 1]) / G.nf;
            push_hist(r, est);
            if (!std::isfinite(est)) {
                G.state = 3;
                continue;
            }
            if (hn != 0.0) c->scale_h[(size_t)r * HSTRIDE + j + 1] = 1.0 / hn;
            if (est <= rtol || G.its >= maxit || j + 1 == m || hn == 0.0) {
                fin.push_back(r);
            } else {
                G.j = j + 1;
            }
        }
        if (!fin.empty()) {
            // y = R^{-1} g, x += M (V y)
            std::vector<Slot> fs;
            for (int r : fin) {
                GmresState& G = gs[r];
                const int k = G.j + 1;
                std::vector<cd> y(k);
                for (int i = k - 1; i >= 0; --i) {
                    cd s = G.g[i];
                    for (int l = i + 1; l < k; ++l) s -= G.H[(size_t)l * (m + 1) + i] * y[l];
                    y[i] = s / G.H[(size_t)i * (m + 1) + i];
                }
                for (int i = 0; i < k; ++i)
                    c->coef_h[(size_t)r * HSTRIDE + i] = tocx(y[i] * c->scale_h[(size_t)r * HSTRIDE + i]);
                Slot s = all[r];
                s.j = G.j;
                s.in_off = (long long)r * N;   // combine output W by buf (= r)
                s.in_scale = 1.0;
                s.out_off = (long long)r * N;
                fs.push_back(s);
            }
            CK(hipMemcpyAsync(c->coef_d, c->coef_h, (size_t)c->nrhs * HSTRIDE * sizeof(cx<double>),
                              hipMemcpyHostToDevice, c->stream));
            int jm = 0;
            for (int r : fin) jm = std::max(jm, gs[r].j + 1);
            for (const SlotTable& st : groups(fs)) {
                mg::CombineArgs cb{};
                cb.st = st;
                cb.N = N;
                cb.Vb = c->V;
                cb.vstride = vs;
                cb.coef = c->coef_d;
                cb.sstride = HSTRIDE;
                cb.t = c->W;
                double nvsum = 0.0;
                for (int q = 0; q < st.n; ++q) nvsum += st.s[q].j + 1;
                const int pi = prof_begin(c, MG_K_COMBINE, 16.0 * N * (nvsum + st.n));
                CK(mg::launch_combine(jm, cb, c->stream));
                prof_end(c, pi);
                CKS(vcycle(c, dir, st, nullptr, c->W, X, true, nullptr));
            }
            CKS(restart(fin));
        }
    }
    CK(hipStreamSynchronize(c->stream));
    mg_status ret = MG_OK;
    for (int r = 0; r < c->nrhs; ++r) {
        if (iters) iters[r] = gs[r].its;
        if (gs[r].state == 3) ret = MG_E_DIVERGED;
        else if (gs[r].state == 2 && ret == MG_OK) ret = MG_NOT_CONVERGED;
    }
    return ret;
}

mg_status solve(mg_ctx* c, int dir, double* u, const double* f, int mode, double rtol, int maxit, int restart,
                int* iters, double* hist) {
    if (!c || !u || !f || maxit < 0 || !(rtol >= 0.0)) return MG_E_INVAL;
    if (hist)
        for (size_t i = 0; i < (size_t)c->nrhs * (maxit + 1); ++i) hist[i] = -1.0;
    if (mode == MG_MODE_STANDALONE) return solve_standalone(c, dir, u, f, rtol, maxit, iters, hist);
    if (mode == MG_MODE_GMRES) {
        if (restart < 1 || restart > MAX_RESTART) return MG_E_INVAL;
        return solve_gmres(c, dir, u, f, rtol, maxit, restart, iters, hist);
    }
    return MG_E_INVAL;
}

void release(mg_ctx* c) {
    if (!c) return;
    for (Level& L : c->lv) {
        for (int d = 0; d < 2; ++d) {
            dfree(L.coef_d[d]);
            dfree(L.coef_f[d]);
        }
        dfree(L.k2);
        dfree(L.k2f);
        dfree(L.F);
        dfree(L.E);
    }
    for (int d = 0; d < 2; ++d) {
        dfree(c->lu[d]);
        dfree(c->piv[d]);
    }
    dfree(c->U1);
    dfree(c->Z);
    dfree(c->W);
    dfree(c->V);
    dfree(c->scale_d);
    dfree(c->coef_d);
    dfree(c->part);
    dfree(c->rpart);
    dfree(c->tot);
    dfree(c->rtot);
    hfree(c->scale_h);
    hfree(c->coef_h);
    hfree(c->tot_h);
    hfree(c->rtot_h);
    for (hipEvent_t e : c->prof.pool) (void)hipEventDestroy(e);
    c->prof.pool.clear();
}

mg_status setup(const mg_params* p, const double* k2_dev, void* stream, mg_ctx* c) {
    c->p = *p;
    c->dim = p->ndim;
    c->nrhs = p->nrhs;
    c->mixed = p->precision == MG_PREC_MIXED;
    c->stream = (hipStream_t)stream;
    const int d = c->dim;

    // level sizes
    int n[3] = {p->n[0], p->n[1], d == 3 ? p->n[2] : 1};
    int L = p->nlevels;
    if (L <= 0) {
        L = 1;
        int m[3] = {n[0], n[1], n[2]};
        for (;;) {
            bool ok = true;
            for (int a = 0; a < d; ++a) ok = ok && (m[a] % 2 == 1) && ((m[a] - 1) / 2 >= 2);
            if (!ok) break;
            for (int a = 0; a < d; ++a) m[a] = (m[a] - 1) / 2;
            ++L;
        }
    }
    if (L < 2) return MG_E_INVAL;
    c->L = L;
    c->lv.resize(L);
    for (int l = 0; l < L; ++l) {
        Level& V = c->lv[l];
        for (int a = 0; a < 3; ++a) {
            V.n[a] = a < d ? (l == 0 ? n[a] : (c->lv[l - 1].n[a] - 1) / 2) : 1;
            V.h[a] = a < d ? (l == 0 ? p->h[a] : 2.0 * c->lv[l - 1].h[a]) : 0.0;
        }
        for (int a = 0; a < d; ++a) {
            if (V.n[a] < 1) return MG_E_INVAL;
            if (l + 1 < L && V.n[a] % 2 == 0) return MG_E_INVAL;
        }
        V.N = (long long)V.n[0] * V.n[1] * V.n[2];
        mg::tile_counts(d, c->mixed, V.n, V.ntiles);
    }
    c->ncoarse = (int)c->lv[L - 1].N;
    if (c->ncoarse > mg::MAX_COARSE) return MG_E_INVAL;

    // shifts (Sec. 3.1): sigma_l = e^{i l theta_max / L} unless given
    for (int l = 0; l < L; ++l) {
        if (p->sigma)
            c->lv[l].sigma = cd(p->sigma[2 * l], p->sigma[2 * l + 1]);
        else
            c->lv[l].sigma = std::polar(1.0, l * p->theta_max / L);
    }
    if (c->lv[0].sigma != cd(1.0, 0.0)) return MG_E_INVAL;

    // coefficients of every level, forward and conjugate transpose
    for (int l = 0; l < L; ++l) {
        Level& V = c->lv[l];
        for (int dir = 0; dir < 2; ++dir) V.coef_host[dir].clear();
        for (int a = 0; a < d; ++a) {
            const double len = (p->n[a] + 1) * p->h[a];
            const double lo = p->ecs_lo[a] * p->h[a];
            const double hi = len - p->ecs_hi[a] * p->h[a];
            std::vector<cd> cm, c0, cp;
            axis_coefficients(V.n[a], V.h[a], lo, hi, p->ecs_angle, cm, c0, cp);
            const int na = V.n[a];
            std::vector<cd> hm(na), h0(na), hp(na);
            for (int j = 0; j < na; ++j) {
                hm[j] = j > 0 ? std::conj(cp[j - 1]) : cd(0.0);
                hp[j] = j + 1 < na ? std::conj(cm[j + 1]) : cd(0.0);
                h0[j] = std::conj(c0[j]);
            }
            auto& F = V.coef_host[0];
            F.insert(F.end(), cm.begin(), cm.end());
            F.insert(F.end(), c0.begin(), c0.end());
            F.insert(F.end(), cp.begin(), cp.end());
            auto& H = V.coef_host[1];
            H.insert(H.end(), hm.begin(), hm.end());
            H.insert(H.end(), h0.begin(), h0.end());
            H.insert(H.end(), hp.begin(), hp.end());
        }
        for (int dir = 0; dir < 2; ++dir) {
            const auto& src = V.coef_host[dir];
            std::vector<cx<double>> cdv(src.size());
            std::vector<cx<float>> cfv(src.size());
            for (size_t i = 0; i < src.size(); ++i) {
                cdv[i] = tocx(src[i]);
                cfv[i] = mg::mk((float)src[i].real(), (float)src[i].imag());
            }
            CKS(dalloc(&V.coef_d[dir], cdv.size() * sizeof(cx<double>)));
            CK(hipMemcpy(V.coef_d[dir], cdv.data(), cdv.size() * sizeof(cx<double>), hipMemcpyHostToDevice));
            if (c->mixed) {
                CKS(dalloc(&V.coef_f[dir], cfv.size() * sizeof(cx<float>)));
                CK(hipMemcpy(V.coef_f[dir], cfv.data(), cfv.size() * sizeof(cx<float>), hipMemcpyHostToDevice));
            }
        }
    }

    // k^2 on every level (rediscretisation: sampled at the coarse nodes)
    CKS(dalloc(&c->lv[0].k2, c->lv[0].N * sizeof(double)));
    CK(hipMemcpyAsync(c->lv[0].k2, k2_dev, c->lv[0].N * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    for (int l = 1; l < L; ++l) {
        CKS(dalloc(&c->lv[l].k2, c->lv[l].N * sizeof(double)));
        CK(mg::launch_inject_k2(d, c->lv[l - 1].k2, c->lv[l - 1].n, c->lv[l].k2, c->lv[l].n, c->stream));
    }
    if (c->mixed)
        for (int l = 0; l < L; ++l) {
            CKS(dalloc(&c->lv[l].k2f, c->lv[l].N * sizeof(float)));
            CK(mg::launch_to_f32(c->lv[l].k2, c->lv[l].k2f, c->lv[l].N, c->stream));
        }

    // coarsest operator and its conjugate transpose, LU in FP64 on the host
    {
        const Level& C = c->lv[L - 1];
        const int nc = c->ncoarse;
        std::vector<double> k2c(nc);
        CK(hipMemcpyAsync(k2c.data(), C.k2, nc * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        CK(hipStreamSynchronize(c->stream));
        std::vector<cd> A((size_t)nc * nc, 0.0);
        const auto& cf = C.coef_host[0];
        long long off[3] = {0, 0, 0};
        for (int a = 1; a < d; ++a) off[a] = off[a - 1] + 3LL * C.n[a - 1];
        const long long stride[3] = {1, C.n[0], (long long)C.n[0] * C.n[1]};
        for (int p0 = 0; p0 < nc; ++p0) {
            int idx[3] = {p0 % C.n[0], (p0 / C.n[0]) % C.n[1], p0 / (C.n[0] * C.n[1])};
            cd diag = -C.sigma * k2c[p0];
            for (int a = 0; a < d; ++a) {
                const int i = idx[a], na = C.n[a];
                diag += cf[off[a] + na + i];
                if (i > 0) A[(size_t)p0 * nc + p0 - stride[a]] += cf[off[a] + i];
                if (i + 1 < na) A[(size_t)p0 * nc + p0 + stride[a]] += cf[off[a] + 2 * na + i];
            }
            A[(size_t)p0 * nc + p0] += diag;
        }
        std::vector<cd> AH((size_t)nc * nc);
        for (int i = 0; i < nc; ++i)
            for (int j = 0; j < nc; ++j) AH[(size_t)i * nc + j] = std::conj(A[(size_t)j * nc + i]);
        for (int dir = 0; dir < 2; ++dir) {
            std::vector<cd>& M = dir ? AH : A;
            std::vector<int> piv;
            if (!lu_factor(M, piv, nc)) return MG_E_INVAL;
            std::vector<cx<double>> Mc(M.size());
            for (size_t i = 0; i < M.size(); ++i) Mc[i] = tocx(M[i]);
            CKS(dalloc(&c->lu[dir], Mc.size() * sizeof(cx<double>)));
            CKS(dalloc(&c->piv[dir], nc * sizeof(int)));
            CK(hipMemcpy(c->lu[dir], Mc.data(), Mc.size() * sizeof(cx<double>), hipMemcpyHostToDevice));
            CK(hipMemcpy(c->piv[dir], piv.data(), nc * sizeof(int), hipMemcpyHostToDevice));
        }
    }

    // work vectors
    const size_t esz = c->mixed ? sizeof(cx<float>) : sizeof(cx<double>);
    for (int l = 1; l < L; ++l) {
        CKS(dalloc(&c->lv[l].F, (size_t)c->nrhs * c->lv[l].N * esz));
        CKS(dalloc(&c->lv[l].E, (size_t)c->nrhs * c->lv[l].N * esz));
    }
    const size_t vbytes = (size_t)c->nrhs * c->lv[0].N * sizeof(cx<double>);
    if (!c->mixed) CKS(dalloc(&c->U1, vbytes));
    CKS(dalloc(&c->Z, vbytes));
    CKS(dalloc(&c->W, vbytes));
    const int ntile0 = c->lv[0].ntiles[0] * c->lv[0].ntiles[1] * c->lv[0].ntiles[2];
    c->part_blocks = std::max<long long>({(long long)ntile0, mg::residual_blocks(c->lv[0].N),
                                          mg::ortho_blocks(c->lv[0].N)});
    CKS(dalloc(&c->part, (size_t)mg::MAX_SLOTS * TOT * c->part_blocks * sizeof(cx<double>)));
    CKS(dalloc(&c->rpart, (size_t)mg::MAX_SLOTS * c->part_blocks * sizeof(double)));
    CKS(dalloc(&c->tot, (size_t)mg::MAX_SLOTS * TOT * sizeof(cx<double>)));
    CKS(dalloc(&c->rtot, (size_t)mg::MAX_SLOTS * sizeof(double)));
    CKS(dalloc(&c->scale_d, (size_t)c->nrhs * HSTRIDE * sizeof(double)));
    CKS(dalloc(&c->coef_d, (size_t)c->nrhs * HSTRIDE * sizeof(cx<double>)));
    CKS(halloc(&c->scale_h, (size_t)c->nrhs * HSTRIDE * sizeof(double)));
    CKS(halloc(&c->coef_h, (size_t)c->nrhs * HSTRIDE * sizeof(cx<double>)));
    CKS(halloc(&c->tot_h, (size_t)std::max(c->nrhs, mg::MAX_SLOTS) * TOT * sizeof(cx<double>)));
    CKS(halloc(&c->rtot_h, (size_t)std::max(c->nrhs, mg::MAX_SLOTS) * sizeof(double)));
    CK(hipStreamSynchronize(c->stream));
    return MG_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

void mg_params_default(mg_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->ndim = 2;
    p->n[0] = p->n[1] = p->n[2] = 1;
    p->h[0] = p->h[1] = p->h[2] = 1.0;
    p->ecs_angle = M_PI / 4;
    p->theta_max = M_PI / 6;
    p->nu1 = p->nu2 = 1;
    p->omega[0] = 2.0 / 3.0;
    p->precision = MG_PREC_C128;
    p->nrhs = 1;
}

mg_status mg_setup(const mg_params* p, const double* k2_dev, void* stream, mg_ctx** out) {
    if (!out) return MG_E_INVAL;
    *out = nullptr;
    if (!p || !k2_dev) return MG_E_INVAL;
    if (p->ndim != 2 && p->ndim != 3) return MG_E_INVAL;
    if (p->nrhs < 1 || p->nu1 != 1 || p->nu2 != 1) return MG_E_INVAL;
    if (p->precision != MG_PREC_C128 && p->precision != MG_PREC_MIXED) return MG_E_INVAL;
    for (int a = 0; a < p->ndim; ++a) {
        if (p->n[a] < 3 || !(p->h[a] > 0.0)) return MG_E_INVAL;
        if (p->ecs_lo[a] < 0 || p->ecs_hi[a] < 0 || p->ecs_lo[a] + p->ecs_hi[a] > p->n[a] + 1) return MG_E_INVAL;
    }
    if (p->nlevels < 0 || !std::isfinite(p->theta_max) || !std::isfinite(p->ecs_angle)) return MG_E_INVAL;
    long long N = 1;
    for (int a = 0; a < p->ndim; ++a) N *= p->n[a];
    if (N >= (1LL << 31)) return MG_E_INVAL;
    mg_ctx* c = new (std::nothrow) mg_ctx();
    if (!c) return MG_E_NOMEM;
    const mg_status st = setup(p, k2_dev, stream, c);
    if (st != MG_OK) {
        release(c);
        delete c;
        return st;
    }
    *out = c;
    return MG_OK;
}

mg_status mg_cycle(mg_ctx* c, double* u, const double* f, double* res_before) {
    if (!c || !u || !f) return MG_E_INVAL;
    const long long N = c->lv[0].N;
    std::vector<Slot> all(c->nrhs);
    for (int r = 0; r < c->nrhs; ++r) {
        all[r] = Slot{};
        all[r].rhs = r;
        all[r].buf = r;
        all[r].in_off = (long long)r * N;
        all[r].out_off = (long long)r * N;
        all[r].in_scale = 1.0;
    }
    cx<double>* U = (cx<double>*)u;
    const cx<double>* F = (const cx<double>*)f;
    const int ntile0 = c->lv[0].ntiles[0] * c->lv[0].ntiles[1] * c->lv[0].ntiles[2];
    for (const SlotTable& st : groups(all)) {
        if (!c->mixed) {
            CKS(vcycle(c, 0, st, U, F, U, false, res_before ? c->rpart : nullptr));
            if (res_before) {
                CKS(reduce_norms_to_host(c, st, ntile0));
                CK(hipStreamSynchronize(c->stream));
                for (int q = 0; q < st.n; ++q) res_before[st.s[q].rhs] = std::sqrt(c->rtot_h[q]);
            }
        } else {
            std::vector<Slot> v(st.s, st.s + st.n);
            for (Slot& x : v) x.out_off = (long long)x.buf * N;
            std::vector<double> nr(c->nrhs);
            CKS(residual(c, 0, 0, v, U, F, c->W, res_before ? &nr : nullptr));
            if (res_before)
                for (int q = 0; q < st.n; ++q) res_before[st.s[q].rhs] = std::sqrt(nr[st.s[q].rhs]);
            SlotTable s2 = st;
            for (int q = 0; q < s2.n; ++q) s2.s[q].in_off = (long long)s2.s[q].buf * N;
            CKS(vcycle(c, 0, s2, nullptr, c->W, U, true, nullptr));
        }
    }
    return MG_OK;
}

mg_status mg_solve(mg_ctx* c, double* u, const double* f, int mode, double rtol, int maxit, int restart,
                   int* iters, double* hist) {
    return solve(c, 0, u, f, mode, rtol, maxit, restart, iters, hist);
}

mg_status mg_solve_adjoint(mg_ctx* c, double* lam, const double* g, int mode, double rtol, int maxit,
                           int restart, int* iters, double* hist) {
    return solve(c, 1, lam, g, mode, rtol, maxit, restart, iters, hist);
}

mg_status mg_grad_k2(mg_ctx* c, const double* u, const double* lam, double* grad) {
    if (!c || !u || !lam || !grad) return MG_E_INVAL;
    const int pi = prof_begin(c, MG_K_OTHER, (double)c->lv[0].N * (32.0 * c->nrhs + 16.0));
    CK(mg::launch_grad_k2((const cx<double>*)u, (const cx<double>*)lam, c->nrhs, c->lv[0].N, grad, c->stream));
    prof_end(c, pi);
    return MG_OK;
}

mg_status mg_apply(mg_ctx* c, int level, int adjoint, const double* x, double* y) {
    if (!c || !x || !y || level < 0 || level >= c->L) return MG_E_INVAL;
    const long long N = c->lv[level].N;
    std::vector<Slot> all(c->nrhs);
    for (int r = 0; r < c->nrhs; ++r) {
        all[r] = Slot{};
        all[r].rhs = r;
        all[r].buf = r;
        all[r].out_off = (long long)r * N;
    }
    return residual(c, level, adjoint ? 1 : 0, all, (const cx<double>*)x, nullptr, (cx<double>*)y, nullptr);
}

int mg_num_levels(const mg_ctx* c) { return c ? c->L : 0; }

mg_status mg_level_dims(const mg_ctx* c, int level, int n[3]) {
    if (!c || !n || level < 0 || level >= c->L) return MG_E_INVAL;
    for (int a = 0; a < 3; ++a) n[a] = c->lv[level].n[a];
    return MG_OK;
}

mg_status mg_get_sigma(const mg_ctx* c, double* sigma) {
    if (!c || !sigma) return MG_E_INVAL;
    for (int l = 0; l < c->L; ++l) {
        sigma[2 * l] = c->lv[l].sigma.real();
        sigma[2 * l + 1] = c->lv[l].sigma.imag();
    }
    return MG_OK;
}

mg_status mg_profile(mg_ctx* c, int enable) {
    if (!c) return MG_E_INVAL;
    CK(hipStreamSynchronize(c->stream));
    c->prof.on = enable != 0;
    c->prof.used = 0;
    return MG_OK;
}

mg_status mg_profile_read(mg_ctx* c, int which, double* total_ms, long long* count, double* bytes) {
    if (!c || which < 0 || which >= MG_K_NUM_CLASSES) return MG_E_INVAL;
    CK(hipStreamSynchronize(c->stream));
    double tot = 0.0, by = 0.0;
    long long n = 0;
    for (size_t i = 0; i < c->prof.used; ++i) {
        if (c->prof.cls[i] != which) continue;
        float ms = 0.0f;
        CK(hipEventElapsedTime(&ms, c->prof.pool[2 * i], c->prof.pool[2 * i + 1]));
        tot += ms;
        by += c->prof.bytes[i];
        ++n;
    }
    if (total_ms) *total_ms = tot;
    if (count) *count = n;
    if (bytes) *bytes = by;
    return MG_OK;
}

void mg_destroy(mg_ctx* c) {
    if (!c) return;
    if (c->stream || true) (void)hipStreamSynchronize(c->stream);
    release(c);
    delete c;
}

const char* mg_status_str(mg_status s) {
    switch (s) {
        case MG_OK: return "ok";
        case MG_NOT_CONVERGED: return "not converged within maxit";
        case MG_E_INVAL: return "invalid argument";
        case MG_E_NOMEM: return "out of memory";
        case MG_E_DEVICE: return "HIP runtime error";
        case MG_E_DIVERGED: return "diverged";
        case MG_E_STATE: return "invalid call for this context";
    }
    return "unknown status";
}

}  // extern "C"
