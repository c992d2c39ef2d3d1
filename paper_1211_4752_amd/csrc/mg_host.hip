// Host runtime of the level-dependent multigrid: hierarchy set-up, tile-shape
// autotuning, the V-cycle driver (coarse part captured as a HIP graph), the
// standalone and GMRES solvers over "items" (one right-hand side of one
// problem), batches of problems, the adjoint, and the C ABI of include/mg.h.
//
// Paper: Cools, Reps, Vanroose, "A new level-dependent coarse grid correction
// scheme for indefinite Helmholtz problems" (NLAA 2013).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "mg.h"
#include "mg_device.hpp"

using cd = std::complex<double>;
using mg::CycleArgs;
using mg::CycleSlot;
using mg::cx;
using mg::LevelView;
using mg::ReduceArgs;
using mg::VecArgs;
using mg::VecSlot;

namespace {

constexpr int MAX_RESTART = 32;
constexpr int HSTRIDE = MAX_RESTART + 1;     // per-slot stride of one set of dot results
constexpr int TOT = 2 * HSTRIDE;             // per-slot totals: H1 | H2
constexpr double DIVERGE = 1e8;
constexpr long long AUTOTUNE_MIN_POINTS = 4096;
constexpr int VEC_PER_DOT = 64;    // points per thread, Arnoldi dot passes
constexpr int VEC_PER_NORM = 16;   // points per thread, Arnoldi norm pass

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
    int shape = 0;                // tile shape of the fused kernels on this level
    // per direction (0 forward, 1 conjugate transpose): per axis cm | c0 | cp
    std::vector<cd> coef_host[2];
    cx<double>* coef_d[2] = {nullptr, nullptr};
    cx<float>* coef_f[2] = {nullptr, nullptr};
    double* k2 = nullptr;
    float* k2f = nullptr;
    void* F = nullptr;            // right-hand sides on levels >= 1, by rhs
    void* E = nullptr;            // corrections on levels >= 1, by rhs
    void* Q[3] = {nullptr, nullptr, nullptr};   // GMRES(3) smoother: q0, q1, q2 by rhs
    void* SU1 = nullptr;          //   u1 by rhs
    void* SU2 = nullptr;          //   u2 by rhs
};

struct Prof {
    bool on = false;
    std::vector<hipEvent_t> pool;
    std::vector<int> cls;
    std::vector<double> bytes;
    size_t used = 0;
};

// Reduction work space and pinned mirrors.
struct Work {
    cx<double>* part = nullptr;   // [(slot * HSTRIDE + i) * bstride + b]
    double* rpart = nullptr;      // [slot * bstride + b]
    int bstride = 0;
    cx<double>* tot = nullptr;    // [slot * TOT + v]
    double* rtot = nullptr;       // [slot]
    cx<double>* tot_h = nullptr;  // pinned [item * TOT + v]
    double* rtot_h = nullptr;     // pinned [item]
    int items = 0;
};

// Captured coarse parts of the V-cycle, keyed by direction and item list.
struct GraphCache {
    std::map<std::vector<uintptr_t>, hipGraphExec_t> execs;
    hipStream_t capture = nullptr;    // private stream used only for capture
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
    int ncoarse = 0;
    cx<double>* lu[2] = {nullptr, nullptr};
    int* piv[2] = {nullptr, nullptr};
    LevelView<double>* views_d[2] = {nullptr, nullptr};   // device, one per level
    LevelView<double>* outer_d[2] = {nullptr, nullptr};   // the unshifted level-0 operator (sigma = 1)
    bool shifted0 = false;            // the cycle's level-0 shift differs from 1 (fixed-shift preconditioner)
    LevelView<float>* views_f[2] = {nullptr, nullptr};
    // level-0 work vectors, by rhs
    cx<double>* U1 = nullptr;
    cx<double>* Z = nullptr;
    cx<double>* W = nullptr;
    // GMRES basis, by rhs: V + (rhs * vstride + i) * N0
    cx<double>* V = nullptr;
    int vstride = 0;
    // FGMRES: z_i = M v_i, by rhs: Zb + (rhs * zstride + i) * N0
    cx<double>* Zb = nullptr;
    int zstride = 0;
    // GMRES(3) smoother
    bool gsmooth = false;
    int lt = 1;                       // first level of the coarse tail (levels lt..L-1 in one launch)
    mg::SmoothBufs* sb_d = nullptr;   // [rhs * L + l]
    cx<double>* gcoef = nullptr;      // [(rhs * L + l) * 8]
    double* scale_d = nullptr;     // [rhs * HSTRIDE + i]
    double* scale_h = nullptr;     // pinned
    cx<double>* coef_d = nullptr;  // [rhs * HSTRIDE + i]
    cx<double>* coef_h = nullptr;  // pinned
    Work work;
    Prof prof;
    GraphCache graphs;
};

struct mg_batch {
    std::vector<mg_ctx*> ctxs;
    Work work;
    GraphCache graphs;
};

namespace {

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

mg_status work_alloc(Work& w, int items, int bstride) {
    w.items = items;
    w.bstride = bstride;
    CKS(dalloc(&w.part, (size_t)mg::MAX_SLOTS * HSTRIDE * bstride * sizeof(cx<double>)));
    CKS(dalloc(&w.rpart, (size_t)mg::MAX_SLOTS * bstride * sizeof(double)));
    CKS(dalloc(&w.tot, (size_t)mg::MAX_SLOTS * TOT * sizeof(cx<double>)));
    CKS(dalloc(&w.rtot, (size_t)mg::MAX_SLOTS * sizeof(double)));
    CKS(halloc(&w.tot_h, (size_t)std::max(items, mg::MAX_SLOTS) * TOT * sizeof(cx<double>)));
    CKS(halloc(&w.rtot_h, (size_t)std::max(items, mg::MAX_SLOTS) * sizeof(double)));
    return MG_OK;
}

void work_free(Work& w) {
    dfree(w.part);
    dfree(w.rpart);
    dfree(w.tot);
    dfree(w.rtot);
    hfree(w.tot_h);
    hfree(w.rtot_h);
}

void graphs_free(GraphCache& g) {
    for (auto& kv : g.execs) (void)hipGraphExecDestroy(kv.second);
    g.execs.clear();
    if (g.capture) (void)hipStreamDestroy(g.capture);
    g.capture = nullptr;
}

// One solve invocation: where launches go and what they record.
struct Run {
    hipStream_t s;
    Prof* prof;
    Work* w;
    GraphCache* gc;
    int dim;
    bool mixed;
};

// bytes: algorithmic (compulsory) traffic of the launch
int prof_begin(Run& R, int cls, double bytes = 0.0) {
    if (!R.prof || !R.prof->on) return -1;
    Prof& P = *R.prof;
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
    (void)hipEventRecord(P.pool[2 * idx], R.s);
    return idx;
}
void prof_end(Run& R, int idx) {
    if (idx >= 0) (void)hipEventRecord(R.prof->pool[2 * idx + 1], R.s);
}

// One right-hand side of one problem.
struct Item {
    mg_ctx* c;
    int rhs;
};

// Level-0 inputs and outputs of one item's cycle.
struct L0 {
    const void* f;            // right-hand side (complex double)
    double fs;                // scale applied to f
    const cx<double>* u;      // incoming iterate or null (zero guess)
    cx<double>* out;          // result (written, or accumulated)
};

const void* view_ptr(const mg_ctx* c, int dir, int l) {
    return c->mixed ? (const void*)(c->views_f[dir] + l) : (const void*)(c->views_d[dir] + l);
}
size_t elem(const mg_ctx* c) { return c->mixed ? sizeof(cx<float>) : sizeof(cx<double>); }
void* lvec(const mg_ctx* c, void* base, int l, int rhs) {
    return (char*)base + (size_t)rhs * c->lv[l].N * elem(c);
}

// Launch groups of at most MAX_SLOTS items each.
template <typename F>
mg_status for_groups(const std::vector<int>& idx, F fn) {
    for (size_t g = 0; g < idx.size(); g += mg::MAX_SLOTS) {
        const size_t n = std::min<size_t>(mg::MAX_SLOTS, idx.size() - g);
        std::vector<int> sub(idx.begin() + g, idx.begin() + g + n);
        CKS(fn(sub, (int)g));
    }
    return MG_OK;
}

// Shape of a launch at depth d: the one tuned for the largest level in it.
int launch_shape(const std::vector<Item>& it, const std::vector<int>& sub, int d) {
    long long best = -1;
    int shape = 0;
    for (int k : sub) {
        const Level& V = it[k].c->lv[d];
        if (V.N > best) {
            best = V.N;
            shape = V.shape;
        }
    }
    return shape;
}

// ---------------------------------------------------------------------------
// V-cycle pieces (Sec. 3.1)
// ---------------------------------------------------------------------------

// K_A at depth d for the items that have a coarser level below d.  With norm
// (level 0 with incoming iterates) ||f - A u||^2 of item k lands in
// w->rtot_h[k] once the stream gets there.
mg_status launch_ka(Run& R, int dir, const std::vector<Item>& it, const std::vector<L0>* l0, int d,
                    bool norm) {
    std::vector<int> who;
    for (int k = 0; k < (int)it.size(); ++k)
        if (d < it[k].c->lt) who.push_back(k);
    const bool zero = !(d == 0 && l0 && (*l0)[0].u);
    return for_groups(who, [&](const std::vector<int>& sub, int gbase) -> mg_status {
        const int shape = launch_shape(it, sub, d);
        CycleArgs a{};
        a.st.n = (int)sub.size();
        int tiles = 0;
        double by = 0.0;
        const double ct = R.mixed ? 8.0 : 16.0, sk = R.mixed ? 4.0 : 8.0;
        for (int q = 0; q < a.st.n; ++q) {
            const Item& I = it[sub[q]];
            mg_ctx* c = I.c;
            CycleSlot& s = a.st.s[q];
            s.lv = view_ptr(c, dir, d);
            if (d == 0) {
                const L0& z = (*l0)[sub[q]];
                s.f = z.f;
                s.fscale = z.fs;
                s.u = z.u;
                s.u1 = z.u ? (void*)(c->U1 + (size_t)I.rhs * c->lv[0].N) : nullptr;
            } else {
                s.f = lvec(c, c->lv[d].F, d, I.rhs);
                s.fscale = 1.0;
            }
            s.c = lvec(c, c->lv[d + 1].F, d + 1, I.rhs);
            s.tile0 = tiles;
            int nt[3];
            mg::tile_counts(R.dim, shape, c->lv[d].n, nt);
            tiles += nt[0] * nt[1] * nt[2];
            by += c->lv[d].N * ((d == 0 ? 16.0 : ct) + sk) + c->lv[d + 1].N * ct;
            if (!zero) by += c->lv[0].N * 2.0 * ct;
        }
        a.st.ntiles = tiles;
        a.norm_part = (norm && !zero) ? R.w->rpart : nullptr;
        a.pstride = R.w->bstride;
        const int pi = prof_begin(R, d == 0 ? MG_K_SMOOTH_RESTRICT_FINE : MG_K_COARSE_LEVELS, by);
        CK(mg::launch_smooth_restrict(R.dim, R.mixed, d == 0, zero, shape, a, R.s));
        prof_end(R, pi);
        if (a.norm_part) {
            ReduceArgs ra{};
            ra.rpart = R.w->rpart;
            ra.rout = R.w->rtot;
            ra.bstride = R.w->bstride;
            for (int q = 0; q < a.st.n; ++q) {
                const int next = q + 1 < a.st.n ? a.st.s[q + 1].tile0 : tiles;
                ra.cnt[q] = next - a.st.s[q].tile0;
            }
            const int pr = prof_begin(R, MG_K_REDUCE);
            CK(mg::launch_reduce(ra, a.st.n, true, R.s));
            prof_end(R, pr);
            CK(hipMemcpyAsync(R.w->rtot_h + gbase, R.w->rtot, a.st.n * sizeof(double), hipMemcpyDeviceToHost,
                              R.s));
        }
        return MG_OK;
    });
}

const mg::SmoothBufs* sbuf(const mg_ctx* c, int l, int rhs);

// The coarse tail of every item (levels lt..L-1 and the coarsest solve),
// one workgroup per item: its correction lands in E_lt.
mg_status launch_tail_items(Run& R, int dir, const std::vector<Item>& it) {
    std::vector<int> all(it.size());
    for (size_t k = 0; k < it.size(); ++k) all[k] = (int)k;
    return for_groups(all, [&](const std::vector<int>& sub, int) -> mg_status {
        mg::TailArgs a{};
        a.n = (int)sub.size();
        a.gmres = it[sub[0]].c->gsmooth ? 1 : 0;
        a.brk = R.mixed ? 1e-5 : 1e-13;
        double by = 0.0;
        for (int q = 0; q < a.n; ++q) {
            const Item& I = it[sub[q]];
            mg_ctx* c = I.c;
            mg::TailSlot& s = a.s[q];
            s.lv = view_ptr(c, dir, c->lt);
            s.sb = sbuf(c, c->lt, I.rhs);
            s.nlev = c->L - c->lt;
            for (int l = c->lt; l < c->L; ++l) by += 2.0 * c->lv[l].N * (R.mixed ? 8.0 : 16.0);
        }
        const int pi = prof_begin(R, MG_K_COARSEST_SOLVE, by);
        CK(mg::launch_tail(R.dim, R.mixed, a, R.s));
        prof_end(R, pi);
        return MG_OK;
    });
}

// K_B at depth d for the items that have a coarser level below d.
mg_status launch_kb(Run& R, int dir, const std::vector<Item>& it, const std::vector<L0>* l0, int d, bool acc) {
    std::vector<int> who;
    for (int k = 0; k < (int)it.size(); ++k)
        if (d < it[k].c->lt) who.push_back(k);
    const bool zero = !(d == 0 && l0 && (*l0)[0].u);
    return for_groups(who, [&](const std::vector<int>& sub, int) -> mg_status {
        const int shape = launch_shape(it, sub, d);
        CycleArgs a{};
        a.st.n = (int)sub.size();
        int tiles = 0;
        double by = 0.0;
        const double ct = R.mixed ? 8.0 : 16.0, sk = R.mixed ? 4.0 : 8.0;
        for (int q = 0; q < a.st.n; ++q) {
            const Item& I = it[sub[q]];
            mg_ctx* c = I.c;
            CycleSlot& s = a.st.s[q];
            s.lv = view_ptr(c, dir, d);
            if (d == 0) {
                const L0& z = (*l0)[sub[q]];
                s.f = z.f;
                s.fscale = z.fs;
                s.u1 = z.u ? (void*)(c->U1 + (size_t)I.rhs * c->lv[0].N) : nullptr;
                s.out = z.out;
            } else {
                s.f = lvec(c, c->lv[d].F, d, I.rhs);
                s.fscale = 1.0;
                s.out = lvec(c, c->lv[d].E, d, I.rhs);
            }
            s.c = lvec(c, c->lv[d + 1].E, d + 1, I.rhs);
            s.tile0 = tiles;
            int nt[3];
            mg::tile_counts(R.dim, shape, c->lv[d].n, nt);
            tiles += nt[0] * nt[1] * nt[2];
            const double cf = d == 0 ? 16.0 : ct;
            by += c->lv[d].N * (cf + sk + cf) + c->lv[d + 1].N * ct;
            if (!zero) by += c->lv[0].N * ct;
            if (d == 0 && acc) by += c->lv[0].N * 16.0;
        }
        a.st.ntiles = tiles;
        const int pi = prof_begin(R, d == 0 ? MG_K_PROLONG_SMOOTH_FINE : MG_K_COARSE_LEVELS, by);
        CK(mg::launch_prolong_smooth(R.dim, R.mixed, d == 0, zero, d == 0 && acc, shape, a, R.s));
        prof_end(R, pi);
        return MG_OK;
    });
}

// ---------------------------------------------------------------------------
// GMRES(3) smoothing (Sec. 3.2.2): pre-smoothing at depth d ends in the
// restriction of its residual, post-smoothing starts from u1 + P e.
// ---------------------------------------------------------------------------
mg_status build_vec(Run& R, int dir, const std::vector<Item>& it, const std::vector<int>& sub, VecArgs& a,
                    int* cnt);
mg_status reduce_real(Run& R, int n, const int* cnt);

const mg::SmoothBufs* sbuf(const mg_ctx* c, int l, int rhs) { return c->sb_d + (size_t)rhs * c->L + l; }
cx<double>* gcoef_of(const mg_ctx* c, int l, int rhs, int phase) {
    return c->gcoef + ((size_t)rhs * c->L + l) * 8 + 4 * phase;
}

// Powers, Gram partials and coefficients of one smoothing step for the slots
// of sa (q0 given by slot.f or the q0 buffer).
mg_status smooth_coef(Run& R, int d, int phase, const std::vector<Item>& it, const std::vector<int>& sub,
                      mg::SmArgs& sa, bool q0f) {
    const bool fine = d == 0;
    const double ct = R.mixed ? 8.0 : 16.0, sk = R.mixed ? 4.0 : 8.0;
    double n = 0.0;
    for (int k : sub) n += (double)it[k].c->lv[d].N;
    const double q0b = (fine && q0f) ? 16.0 : ct;
    for (int stage = 1; stage <= 2; ++stage) {
        const double by = n * ((stage == 1 ? q0b : ct) + sk + ct);
        const int pi = prof_begin(R, fine ? MG_K_SMOOTH_POWER_FINE : MG_K_COARSE_LEVELS, by);
        CK(mg::launch_sm_power(R.dim, R.mixed, fine, stage, sa, R.s));
        prof_end(R, pi);
    }
    const int gcls = phase ? MG_K_SMOOTH_GRAM_POST_FINE : MG_K_SMOOTH_GRAM_FINE;
    int pi = prof_begin(R, fine ? gcls : MG_K_COARSE_LEVELS, n * (q0b + 2.0 * ct + sk));
    CK(mg::launch_sm_gram(R.dim, R.mixed, fine, sa, R.s));
    prof_end(R, pi);
    mg::SmCoefArgs ca{};
    ca.part = R.w->part;
    ca.pstride = HSTRIDE;
    ca.bstride = R.w->bstride;
    for (int q = 0; q < sa.st.n; ++q) {
        const Item& I = it[sub[q]];
        ca.cnt[q] = mg::vec_blocks(I.c->lv[d].N);
        ca.coef[q] = gcoef_of(I.c, d, I.rhs, phase);
    }
    pi = prof_begin(R, fine ? MG_K_REDUCE : MG_K_COARSE_LEVELS);
    CK(mg::launch_sm_coef(R.mixed, ca, sa.st.n, R.s));
    prof_end(R, pi);
    return MG_OK;
}

mg_status build_sm(Run& R, int dir, int d, const std::vector<Item>& it, const std::vector<int>& sub,
                   mg::SmArgs& sa) {
    sa.st.n = (int)sub.size();
    int blocks = 0;
    for (int q = 0; q < sa.st.n; ++q) {
        const Item& I = it[sub[q]];
        mg::SmSlot& s = sa.st.s[q];
        s.lv = view_ptr(I.c, dir, d);
        s.sb = sbuf(I.c, d, I.rhs);
        s.block0 = blocks;
        const int nb = mg::vec_blocks(I.c->lv[d].N);
        if (nb > R.w->bstride) return MG_E_STATE;
        blocks += nb;
    }
    sa.st.nblocks = blocks;
    sa.part = R.w->part;
    sa.pstride = HSTRIDE;
    sa.bstride = R.w->bstride;
    return MG_OK;
}

// 2D: the fused tile passes of mg_smooth2d.hip.  Slots carry f (q0 source;
// null: the q0 buffer), u (incoming iterate, NZ), c (coarse rhs out for the
// pre-smoothing step, coarse correction in for the post-smoothing step), out.
mg_status coef_from_tiles(Run& R, int d, int phase, const std::vector<Item>& it, const std::vector<int>& sub,
                          const CycleArgs& a) {
    mg::SmCoefArgs ca{};
    ca.part = R.w->part;
    ca.pstride = HSTRIDE;
    ca.bstride = R.w->bstride;
    for (int q = 0; q < a.st.n; ++q) {
        const Item& I = it[sub[q]];
        const int next = q + 1 < a.st.n ? a.st.s[q + 1].tile0 : a.st.ntiles;
        ca.cnt[q] = next - a.st.s[q].tile0;
        ca.coef[q] = gcoef_of(I.c, d, I.rhs, phase);
    }
    const int pi = prof_begin(R, d == 0 ? MG_K_REDUCE : MG_K_COARSE_LEVELS);
    CK(mg::launch_sm_coef(R.mixed, ca, a.st.n, R.s));
    prof_end(R, pi);
    return MG_OK;
}

mg_status pre_fused_2d(Run& R, int dir, const std::vector<Item>& it, const std::vector<L0>* l0, int d, bool nz,
                       const std::vector<int>& sub) {
    const int shape = launch_shape(it, sub, d);
    const double ct = R.mixed ? 8.0 : 16.0, sk = R.mixed ? 4.0 : 8.0;
    CycleArgs a{};
    a.st.n = (int)sub.size();
    int tiles = 0;
    double bg = 0.0, ba = 0.0;
    for (int q = 0; q < a.st.n; ++q) {
        const Item& I = it[sub[q]];
        mg_ctx* c = I.c;
        CycleSlot& s = a.st.s[q];
        s.lv = view_ptr(c, dir, d);
        if (nz) {
            s.f = nullptr;
            s.fscale = 1.0;
            s.u = (*l0)[sub[q]].u;
        } else if (d == 0) {
            s.f = (*l0)[sub[q]].f;
            s.fscale = (*l0)[sub[q]].fs;
        } else {
            s.f = lvec(c, c->lv[d].F, d, I.rhs);
            s.fscale = 1.0;
        }
        s.c = lvec(c, c->lv[d + 1].F, d + 1, I.rhs);
        s.sb = sbuf(c, d, I.rhs);
        s.tile0 = tiles;
        int nt[3];
        mg::march_counts(shape, c->lv[d].n, nt);
        tiles += nt[0] * nt[1];
        const double q0b = (d == 0 && !nz) ? 16.0 : ct;
        bg += c->lv[d].N * (q0b + sk);
        ba += c->lv[d].N * (q0b + sk + ct + (nz ? 16.0 : 0.0)) + c->lv[d + 1].N * ct;
    }
    a.st.ntiles = tiles;
    int pi = prof_begin(R, d == 0 ? MG_K_SMOOTH_GRAM_FINE : MG_K_COARSE_LEVELS, bg);
    CK(mg::launch_sm2_gram(R.mixed, d == 0, false, shape, a, R.w->part, HSTRIDE, R.w->bstride, R.s));
    prof_end(R, pi);
    CKS(coef_from_tiles(R, d, 0, it, sub, a));
    pi = prof_begin(R, d == 0 ? MG_K_SMOOTH_RESTRICT_FINE : MG_K_COARSE_LEVELS, ba);
    CK(mg::launch_sm2_apply_restrict(R.mixed, d == 0, nz, shape, a, R.s));
    prof_end(R, pi);
    return MG_OK;
}

mg_status post_fused_2d(Run& R, int dir, const std::vector<Item>& it, const std::vector<L0>* l0, int d, bool acc,
                        const std::vector<int>& sub) {
    const int shape = launch_shape(it, sub, d);
    const double ct = R.mixed ? 8.0 : 16.0, sk = R.mixed ? 4.0 : 8.0;
    CycleArgs a{};
    a.st.n = (int)sub.size();
    int tiles = 0;
    double bg = 0.0, ba = 0.0;
    for (int q = 0; q < a.st.n; ++q) {
        const Item& I = it[sub[q]];
        mg_ctx* c = I.c;
        CycleSlot& s = a.st.s[q];
        s.lv = view_ptr(c, dir, d);
        if (d == 0) {
            s.f = (*l0)[sub[q]].f;
            s.fscale = (*l0)[sub[q]].fs;
            s.out = (*l0)[sub[q]].out;
        } else {
            s.f = lvec(c, c->lv[d].F, d, I.rhs);
            s.fscale = 1.0;
            s.out = lvec(c, c->lv[d].E, d, I.rhs);
        }
        s.c = lvec(c, c->lv[d + 1].E, d + 1, I.rhs);
        s.sb = sbuf(c, d, I.rhs);
        s.tile0 = tiles;
        int nt[3];
        mg::march_counts(shape, c->lv[d].n, nt);
        tiles += nt[0] * nt[1];
        const double fb = d == 0 ? 16.0 : ct;
        bg += c->lv[d].N * (ct + fb + sk) + c->lv[d + 1].N * ct;
        ba += c->lv[d].N * (ct + fb + sk + fb + (d == 0 && acc ? 16.0 : 0.0)) + c->lv[d + 1].N * ct;
    }
    a.st.ntiles = tiles;
    int pi = prof_begin(R, d == 0 ? MG_K_SMOOTH_GRAM_POST_FINE : MG_K_COARSE_LEVELS, bg);
    CK(mg::launch_sm2_gram(R.mixed, d == 0, true, shape, a, R.w->part, HSTRIDE, R.w->bstride, R.s));
    prof_end(R, pi);
    CKS(coef_from_tiles(R, d, 1, it, sub, a));
    pi = prof_begin(R, d == 0 ? MG_K_PROLONG_SMOOTH_FINE : MG_K_COARSE_LEVELS, ba);
    CK(mg::launch_sm2_apply_out(R.mixed, d == 0, d == 0 && acc, shape, a, R.s));
    prof_end(R, pi);
    return MG_OK;
}

// Pre-smoothing at depth d and restriction of its residual to depth d + 1.
// Level 0 with incoming iterates (FP64 only): q0 = f - A u by the FP64
// residual kernel, whose ||q0||^2 of item k lands in w->rtot_h[k] when norm.
mg_status launch_pre_g(Run& R, int dir, const std::vector<Item>& it, const std::vector<L0>* l0, int d, bool norm) {
    std::vector<int> who;
    for (int k = 0; k < (int)it.size(); ++k)
        if (d < it[k].c->lt) who.push_back(k);
    const bool nz = d == 0 && l0 && (*l0)[0].u;
    if (nz && R.mixed) return MG_E_STATE;
    return for_groups(who, [&](const std::vector<int>& sub, int gbase) -> mg_status {
        if (nz) {
            VecArgs a{};
            int cnt[mg::MAX_SLOTS];
            CKS(build_vec(R, dir, it, sub, a, cnt));
            double by = 0.0;
            for (int q = 0; q < a.st.n; ++q) {
                const Item& I = it[sub[q]];
                const L0& z = (*l0)[sub[q]];
                if (z.fs != 1.0) return MG_E_STATE;
                a.st.s[q].x = z.u;
                a.st.s[q].f = (const cx<double>*)z.f;
                a.st.s[q].y = (cx<double>*)lvec(I.c, I.c->lv[0].Q[0], 0, I.rhs);
                by += I.c->lv[0].N * 56.0;
            }
            if (!norm) a.rpart = nullptr;
            const int pi = prof_begin(R, MG_K_RESIDUAL, by);
            CK(mg::launch_residual(R.dim, a, R.s));
            prof_end(R, pi);
            if (norm) {
                CKS(reduce_real(R, a.st.n, cnt));
                CK(hipMemcpyAsync(R.w->rtot_h + gbase, R.w->rtot, a.st.n * sizeof(double), hipMemcpyDeviceToHost,
                                  R.s));
            }
        }
        if (R.dim == 2) return pre_fused_2d(R, dir, it, l0, d, nz, sub);
        mg::SmArgs sa{};
        CKS(build_sm(R, dir, d, it, sub, sa));
        for (int q = 0; q < sa.st.n; ++q) {
            const Item& I = it[sub[q]];
            mg::SmSlot& s = sa.st.s[q];
            if (nz) {
                s.f = nullptr;
                s.fscale = 1.0;
            } else if (d == 0) {
                s.f = (*l0)[sub[q]].f;
                s.fscale = (*l0)[sub[q]].fs;
            } else {
                s.f = lvec(I.c, I.c->lv[d].F, d, I.rhs);
                s.fscale = 1.0;
            }
        }
        CKS(smooth_coef(R, d, 0, it, sub, sa, !nz));
        const int shape = launch_shape(it, sub, d);
        CycleArgs a{};
        a.st.n = sa.st.n;
        int tiles = 0;
        double by = 0.0;
        const double ct = R.mixed ? 8.0 : 16.0, sk = R.mixed ? 4.0 : 8.0;
        for (int q = 0; q < a.st.n; ++q) {
            const Item& I = it[sub[q]];
            mg_ctx* c = I.c;
            CycleSlot& s = a.st.s[q];
            s.lv = sa.st.s[q].lv;
            s.f = sa.st.s[q].f;
            s.fscale = sa.st.s[q].fscale;
            s.u = nz ? (const void*)(*l0)[sub[q]].u : nullptr;
            s.c = lvec(c, c->lv[d + 1].F, d + 1, I.rhs);
            s.sb = sbuf(c, d, I.rhs);
            s.tile0 = tiles;
            int nt[3];
            mg::tile_counts(R.dim, shape, c->lv[d].n, nt);
            tiles += nt[0] * nt[1] * nt[2];
            const double q0b = (d == 0 && !nz) ? 16.0 : ct;
            by += c->lv[d].N * (q0b + 3.0 * ct + sk + (nz ? 16.0 : 0.0)) + c->lv[d + 1].N * ct;
        }
        a.st.ntiles = tiles;
        const int pi = prof_begin(R, d == 0 ? MG_K_SMOOTH_RESTRICT_FINE : MG_K_COARSE_LEVELS, by);
        CK(mg::launch_sm_apply_restrict(R.dim, R.mixed, d == 0, nz, shape, a, R.s));
        prof_end(R, pi);
        return MG_OK;
    });
}

// Coarse-grid correction and post-smoothing at depth d.
mg_status launch_post_g(Run& R, int dir, const std::vector<Item>& it, const std::vector<L0>* l0, int d, bool acc) {
    std::vector<int> who;
    for (int k = 0; k < (int)it.size(); ++k)
        if (d < it[k].c->lt) who.push_back(k);
    return for_groups(who, [&](const std::vector<int>& sub, int) -> mg_status {
        if (R.dim == 2) return post_fused_2d(R, dir, it, l0, d, acc, sub);
        const int shape = launch_shape(it, sub, d);
        const double ct = R.mixed ? 8.0 : 16.0, sk = R.mixed ? 4.0 : 8.0;
        CycleArgs a{};
        a.st.n = (int)sub.size();
        int tiles = 0;
        double by = 0.0;
        for (int q = 0; q < a.st.n; ++q) {
            const Item& I = it[sub[q]];
            mg_ctx* c = I.c;
            CycleSlot& s = a.st.s[q];
            s.lv = view_ptr(c, dir, d);
            if (d == 0) {
                s.f = (*l0)[sub[q]].f;
                s.fscale = (*l0)[sub[q]].fs;
            } else {
                s.f = lvec(c, c->lv[d].F, d, I.rhs);
                s.fscale = 1.0;
            }
            s.c = lvec(c, c->lv[d + 1].E, d + 1, I.rhs);
            s.sb = sbuf(c, d, I.rhs);
            s.tile0 = tiles;
            int nt[3];
            mg::tile_counts(R.dim, shape, c->lv[d].n, nt);
            tiles += nt[0] * nt[1] * nt[2];
            by += c->lv[d].N * (ct + (d == 0 ? 16.0 : ct) + sk + 2.0 * ct) + c->lv[d + 1].N * ct;
        }
        a.st.ntiles = tiles;
        int pi = prof_begin(R, d == 0 ? MG_K_PROLONG_SMOOTH_FINE : MG_K_COARSE_LEVELS, by);
        CK(mg::launch_sm_prolong_resid(R.dim, R.mixed, d == 0, shape, a, R.s));
        prof_end(R, pi);
        mg::SmArgs sa{};
        CKS(build_sm(R, dir, d, it, sub, sa));
        CKS(smooth_coef(R, d, 1, it, sub, sa, false));
        by = 0.0;
        for (int q = 0; q < sa.st.n; ++q) {
            const Item& I = it[sub[q]];
            mg_ctx* c = I.c;
            sa.st.s[q].out = d == 0 ? (void*)(*l0)[sub[q]].out : lvec(c, c->lv[d].E, d, I.rhs);
            by += c->lv[d].N * (4.0 * ct + (d == 0 ? 16.0 : ct) + (d == 0 && acc ? 16.0 : 0.0));
        }
        pi = prof_begin(R, d == 0 ? MG_K_PROLONG_SMOOTH_FINE : MG_K_COARSE_LEVELS, by);
        CK(mg::launch_sm_apply_out(R.mixed, d == 0, d == 0 && acc, sa, R.s));
        prof_end(R, pi);
        return MG_OK;
    });
}

// The descending / ascending halves of one level's cycle work.
mg_status cycle_down(Run& R, int dir, const std::vector<Item>& it, const std::vector<L0>* l0, int d, bool norm) {
    return it[0].c->gsmooth ? launch_pre_g(R, dir, it, l0, d, norm) : launch_ka(R, dir, it, l0, d, norm);
}
mg_status cycle_up(Run& R, int dir, const std::vector<Item>& it, const std::vector<L0>* l0, int d, bool acc) {
    return it[0].c->gsmooth ? launch_post_g(R, dir, it, l0, d, acc) : launch_kb(R, dir, it, l0, d, acc);
}

// Levels >= 1 and the coarsest solve of one cycle: captured once per
// (direction, item list) as a HIP graph and replayed; every pointer in it is
// fixed per item (F_l and E_l by rhs).
mg_status coarse_part(Run& R, int dir, const std::vector<Item>& it) {
    int maxT = 0;
    for (const Item& I : it) maxT = std::max(maxT, I.c->lt);
    auto record = [&](Run& Q) -> mg_status {
        for (int d = 1; d < maxT; ++d) CKS(cycle_down(Q, dir, it, nullptr, d, false));
        CKS(launch_tail_items(Q, dir, it));
        for (int d = maxT - 1; d >= 1; --d) CKS(cycle_up(Q, dir, it, nullptr, d, false));
        return MG_OK;
    };
    if (!R.gc) return record(R);
    std::vector<uintptr_t> key;
    key.push_back((uintptr_t)dir);
    for (const Item& I : it) {
        key.push_back((uintptr_t)I.c);
        key.push_back((uintptr_t)I.rhs);
    }
    auto f = R.gc->execs.find(key);
    if (f == R.gc->execs.end()) {
        if (!R.gc->capture) CK(hipStreamCreateWithFlags(&R.gc->capture, hipStreamNonBlocking));
        Run Q = R;
        Q.s = R.gc->capture;
        Q.prof = nullptr;
        CK(hipStreamBeginCapture(Q.s, hipStreamCaptureModeThreadLocal));
        const mg_status st = record(Q);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(Q.s, &g);
        if (st != MG_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        CK(e);
        hipGraphExec_t ex = nullptr;
        const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        CK(ei);
        f = R.gc->execs.emplace(key, ex).first;
    }
    double by = 0.0;   // algorithmic bytes of every level >= 1 kernel
    if (R.prof && R.prof->on) {
        const double ct = R.mixed ? 8.0 : 16.0, sk = R.mixed ? 4.0 : 8.0;
        for (const Item& I : it)
            for (int l = 1; l < I.c->lt; ++l) {
                if (I.c->gsmooth && I.c->dim == 2)   // fused Gram and apply passes of both steps
                    by += I.c->lv[l].N * (8 * ct + 4 * sk) + 3 * I.c->lv[l + 1].N * ct;
                else if (I.c->gsmooth)   // powers, Gram, apply passes of both smoothing steps
                    by += I.c->lv[l].N * (27 * ct + 8 * sk) + 2 * I.c->lv[l + 1].N * ct;
                else
                    by += I.c->lv[l].N * (ct + sk) + I.c->lv[l + 1].N * ct +
                          I.c->lv[l].N * (3 * ct + sk) + I.c->lv[l + 1].N * ct;
            }
    }
    const int pi = prof_begin(R, MG_K_COARSE_LEVELS, by);
    CK(hipGraphLaunch(f->second, R.s));
    prof_end(R, pi);
    return MG_OK;
}

// One V(1,1) cycle for the items.  With norms (and incoming iterates),
// ||f - A u||^2 of item k lands in w->rtot_h[k] once the stream gets there.
mg_status vcycle(Run& R, int dir, const std::vector<Item>& it, const std::vector<L0>& l0, bool acc,
                 bool norms) {
    if (R.mixed && l0[0].u) return MG_E_STATE;
    CKS(cycle_down(R, dir, it, &l0, 0, norms));
    CKS(coarse_part(R, dir, it));
    CKS(cycle_up(R, dir, it, &l0, 0, acc));
    return MG_OK;
}

// ---------------------------------------------------------------------------
// Vector kernels over items
// ---------------------------------------------------------------------------
mg_status build_vec(Run& R, int dir, const std::vector<Item>& it, const std::vector<int>& sub,
                    VecArgs& a, int* cnt) {
    a.st.n = (int)sub.size();
    int blocks = 0;
    for (int q = 0; q < a.st.n; ++q) {
        const Item& I = it[sub[q]];
        VecSlot& s = a.st.s[q];
        s.lv = I.c->outer_d[dir];
        s.block0 = blocks;
        const int nb = mg::vec_blocks(I.c->lv[0].N);
        if (nb > R.w->bstride) return MG_E_STATE;
        cnt[q] = nb;
        blocks += nb;
    }
    a.st.nblocks = blocks;
    a.part = R.w->part;
    a.rpart = R.w->rpart;
    a.pstride = HSTRIDE;
    a.bstride = R.w->bstride;
    return MG_OK;
}

mg_status reduce_real(Run& R, int n, const int* cnt) {
    ReduceArgs ra{};
    ra.rpart = R.w->rpart;
    ra.rout = R.w->rtot;
    ra.bstride = R.w->bstride;
    for (int q = 0; q < n; ++q) ra.cnt[q] = cnt[q];
    const int pi = prof_begin(R, MG_K_REDUCE);
    CK(mg::launch_reduce(ra, n, true, R.s));
    prof_end(R, pi);
    return MG_OK;
}

mg_status reduce_complex(Run& R, int n, const int* cnt, int nvals, int toff) {
    ReduceArgs ra{};
    ra.part = R.w->part;
    ra.out = R.w->tot + toff;
    ra.nvals = nvals;
    ra.pstride = HSTRIDE;
    ra.bstride = R.w->bstride;
    ra.ostride = TOT;
    for (int q = 0; q < n; ++q) ra.cnt[q] = cnt[q];
    const int pi = prof_begin(R, MG_K_REDUCE);
    CK(mg::launch_reduce(ra, n, false, R.s));
    prof_end(R, pi);
    return MG_OK;
}

// ||x_k||^2 of every item (x[k] a full-length level-0 vector), synchronising.
mg_status norms(Run& R, const std::vector<Item>& it, const std::vector<const cx<double>*>& x,
                std::vector<double>& out) {
    std::vector<int> all(it.size());
    for (size_t k = 0; k < it.size(); ++k) all[k] = (int)k;
    CKS(for_groups(all, [&](const std::vector<int>& sub, int gbase) -> mg_status {
        VecArgs a{};
        int cnt[mg::MAX_SLOTS];
        CKS(build_vec(R, 0, it, sub, a, cnt));
        for (int q = 0; q < a.st.n; ++q) a.st.s[q].x = x[sub[q]];
        CK(mg::launch_norm(a, R.s));
        CKS(reduce_real(R, a.st.n, cnt));
        CK(hipMemcpyAsync(R.w->rtot_h + gbase, R.w->rtot, a.st.n * sizeof(double), hipMemcpyDeviceToHost, R.s));
        return MG_OK;
    }));
    CK(hipStreamSynchronize(R.s));
    out.resize(it.size());
    for (size_t k = 0; k < it.size(); ++k) out[k] = R.w->rtot_h[k];
    return MG_OK;
}

// y_k = f_k - A x_k (f_k null: y_k = A x_k) on level 0 for the items in
// `who`; with nrm, ||y_k||^2 into (*nrm)[k] (synchronising).
mg_status residual(Run& R, int dir, const std::vector<Item>& it, const std::vector<int>& who,
                   const std::vector<const cx<double>*>& x, const std::vector<const cx<double>*>& f,
                   const std::vector<cx<double>*>& y, std::vector<double>* nrm) {
    CKS(for_groups(who, [&](const std::vector<int>& sub, int gbase) -> mg_status {
        VecArgs a{};
        int cnt[mg::MAX_SLOTS];
        CKS(build_vec(R, dir, it, sub, a, cnt));
        double by = 0.0;
        for (int q = 0; q < a.st.n; ++q) {
            a.st.s[q].x = x[sub[q]];
            a.st.s[q].f = f[sub[q]];
            a.st.s[q].y = y[sub[q]];
            by += it[sub[q]].c->lv[0].N * (40.0 + (f[sub[q]] ? 16.0 : 0.0));
        }
        if (!nrm) a.rpart = nullptr;
        const int pi = prof_begin(R, MG_K_RESIDUAL, by);
        CK(mg::launch_residual(R.dim, a, R.s));
        prof_end(R, pi);
        if (nrm) {
            CKS(reduce_real(R, a.st.n, cnt));
            CK(hipMemcpyAsync(R.w->rtot_h + gbase, R.w->rtot, a.st.n * sizeof(double), hipMemcpyDeviceToHost,
                              R.s));
        }
        return MG_OK;
    }));
    if (nrm) {
        CK(hipStreamSynchronize(R.s));
        nrm->assign(it.size(), 0.0);
        for (size_t g = 0; g < who.size(); ++g) (*nrm)[who[g]] = R.w->rtot_h[g];
    }
    return MG_OK;
}

mg_status ensure_basis(mg_ctx* c, int restart, bool flexible) {
    if (!c->V || c->vstride < restart + 1) {
        dfree(c->V);
        c->vstride = 0;
        const size_t bytes = (size_t)c->nrhs * (restart + 1) * c->lv[0].N * sizeof(cx<double>);
        CKS(dalloc(&c->V, bytes));
        c->vstride = restart + 1;
    }
    if (flexible && (!c->Zb || c->zstride < restart)) {
        dfree(c->Zb);
        c->zstride = 0;
        const size_t bytes = (size_t)c->nrhs * restart * c->lv[0].N * sizeof(cx<double>);
        CKS(dalloc(&c->Zb, bytes));
        c->zstride = restart;
    }
    return MG_OK;
}

// ---------------------------------------------------------------------------
// Standalone iteration (Sec. 4.1, LVL-MG): repeated cycles; the residual of
// the incoming iterate is formed inside the first fused kernel of each cycle
// (FP64) or by the FP64 residual of the refinement step (mixed).
// ---------------------------------------------------------------------------
mg_status solve_standalone(Run& R, int dir, const std::vector<Item>& it, const std::vector<cx<double>*>& U,
                           const std::vector<const cx<double>*>& F, double rtol, int maxit, int* iters,
                           double* hist) {
    const int n = (int)it.size();
    std::vector<double> nf;
    CKS(norms(R, it, F, nf));
    std::vector<int> state(n, 0);   // 0 running, 1 converged, 2 maxit, 3 diverged
    std::vector<int> its(n, 0);
    std::vector<int> active;
    for (int k = 0; k < n; ++k) {
        if (nf[k] == 0.0) {   // f = 0: the solution is 0
            CK(mg::launch_fill_zero(U[k], it[k].c->lv[0].N * sizeof(cx<double>), R.s));
            state[k] = 1;
            if (hist) hist[(size_t)k * (maxit + 1)] = 0.0;
        } else {
            active.push_back(k);
        }
    }
    for (int cyc = 0; cyc < maxit && !active.empty(); ++cyc) {
        std::vector<Item> sub;
        std::vector<L0> l0;
        for (int k : active) {
            sub.push_back(it[k]);
            mg_ctx* c = it[k].c;
            if (!R.mixed && !c->shifted0)
                l0.push_back(L0{F[k], 1.0, U[k], U[k]});
            else
                l0.push_back(L0{c->W + (size_t)it[k].rhs * c->lv[0].N, 1.0, nullptr, U[k]});
        }
        std::vector<double> rho(sub.size(), 0.0);
        if (!R.mixed && !it[0].c->shifted0) {
            CKS(vcycle(R, dir, sub, l0, false, true));
            CK(hipStreamSynchronize(R.s));
            for (size_t q = 0; q < sub.size(); ++q) rho[q] = R.w->rtot_h[q];
        } else {
            // iterative refinement form: r = f - A u (FP64), u += M r
            std::vector<int> who(sub.size());
            std::vector<const cx<double>*> xs, fs;
            std::vector<cx<double>*> ys;
            for (size_t q = 0; q < sub.size(); ++q) {
                who[q] = (int)q;
                xs.push_back(U[active[q]]);
                fs.push_back(F[active[q]]);
                ys.push_back((cx<double>*)l0[q].f);
            }
            std::vector<double> nr;
            CKS(residual(R, dir, sub, who, xs, fs, ys, &nr));
            rho = nr;
            CKS(vcycle(R, dir, sub, l0, true, false));
        }
        std::vector<int> next;
        for (size_t q = 0; q < sub.size(); ++q) {
            const int k = active[q];
            const double ratio = std::sqrt(rho[q]) / std::sqrt(nf[k]);
            if (hist) hist[(size_t)k * (maxit + 1) + cyc] = ratio;
            its[k] = cyc;
            if (ratio <= rtol) {
                state[k] = 1;
            } else if (!std::isfinite(ratio) || ratio > DIVERGE) {
                state[k] = 3;
            } else {
                its[k] = cyc + 1;
                next.push_back(k);
            }
        }
        active.swap(next);
    }
    CK(hipStreamSynchronize(R.s));
    mg_status ret = MG_OK;
    for (int k = 0; k < n; ++k) {
        if (state[k] == 0) state[k] = 2;
        if (iters) iters[k] = its[k];
        if (state[k] == 3) ret = MG_E_DIVERGED;
        else if (state[k] == 2 && ret == MG_OK) ret = MG_NOT_CONVERGED;
    }
    return ret;
}

// ---------------------------------------------------------------------------
// Restarted right-preconditioned GMRES(m) (Sec. 4.1: one V(1,1) cycle from a
// zero guess per outer step).  Arnoldi by classical Gram-Schmidt with one
// re-orthogonalisation pass; Hessenberg least squares by complex Givens
// rotations on the host; x += M (V y) at the end of each restart cycle (the
// cycle is a fixed linear map).  Flexible GMRES (Sec. 3.2.2, for the
// nonlinear GMRES(3)-smoothed cycle) keeps z_j = M v_j and adds Z y.
// ---------------------------------------------------------------------------
struct GmresState {
    int j = 0;                  // basis vectors V_0..V_j exist
    int its = 0;
    int state = 0;              // 0 arnoldi, 1 converged, 2 maxit, 3 diverged
    double nf = 0.0;
    std::vector<cd> H;          // (m+1) x m, column-major
    std::vector<double> cs;
    std::vector<cd> sn;
    std::vector<cd> g;
};

cx<double>* basis(const Item& I, int i) {
    mg_ctx* c = I.c;
    return c->V + ((size_t)I.rhs * c->vstride + i) * c->lv[0].N;
}
cx<double>* zbasis(const Item& I, int i) {
    mg_ctx* c = I.c;
    return c->Zb + ((size_t)I.rhs * c->zstride + i) * c->lv[0].N;
}

mg_status solve_gmres(Run& R, int dir, const std::vector<Item>& it, const std::vector<cx<double>*>& X,
                      const std::vector<const cx<double>*>& F, double rtol, int maxit, int m, bool flexible,
                      int* iters, double* hist) {
    const int n = (int)it.size();
    for (const Item& I : it) CKS(ensure_basis(I.c, m, flexible));
    std::vector<GmresState> gs(n);
    for (int k = 0; k < n; ++k) {
        gs[k].H.assign((size_t)(m + 1) * m, 0.0);
        gs[k].cs.assign(m, 0.0);
        gs[k].sn.assign(m, 0.0);
        gs[k].g.assign(m + 1, 0.0);
    }
    std::vector<double> nf;
    CKS(norms(R, it, F, nf));
    std::vector<int> hist_len(n, 0);
    auto push_hist = [&](int k, double v) {
        if (hist && hist_len[k] <= maxit) hist[(size_t)k * (maxit + 1) + hist_len[k]] = v;
        hist_len[k]++;
    };
    auto scale_h = [&](int k, int i) -> double& { return it[k].c->scale_h[(size_t)it[k].rhs * HSTRIDE + i]; };

    // (Re)start: r = f - A x into V_0, beta = ||r||; decide per item.
    auto restart = [&](const std::vector<int>& who) -> mg_status {
        std::vector<const cx<double>*> xs(n), fs(n);
        std::vector<cx<double>*> ys(n);
        for (int k : who) {
            xs[k] = X[k];
            fs[k] = F[k];
            ys[k] = basis(it[k], 0);
        }
        std::vector<double> beta2;
        CKS(residual(R, dir, it, who, xs, fs, ys, &beta2));
        for (int k : who) {
            GmresState& G = gs[k];
            const double beta = std::sqrt(beta2[k]);
            const double ratio = beta / G.nf;
            if (hist_len[k] == 0) push_hist(k, ratio);
            if (ratio <= rtol) {
                G.state = 1;
            } else if (!std::isfinite(ratio)) {
                G.state = 3;
            } else if (G.its >= maxit) {
                G.state = 2;
            } else {
                G.j = 0;
                std::fill(G.g.begin(), G.g.end(), cd(0.0));
                G.g[0] = beta;
                scale_h(k, 0) = 1.0 / beta;
            }
        }
        return MG_OK;
    };

    std::vector<int> who;
    for (int k = 0; k < n; ++k) {
        gs[k].nf = std::sqrt(nf[k]);
        if (nf[k] == 0.0) {
            CK(mg::launch_fill_zero(X[k], it[k].c->lv[0].N * sizeof(cx<double>), R.s));
            gs[k].state = 1;
            push_hist(k, 0.0);
        } else {
            who.push_back(k);
        }
    }
    CKS(restart(who));

    std::vector<mg_ctx*> ctxs;
    for (const Item& I : it)
        if (std::find(ctxs.begin(), ctxs.end(), I.c) == ctxs.end()) ctxs.push_back(I.c);

    for (;;) {
        std::vector<int> act;
        int jmax = 0;
        for (int k = 0; k < n; ++k)
            if (gs[k].state == 0) {
                act.push_back(k);
                jmax = std::max(jmax, gs[k].j + 1);
            }
        if (act.empty()) break;
        // scales of every basis to the device
        for (mg_ctx* c : ctxs)
            CK(hipMemcpyAsync(c->scale_d, c->scale_h, (size_t)c->nrhs * HSTRIDE * sizeof(double),
                              hipMemcpyHostToDevice, R.s));
        // z = M v_j for every active item
        std::vector<Item> sub;
        std::vector<L0> l0;
        for (int k : act) {
            sub.push_back(it[k]);
            mg_ctx* c = it[k].c;
            l0.push_back(L0{basis(it[k], gs[k].j), scale_h(k, gs[k].j), nullptr,
                            flexible ? zbasis(it[k], gs[k].j) : c->Z + (size_t)it[k].rhs * c->lv[0].N});
        }
        CKS(vcycle(R, dir, sub, l0, false, false));
        std::vector<int> local(act.size());
        for (size_t q = 0; q < act.size(); ++q) local[q] = (int)q;
        CKS(for_groups(local, [&](const std::vector<int>& g, int gbase) -> mg_status {
            VecArgs a{};
            int cnt[mg::MAX_SLOTS];
            CKS(build_vec(R, dir, sub, g, a, cnt));
            double nvsum = 0.0, vb = 0.0;
            for (int q = 0; q < a.st.n; ++q) {
                const int k = act[g[q]];
                mg_ctx* c = it[k].c;
                VecSlot& s = a.st.s[q];
                s.x = flexible ? zbasis(it[k], gs[k].j) : c->Z + (size_t)it[k].rhs * c->lv[0].N;
                s.y = c->W + (size_t)it[k].rhs * c->lv[0].N;
                s.V = basis(it[k], 0);
                s.scale = c->scale_d + (size_t)it[k].rhs * HSTRIDE;
                s.j = gs[k].j;
                s.hin = R.w->tot + (size_t)q * TOT;
                nvsum += 16.0 * c->lv[0].N * (gs[k].j + 1);
                vb += 16.0 * c->lv[0].N;
            }
            // Workgroups per pass: the two dot passes hold 2 (j+1) complex
            // values per thread and run at 1-2 waves per SIMD, so a round or
            // two of 64-point-per-thread workgroups fills the chip for the
            // 8-rhs batch; the lighter norm pass wants more, smaller ones.
            // The split depends on N only, so a batched solve reduces in the
            // same order as a single one.
            auto split = [&](int per, bool mv) -> mg_status {
                int blocks = 0;
                for (int q = 0; q < a.st.n; ++q) {
                    const Level& l0 = it[act[g[q]]].c->lv[0];
                    cnt[q] = mv ? mg::mv_blocks(R.dim, l0.n, per) : mg::vec_blocks(l0.N, per);
                    if (cnt[q] > R.w->bstride) return MG_E_STATE;
                    a.st.s[q].block0 = blocks;
                    blocks += cnt[q];
                }
                a.st.nblocks = blocks;
                return MG_OK;
            };
            // pass 1: w = A z, h1 = V^H w; reads z, k^2, V_0..V_j, writes w
            CKS(split(VEC_PER_DOT, true));
            int pi = prof_begin(R, MG_K_MATVEC_DOT, nvsum + 2.0 * vb + 0.5 * vb);
            CK(mg::launch_matvec_dot(R.dim, jmax, a, R.s));
            prof_end(R, pi);
            CKS(reduce_complex(R, a.st.n, cnt, jmax, 0));
            // pass 2: w -= V h1, h2 = V^H w
            CKS(split(VEC_PER_DOT, false));
            pi = prof_begin(R, MG_K_UPDATE_DOT, nvsum + 2.0 * vb);
            CK(mg::launch_update_dot(jmax, a, R.s));
            prof_end(R, pi);
            CKS(reduce_complex(R, a.st.n, cnt, jmax, HSTRIDE));
            // pass 3: V_{j+1} = w - V h2, ||V_{j+1}||^2
            CKS(split(VEC_PER_NORM, false));
            for (int q = 0; q < a.st.n; ++q) a.st.s[q].hin = R.w->tot + (size_t)q * TOT + HSTRIDE;
            pi = prof_begin(R, MG_K_UPDATE_NORM, nvsum + 2.0 * vb);
            CK(mg::launch_update_norm(jmax, a, R.s));
            prof_end(R, pi);
            CKS(reduce_real(R, a.st.n, cnt));
            CK(hipMemcpyAsync(R.w->tot_h + (size_t)gbase * TOT, R.w->tot, (size_t)a.st.n * TOT * sizeof(cx<double>),
                              hipMemcpyDeviceToHost, R.s));
            CK(hipMemcpyAsync(R.w->rtot_h + gbase, R.w->rtot, a.st.n * sizeof(double), hipMemcpyDeviceToHost,
                              R.s));
            return MG_OK;
        }));
        CK(hipStreamSynchronize(R.s));

        std::vector<int> fin;
        for (size_t q = 0; q < act.size(); ++q) {
            const int k = act[q];
            GmresState& G = gs[k];
            const cx<double>* T = R.w->tot_h + q * TOT;
            const int j = G.j;
            cd* col = &G.H[(size_t)j * (m + 1)];
            for (int i = 0; i <= j; ++i) col[i] = cd(T[i].r, T[i].i) + cd(T[HSTRIDE + i].r, T[HSTRIDE + i].i);
            const double hn = std::sqrt(std::max(0.0, R.w->rtot_h[q]));
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
            push_hist(k, est);
            if (!std::isfinite(est)) {
                G.state = 3;
                continue;
            }
            if (hn != 0.0) scale_h(k, j + 1) = 1.0 / hn;
            if (est <= rtol || G.its >= maxit || j + 1 == m || hn == 0.0)
                fin.push_back(k);
            else
                G.j = j + 1;
        }
        if (!fin.empty()) {
            // y = R^{-1} g, x += M (V y) (flexible: x += Z y)
            int jm = 0;
            std::vector<Item> fs;
            std::vector<L0> fl0;
            for (int k : fin) {
                GmresState& G = gs[k];
                const int kk = G.j + 1;
                std::vector<cd> y(kk);
                for (int i = kk - 1; i >= 0; --i) {
                    cd s = G.g[i];
                    for (int l = i + 1; l < kk; ++l) s -= G.H[(size_t)l * (m + 1) + i] * y[l];
                    y[i] = s / G.H[(size_t)i * (m + 1) + i];
                }
                mg_ctx* c = it[k].c;
                for (int i = 0; i < kk; ++i)
                    c->coef_h[(size_t)it[k].rhs * HSTRIDE + i] = tocx(flexible ? y[i] : y[i] * scale_h(k, i));
                jm = std::max(jm, kk);
                fs.push_back(it[k]);
                fl0.push_back(L0{c->W + (size_t)it[k].rhs * c->lv[0].N, 1.0, nullptr, X[k]});
            }
            for (mg_ctx* c : ctxs)
                CK(hipMemcpyAsync(c->coef_d, c->coef_h, (size_t)c->nrhs * HSTRIDE * sizeof(cx<double>),
                                  hipMemcpyHostToDevice, R.s));
            std::vector<int> local2(fin.size());
            for (size_t q = 0; q < fin.size(); ++q) local2[q] = (int)q;
            CKS(for_groups(local2, [&](const std::vector<int>& g, int) -> mg_status {
                VecArgs a{};
                int cnt[mg::MAX_SLOTS];
                CKS(build_vec(R, dir, fs, g, a, cnt));
                double by = 0.0;
                for (int q = 0; q < a.st.n; ++q) {
                    const int k = fin[g[q]];
                    mg_ctx* c = it[k].c;
                    VecSlot& s = a.st.s[q];
                    s.V = flexible ? zbasis(it[k], 0) : basis(it[k], 0);
                    s.coef = c->coef_d + (size_t)it[k].rhs * HSTRIDE;
                    s.y = flexible ? X[k] : c->W + (size_t)it[k].rhs * c->lv[0].N;
                    s.j = gs[k].j;
                    by += 16.0 * c->lv[0].N * (gs[k].j + 2 + (flexible ? 1 : 0));
                }
                const int pi = prof_begin(R, MG_K_COMBINE, by);
                CK(mg::launch_combine(jm, flexible, a, R.s));
                prof_end(R, pi);
                return MG_OK;
            }));
            if (!flexible) CKS(vcycle(R, dir, fs, fl0, true, false));
            CKS(restart(fin));
        }
    }
    CK(hipStreamSynchronize(R.s));
    mg_status ret = MG_OK;
    for (int k = 0; k < n; ++k) {
        if (iters) iters[k] = gs[k].its;
        if (gs[k].state == 3) ret = MG_E_DIVERGED;
        else if (gs[k].state == 2 && ret == MG_OK) ret = MG_NOT_CONVERGED;
    }
    return ret;
}

mg_status solve_items(Run& R, int dir, const std::vector<Item>& it, const std::vector<cx<double>*>& U,
                      const std::vector<const cx<double>*>& F, int mode, double rtol, int maxit, int restart,
                      int* iters, double* hist) {
    if (maxit < 0 || !(rtol >= 0.0)) return MG_E_INVAL;
    if (hist)
        for (size_t i = 0; i < it.size() * (size_t)(maxit + 1); ++i) hist[i] = -1.0;
    if (mode == MG_MODE_STANDALONE) return solve_standalone(R, dir, it, U, F, rtol, maxit, iters, hist);
    if (mode == MG_MODE_GMRES || mode == MG_MODE_FGMRES) {
        if (restart < 1 || restart > MAX_RESTART) return MG_E_INVAL;
        const bool flexible = mode == MG_MODE_FGMRES || it[0].c->gsmooth;
        return solve_gmres(R, dir, it, U, F, rtol, maxit, restart, flexible, iters, hist);
    }
    return MG_E_INVAL;
}

Run ctx_run(mg_ctx* c) { return Run{c->stream, &c->prof, &c->work, &c->graphs, c->dim, c->mixed}; }

mg_status ctx_solve(mg_ctx* c, int dir, double* u, const double* f, int mode, double rtol, int maxit,
                    int restart, int* iters, double* hist) {
    if (!c || !u || !f) return MG_E_INVAL;
    std::vector<Item> it;
    std::vector<cx<double>*> U;
    std::vector<const cx<double>*> F;
    const long long N = c->lv[0].N;
    for (int r = 0; r < c->nrhs; ++r) {
        it.push_back(Item{c, r});
        U.push_back((cx<double>*)u + (size_t)r * N);
        F.push_back((const cx<double>*)f + (size_t)r * N);
    }
    Run R = ctx_run(c);
    return solve_items(R, dir, it, U, F, mode, rtol, maxit, restart, iters, hist);
}

// ---------------------------------------------------------------------------
// Set-up
// ---------------------------------------------------------------------------
void release(mg_ctx* c) {
    if (!c) return;
    graphs_free(c->graphs);
    for (Level& L : c->lv) {
        for (int d = 0; d < 2; ++d) {
            dfree(L.coef_d[d]);
            dfree(L.coef_f[d]);
        }
        dfree(L.k2);
        dfree(L.k2f);
        dfree(L.F);
        dfree(L.E);
        for (int i = 0; i < 3; ++i) dfree(L.Q[i]);
        dfree(L.SU1);
        dfree(L.SU2);
    }
    dfree(c->sb_d);
    dfree(c->gcoef);
    dfree(c->Zb);
    for (int d = 0; d < 2; ++d) {
        dfree(c->lu[d]);
        dfree(c->piv[d]);
        dfree(c->views_d[d]);
        dfree(c->outer_d[d]);
        dfree(c->views_f[d]);
    }
    dfree(c->U1);
    dfree(c->Z);
    dfree(c->W);
    dfree(c->V);
    dfree(c->scale_d);
    dfree(c->coef_d);
    hfree(c->scale_h);
    hfree(c->coef_h);
    work_free(c->work);
    for (hipEvent_t e : c->prof.pool) (void)hipEventDestroy(e);
    c->prof.pool.clear();
}

// Device descriptors of every level, both directions and precisions.
mg_status upload_views(mg_ctx* c) {
    const int d = c->dim;
    for (int dir = 0; dir < 2; ++dir) {
        std::vector<LevelView<double>> vd(c->L);
        std::vector<LevelView<float>> vf(c->L);
        for (int l = 0; l < c->L; ++l) {
            const Level& V = c->lv[l];
            LevelView<double>& a = vd[l];
            LevelView<float>& b = vf[l];
            a = LevelView<double>{};
            b = LevelView<float>{};
            for (int ax = 0; ax < 3; ++ax) {
                const int aa = ax < d ? ax : 0;
                long long o = 0;
                for (int q = 0; q < aa; ++q) o += 3LL * V.n[q];
                a.n[ax] = b.n[ax] = ax < d ? V.n[ax] : 1;
                a.cm[ax] = V.coef_d[dir] + o;
                a.c0[ax] = V.coef_d[dir] + o + V.n[aa];
                a.cp[ax] = V.coef_d[dir] + o + 2LL * V.n[aa];
                if (c->mixed) {
                    b.cm[ax] = V.coef_f[dir] + o;
                    b.c0[ax] = V.coef_f[dir] + o + V.n[aa];
                    b.cp[ax] = V.coef_f[dir] + o + 2LL * V.n[aa];
                }
            }
            a.N = b.N = V.N;
            a.k2 = V.k2;
            b.k2 = V.k2f;
            const cd s = dir ? std::conj(V.sigma) : V.sigma;
            a.sigma = tocx(s);
            b.sigma = mg::mk((float)s.real(), (float)s.imag());
            a.omega = mg::mk(c->p.omega[0], c->p.omega[1]);
            b.omega = mg::mk((float)c->p.omega[0], (float)c->p.omega[1]);
            double sc = 0.0;   // bound of the Laplacian part: sum over axes of 4 / h^2
            for (int ax = 0; ax < d; ++ax) sc += 4.0 / (V.h[ax] * V.h[ax]);
            a.sinv = 1.0 / sc;
            b.sinv = (float)(1.0 / sc);
            if (l == c->L - 1) {
                a.lu = b.lu = c->lu[dir];
                a.piv = b.piv = c->piv[dir];
            }
        }
        CKS(dalloc(&c->views_d[dir], vd.size() * sizeof(LevelView<double>)));
        CK(hipMemcpy(c->views_d[dir], vd.data(), vd.size() * sizeof(LevelView<double>), hipMemcpyHostToDevice));
        LevelView<double> outer = vd[0];   // residuals and Krylov steps: the problem's own operator
        outer.sigma = mg::mk(1.0, 0.0);
        outer.lu = nullptr;
        outer.piv = nullptr;
        CKS(dalloc(&c->outer_d[dir], sizeof(LevelView<double>)));
        CK(hipMemcpy(c->outer_d[dir], &outer, sizeof(LevelView<double>), hipMemcpyHostToDevice));
        if (c->mixed) {
            CKS(dalloc(&c->views_f[dir], vf.size() * sizeof(LevelView<float>)));
            CK(hipMemcpy(c->views_f[dir], vf.data(), vf.size() * sizeof(LevelView<float>), hipMemcpyHostToDevice));
        }
    }
    return MG_OK;
}

// Pick the tile shape of every large enough level by timing the two fused
// kernels (zero-guess variants, all right-hand sides) for every shape.
mg_status autotune(mg_ctx* c) {
    std::vector<Item> it;
    std::vector<L0> l0;
    const long long N0 = c->lv[0].N;
    if (N0 < AUTOTUNE_MIN_POINTS) return MG_OK;
    CK(mg::launch_fill_zero(c->Z, (long long)c->nrhs * N0 * sizeof(cx<double>), c->stream));
    for (int r = 0; r < c->nrhs; ++r) {
        it.push_back(Item{c, r});
        l0.push_back(L0{c->Z + (size_t)r * N0, 1.0, nullptr, c->W + (size_t)r * N0});
    }
    for (int l = 1; l < c->L; ++l) {
        CK(mg::launch_fill_zero(c->lv[l].F, (long long)c->nrhs * c->lv[l].N * elem(c), c->stream));
        CK(mg::launch_fill_zero(c->lv[l].E, (long long)c->nrhs * c->lv[l].N * elem(c), c->stream));
    }
    hipEvent_t e0, e1;
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    Run R = ctx_run(c);
    R.prof = nullptr;
    R.gc = nullptr;
    mg_status st = MG_OK;
    for (int l = 0; l < c->lt && st == MG_OK; ++l) {
        if (c->lv[l].N < AUTOTUNE_MIN_POINTS) break;
        float best = 1e30f;
        int best_shape = 0;
        for (int shape = 0; shape < mg::NUM_TILE_SHAPES && st == MG_OK; ++shape) {
            c->lv[l].shape = shape;
            float tot = 0.0f;
            for (int rep = 0; rep < 4 && st == MG_OK; ++rep) {
                if (hipEventRecord(e0, c->stream) != hipSuccess) st = MG_E_DEVICE;
                if (st == MG_OK) st = cycle_down(R, 0, it, &l0, l, false);
                if (st == MG_OK) st = cycle_up(R, 0, it, &l0, l, false);
                if (st == MG_OK && hipEventRecord(e1, c->stream) != hipSuccess) st = MG_E_DEVICE;
                if (st == MG_OK && hipEventSynchronize(e1) != hipSuccess) st = MG_E_DEVICE;
                float ms = 0.0f;
                if (st == MG_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = MG_E_DEVICE;
                if (rep > 0) tot += ms;
            }
            if (tot < best) {
                best = tot;
                best_shape = shape;
            }
        }
        c->lv[l].shape = best_shape;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
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
    // sigma_0 != 1: a fixed-shift (comparator) preconditioner; the outer
    // operator stays -Delta - k^2
    c->shifted0 = c->lv[0].sigma != cd(1.0, 0.0);

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
            auto& Fw = V.coef_host[0];
            Fw.insert(Fw.end(), cm.begin(), cm.end());
            Fw.insert(Fw.end(), c0.begin(), c0.end());
            Fw.insert(Fw.end(), cp.begin(), cp.end());
            auto& Hw = V.coef_host[1];
            Hw.insert(Hw.end(), hm.begin(), hm.end());
            Hw.insert(Hw.end(), h0.begin(), h0.end());
            Hw.insert(Hw.end(), hp.begin(), hp.end());
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
    CKS(upload_views(c));

    // work vectors
    const size_t esz = elem(c);
    for (int l = 1; l < L; ++l) {
        CKS(dalloc(&c->lv[l].F, (size_t)c->nrhs * c->lv[l].N * esz));
        CKS(dalloc(&c->lv[l].E, (size_t)c->nrhs * c->lv[l].N * esz));
    }
    c->gsmooth = p->smoother == MG_SMOOTH_GMRES3;
    // coarse tail: from the first level >= 1 with at most TAIL_POINTS points
    c->lt = L - 1;
    for (int l = 1; l < L; ++l)
        if (c->lv[l].N <= mg::TAIL_POINTS) {
            c->lt = l;
            break;
        }
    {
        std::vector<mg::SmoothBufs> sb((size_t)c->nrhs * L);
        CKS(dalloc(&c->gcoef, (size_t)c->nrhs * L * 8 * sizeof(cx<double>)));
        for (int l = 0; l < L; ++l) {
            Level& V = c->lv[l];
            const size_t bytes = (size_t)c->nrhs * V.N * esz;
            const bool tail = l >= c->lt;
            // the 2D GMRES(3) passes keep only u1 (and q0 of an incoming
            // iterate); the 3D passes and the tail use q0..q2 and u1
            for (int i = 0; i < 3; ++i)
                if (tail || (c->gsmooth && (d == 3 || (i == 0 && l == 0)))) CKS(dalloc(&V.Q[i], bytes));
            if (tail || c->gsmooth) CKS(dalloc(&V.SU1, bytes));
            if (c->gsmooth && d == 3 && !tail) CKS(dalloc(&V.SU2, bytes));
            for (int r = 0; r < c->nrhs; ++r) {
                mg::SmoothBufs& b = sb[(size_t)r * L + l];
                for (int i = 0; i < 3; ++i) b.q[i] = V.Q[i] ? lvec(c, V.Q[i], l, r) : nullptr;
                b.u1 = V.SU1 ? lvec(c, V.SU1, l, r) : nullptr;
                b.u2 = V.SU2 ? lvec(c, V.SU2, l, r) : nullptr;
                b.coef = c->gcoef + ((size_t)r * L + l) * 8;
                b.f = l > 0 ? lvec(c, V.F, l, r) : nullptr;
                b.e = l > 0 ? lvec(c, V.E, l, r) : nullptr;
            }
        }
        CKS(dalloc(&c->sb_d, sb.size() * sizeof(mg::SmoothBufs)));
        CK(hipMemcpy(c->sb_d, sb.data(), sb.size() * sizeof(mg::SmoothBufs), hipMemcpyHostToDevice));
    }
    const size_t vbytes = (size_t)c->nrhs * c->lv[0].N * sizeof(cx<double>);
    if (!c->mixed) CKS(dalloc(&c->U1, vbytes));
    CKS(dalloc(&c->Z, vbytes));
    CKS(dalloc(&c->W, vbytes));
    int maxt = 0;
    for (int shape = 0; shape < mg::NUM_TILE_SHAPES; ++shape) {
        int nt[3];
        mg::tile_counts(d, shape, c->lv[0].n, nt);
        maxt = std::max(maxt, nt[0] * nt[1] * nt[2]);
        if (d == 2) {
            mg::march_counts(shape, c->lv[0].n, nt);
            maxt = std::max(maxt, nt[0] * nt[1]);
        }
    }
    maxt = std::max(maxt, mg::mv_blocks(c->dim, c->lv[0].n, VEC_PER_DOT));
    CKS(work_alloc(c->work, c->nrhs, std::max(maxt, mg::vec_blocks(c->lv[0].N))));
    CKS(dalloc(&c->scale_d, (size_t)c->nrhs * HSTRIDE * sizeof(double)));
    CKS(dalloc(&c->coef_d, (size_t)c->nrhs * HSTRIDE * sizeof(cx<double>)));
    CKS(halloc(&c->scale_h, (size_t)c->nrhs * HSTRIDE * sizeof(double)));
    CKS(halloc(&c->coef_h, (size_t)c->nrhs * HSTRIDE * sizeof(cx<double>)));
    CK(hipStreamSynchronize(c->stream));
    CKS(autotune(c));
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
    if (p->smoother != MG_SMOOTH_JACOBI && p->smoother != MG_SMOOTH_GMRES3) return MG_E_INVAL;
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
    std::vector<Item> it;
    std::vector<L0> l0;
    Run R = ctx_run(c);
    for (int r = 0; r < c->nrhs; ++r) {
        it.push_back(Item{c, r});
        cx<double>* ur = (cx<double>*)u + (size_t)r * N;
        const cx<double>* fr = (const cx<double>*)f + (size_t)r * N;
        if (!c->mixed && !c->shifted0)
            l0.push_back(L0{fr, 1.0, ur, ur});
        else
            l0.push_back(L0{c->W + (size_t)r * N, 1.0, nullptr, ur});
    }
    if (!c->mixed && !c->shifted0) {
        CKS(vcycle(R, 0, it, l0, false, res_before != nullptr));
        if (res_before) {
            CK(hipStreamSynchronize(c->stream));
            for (int r = 0; r < c->nrhs; ++r) res_before[r] = std::sqrt(c->work.rtot_h[r]);
        }
    } else {
        std::vector<int> who(c->nrhs);
        std::vector<const cx<double>*> xs, fs;
        std::vector<cx<double>*> ys;
        for (int r = 0; r < c->nrhs; ++r) {
            who[r] = r;
            xs.push_back((const cx<double>*)u + (size_t)r * N);
            fs.push_back((const cx<double>*)f + (size_t)r * N);
            ys.push_back(c->W + (size_t)r * N);
        }
        std::vector<double> nr;
        CKS(residual(R, 0, it, who, xs, fs, ys, res_before ? &nr : nullptr));
        if (res_before)
            for (int r = 0; r < c->nrhs; ++r) res_before[r] = std::sqrt(nr[r]);
        CKS(vcycle(R, 0, it, l0, true, false));
    }
    return MG_OK;
}

mg_status mg_solve(mg_ctx* c, double* u, const double* f, int mode, double rtol, int maxit, int restart,
                   int* iters, double* hist) {
    return ctx_solve(c, 0, u, f, mode, rtol, maxit, restart, iters, hist);
}

mg_status mg_solve_adjoint(mg_ctx* c, double* lam, const double* g, int mode, double rtol, int maxit,
                           int restart, int* iters, double* hist) {
    return ctx_solve(c, 1, lam, g, mode, rtol, maxit, restart, iters, hist);
}

mg_status mg_grad_k2(mg_ctx* c, const double* u, const double* lam, double* grad) {
    if (!c || !u || !lam || !grad) return MG_E_INVAL;
    Run R = ctx_run(c);
    const int pi = prof_begin(R, MG_K_OTHER, (double)c->lv[0].N * (32.0 * c->nrhs + 16.0));
    CK(mg::launch_grad_k2((const cx<double>*)u, (const cx<double>*)lam, c->nrhs, c->lv[0].N, grad, c->stream));
    prof_end(R, pi);
    return MG_OK;
}

mg_status mg_apply(mg_ctx* c, int level, int adjoint, const double* x, double* y) {
    if (!c || !x || !y || level < 0 || level >= c->L) return MG_E_INVAL;
    const long long N = c->lv[level].N;
    const int dir = adjoint ? 1 : 0;
    for (int r0 = 0; r0 < c->nrhs; r0 += mg::MAX_SLOTS) {
        VecArgs a{};
        a.st.n = std::min(mg::MAX_SLOTS, c->nrhs - r0);
        int blocks = 0;
        for (int q = 0; q < a.st.n; ++q) {
            VecSlot& s = a.st.s[q];
            s.lv = c->views_d[dir] + level;
            s.x = (const cx<double>*)x + (size_t)(r0 + q) * N;
            s.y = (cx<double>*)y + (size_t)(r0 + q) * N;
            s.block0 = blocks;
            blocks += mg::vec_blocks(N);
        }
        a.st.nblocks = blocks;
        a.bstride = c->work.bstride;
        CK(mg::launch_residual(c->dim, a, c->stream));
    }
    return MG_OK;
}

int mg_tile_shape(mg_ctx* c, int level, int shape) {
    if (!c || level < 0 || level >= c->L) return MG_E_INVAL;
    if (shape >= mg::NUM_TILE_SHAPES) return MG_E_INVAL;
    if (shape >= 0) {
        if (hipStreamSynchronize(c->stream) != hipSuccess) return MG_E_DEVICE;
        c->lv[level].shape = shape;
        graphs_free(c->graphs);   // captured coarse parts hold the old shapes
    }
    return c->lv[level].shape;
}

mg_status mg_batch_create(mg_ctx* const* ctxs, int count, mg_batch** out) {
    if (!out) return MG_E_INVAL;
    *out = nullptr;
    if (!ctxs || count < 1) return MG_E_INVAL;
    int items = 0, bstride = 0;
    for (int i = 0; i < count; ++i) {
        const mg_ctx* c = ctxs[i];
        if (!c || c->dim != ctxs[0]->dim || c->mixed != ctxs[0]->mixed || c->stream != ctxs[0]->stream ||
            c->gsmooth != ctxs[0]->gsmooth || c->shifted0 != ctxs[0]->shifted0)
            return MG_E_INVAL;
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == c) return MG_E_INVAL;
        items += c->nrhs;
        bstride = std::max(bstride, c->work.bstride);
    }
    mg_batch* b = new (std::nothrow) mg_batch();
    if (!b) return MG_E_NOMEM;
    b->ctxs.assign(ctxs, ctxs + count);
    const mg_status st = work_alloc(b->work, items, bstride);
    if (st != MG_OK) {
        work_free(b->work);
        delete b;
        return st;
    }
    *out = b;
    return MG_OK;
}

mg_status mg_batch_solve(mg_batch* b, double* const* u, const double* const* f, int mode, double rtol,
                         int maxit, int restart, int* iters, double* hist) {
    if (!b || !u || !f) return MG_E_INVAL;
    std::vector<Item> it;
    std::vector<cx<double>*> U;
    std::vector<const cx<double>*> F;
    for (size_t i = 0; i < b->ctxs.size(); ++i) {
        mg_ctx* c = b->ctxs[i];
        if (!u[i] || !f[i]) return MG_E_INVAL;
        const long long N = c->lv[0].N;
        for (int r = 0; r < c->nrhs; ++r) {
            it.push_back(Item{c, r});
            U.push_back((cx<double>*)u[i] + (size_t)r * N);
            F.push_back((const cx<double>*)f[i] + (size_t)r * N);
        }
    }
    mg_ctx* c0 = b->ctxs[0];
    Run R{c0->stream, &c0->prof, &b->work, &b->graphs, c0->dim, c0->mixed};
    return solve_items(R, 0, it, U, F, mode, rtol, maxit, restart, iters, hist);
}

void mg_batch_destroy(mg_batch* b) {
    if (!b) return;
    if (!b->ctxs.empty()) (void)hipStreamSynchronize(b->ctxs[0]->stream);
    graphs_free(b->graphs);
    work_free(b->work);
    delete b;
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
    (void)hipStreamSynchronize(c->stream);
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
