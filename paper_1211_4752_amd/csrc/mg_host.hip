// Host runtime of the level-dependent multigrid: hierarchy set-up, tile-shape
// and sweep-schedule autotuning, recorded operations (fixed launch sequences
// with device-resident slot tables, replayed as HIP graphs), the standalone
// and (F)GMRES solvers over "items" (one right-hand side of one problem) with
// their control on the device, batches of problems, the adjoint, and the C
// ABI of include/mg.h.
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
#include <functional>
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

using mg::HSTRIDE;
using mg::MAX_RESTART;
constexpr long long AUTOTUNE_MIN_POINTS = 1024;

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

// Solve (LU) x = b in place with the factors and interchanges of lu_factor.
void lu_solve(const std::vector<cd>& A, const std::vector<int>& piv, int n, std::vector<cd>& b) {
    for (int k = 0; k < n; ++k)
        if (piv[k] != k) std::swap(b[k], b[piv[k]]);
    for (int k = 0; k < n; ++k)
        for (int i = k + 1; i < n; ++i) b[i] -= A[(size_t)i * n + k] * b[k];
    for (int k = n - 1; k >= 0; --k) {
        cd s = b[k];
        for (int j = k + 1; j < n; ++j) s -= A[(size_t)k * n + j] * b[j];
        b[k] = s / A[(size_t)k * n + k];
    }
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

// Kernel timing: per class, summed milliseconds, launches and algorithmic
// bytes since profiling was enabled.
struct Prof {
    bool on = false;
    double ms[MG_K_NUM_CLASSES] = {};
    long long cnt[MG_K_NUM_CLASSES] = {};
    double bytes[MG_K_NUM_CLASSES] = {};
    void clear() {
        for (int i = 0; i < MG_K_NUM_CLASSES; ++i) {
            ms[i] = bytes[i] = 0.0;
            cnt[i] = 0;
        }
    }
};

// Reduction work space and the device state of the Krylov control, for the
// items (right-hand sides) of one context or one batch.
struct Work {
    cx<double>* part = nullptr;   // [(slot * HSTRIDE + v) * bstride + b]
    double* rpart = nullptr;      // [slot * bstride + b]
    int bstride = 0;
    int items = 0;
    double* rtot = nullptr;       // [slot]: generic reductions
    double* rtot_h = nullptr;     // pinned mirror
    mg::GmState* gst = nullptr;   // [item]
    mg::GmFlags* gfl = nullptr;   // [item]
    mg::GmFlags* gfl_h = nullptr; // pinned mirror
    mg::GmParams* prm = nullptr;  // device
    mg::GmParams* prm_h = nullptr;// pinned
    double* hist = nullptr;       // [item][hstride]
    size_t hcap = 0;              // doubles
};

// ---------------------------------------------------------------------------
// Recorded operations.  An operation is a fixed sequence of kernel launches
// whose slot tables are staged on the host while it is recorded and then
// live in one device buffer; it runs either launch by launch or, captured
// once, as a HIP graph.  Everything that changes from run to run (which
// right-hand sides still iterate, step coefficients, scales) is read by the
// kernels from device memory, so a recording stays valid.
// ---------------------------------------------------------------------------
constexpr int TAG_ALWAYS = -1;    // step runs for every item of the operation
constexpr int TAG_FIN = -2;       // step of the end of a restart cycle

struct ItemBytes {
    int k;             // item
    double base;       // algorithmic bytes of the launch for this item
    double per;        // plus this many per Arnoldi step of the restart cycle
};

struct Step {
    std::function<hipError_t(hipStream_t, const char*)> fn;
    int cls;                      // profiling class
    int tag;                      // TAG_ALWAYS, TAG_FIN or the step / cycle index
    std::vector<ItemBytes> ib;
};

struct Op {
    std::vector<char> tab;        // staged device tables
    char* dtab = nullptr;
    std::vector<Step> steps;
    hipGraphExec_t exec = nullptr;
    std::vector<hipEvent_t> ev;       // 2 per step, recorded by profiled runs
    bool uploaded = false;
    // after step `mark` every run records mark_ev (in the graph as an event
    // node), so that another stream can start its own work once this one
    // has got that far
    int mark = -1;
    hipEvent_t mark_ev = nullptr;
};

struct OpCache {
    std::map<std::vector<uintptr_t>, Op*> ops;
    hipStream_t capture = nullptr;   // private stream used only for capture
};

}  // namespace

// Groups of right-hand sides a multi-rhs (F)GMRES solve of one context is
// split into (each on its own stream, see solve_groups).
constexpr int SOLVE_GROUPS = 3;

struct mg_ctx {
    mg_params p{};
    int dim = 2;
    int L = 0;
    bool mixed = false;
    int nrhs = 1;
    hipStream_t stream = nullptr;
    std::vector<Level> lv;
    int ncoarse = 0;
    cx<double>* cinv[2] = {nullptr, nullptr};   // inverse of the coarsest operator per direction
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
    double* scale_d = nullptr;        // [rhs * HSTRIDE + i]
    cx<double>* coef_d = nullptr;     // [rhs * HSTRIDE + i]
    int vper = 64;                    // points per thread of the Arnoldi passes (sweep schedule)
    bool vtuned = false;
    unsigned gen = 0;                 // bumped when buffers baked into recordings move
    int device = 0;                   // HIP device of the context
    char* stage = nullptr;            // pinned staging of mg_cycle_noalloc's tables
    hipEvent_t stage_ev = nullptr;    // marks the end of the last staging copy
    Work work;
    Prof prof;
    OpCache cache;
    // further groups of the right-hand sides of a (F)GMRES solve, each on
    // its own stream (created on first use)
    Work workg[SOLVE_GROUPS - 1];
    hipStream_t streamg[SOLVE_GROUPS - 1] = {};
};

struct mg_batch {
    std::vector<mg_ctx*> ctxs;
    Work work;
    OpCache cache;
    Work workg[SOLVE_GROUPS - 1];             // as in mg_ctx
    hipStream_t streamg[SOLVE_GROUPS - 1] = {};
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
    CKS(dalloc(&w.part, (size_t)items * HSTRIDE * bstride * sizeof(cx<double>)));
    CKS(dalloc(&w.rpart, (size_t)items * bstride * sizeof(double)));
    CKS(dalloc(&w.rtot, (size_t)items * sizeof(double)));
    CKS(halloc(&w.rtot_h, (size_t)items * sizeof(double)));
    CKS(dalloc(&w.gst, (size_t)items * sizeof(mg::GmState)));
    CKS(dalloc(&w.gfl, (size_t)items * sizeof(mg::GmFlags)));
    CKS(halloc(&w.gfl_h, (size_t)items * sizeof(mg::GmFlags)));
    CKS(dalloc(&w.prm, sizeof(mg::GmParams)));
    CKS(halloc(&w.prm_h, sizeof(mg::GmParams)));
    return MG_OK;
}

void work_free(Work& w) {
    dfree(w.part);
    dfree(w.rpart);
    dfree(w.rtot);
    hfree(w.rtot_h);
    dfree(w.gst);
    dfree(w.gfl);
    hfree(w.gfl_h);
    dfree(w.prm);
    hfree(w.prm_h);
    dfree(w.hist);
    w.hcap = 0;
}

// History rows of every item (the stream must be idle).
mg_status ensure_hist(Work& w, size_t doubles) {
    if (w.hcap >= doubles) return MG_OK;
    dfree(w.hist);
    w.hcap = 0;
    CKS(dalloc(&w.hist, doubles * sizeof(double)));
    w.hcap = doubles;
    return MG_OK;
}

void op_release(Op& op) {
    if (op.exec) (void)hipGraphExecDestroy(op.exec);
    op.exec = nullptr;
    for (hipEvent_t e : op.ev) (void)hipEventDestroy(e);
    op.ev.clear();
    if (op.mark_ev) (void)hipEventDestroy(op.mark_ev);
    op.mark_ev = nullptr;
    dfree(op.dtab);
}

void op_free(Op* op) {
    if (!op) return;
    op_release(*op);
    delete op;
}

void cache_clear(OpCache& c) {
    for (auto& kv : c.ops) op_free(kv.second);
    c.ops.clear();
}

void cache_free(OpCache& c) {
    cache_clear(c);
    if (c.capture) (void)hipStreamDestroy(c.capture);
    c.capture = nullptr;
}

template <typename T>
size_t put(Op& op, const std::vector<T>& v) {
    const size_t off = (op.tab.size() + 255) & ~(size_t)255;
    op.tab.resize(off + std::max<size_t>(1, v.size()) * sizeof(T));
    if (!v.empty()) std::memcpy(op.tab.data() + off, v.data(), v.size() * sizeof(T));
    return off;
}

// Where and how operations run.
struct Exec {
    hipStream_t s;
    Prof* prof;
    OpCache* cache;
    bool graphs;
};

double step_bytes(const Step& st, const std::vector<int>* live) {
    double b = 0.0;
    for (const ItemBytes& x : st.ib) {
        const int n = live ? (*live)[x.k] : 0;
        if (live) {
            if (st.tag >= 0 && n <= st.tag) continue;
            if (st.tag == TAG_FIN && n <= 0) continue;
        }
        b += x.base + x.per * n;
    }
    return b;
}

bool profiling(const Exec& E) { return E.prof && E.prof->on; }

// Capture the steps of op on the cache's capture stream and instantiate
// the graph.
mg_status op_capture(Exec& E, Op& op, hipGraphExec_t* out) {
    if (!E.cache->capture) CK(hipStreamCreateWithFlags(&E.cache->capture, hipStreamNonBlocking));
    hipStream_t cs = E.cache->capture;
    CK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    hipError_t err = hipSuccess;
    for (size_t i = 0; i < op.steps.size() && err == hipSuccess; ++i) {
        err = op.steps[i].fn(cs, op.dtab);
        if (err == hipSuccess && (int)i == op.mark) err = hipEventRecord(op.mark_ev, cs);
    }
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(cs, &g);
    if (err != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return MG_E_DEVICE;
    }
    const hipError_t ei = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    CK(ei);
    return MG_OK;
}

// Run op on E.s, as its captured graph, or launch by launch.  Profiled runs
// go launch by launch with a HIP event before and after every launch (the
// runtime records events captured into a graph but cannot time them);
// op_collect adds the timings once the stream has passed the run.
mg_status op_run(Exec& E, Op& op) {
    if (op.steps.empty()) return MG_OK;
    if (!op.uploaded) {
        if (!op.tab.empty()) {
            CKS(dalloc(&op.dtab, op.tab.size()));
            CK(hipMemcpy(op.dtab, op.tab.data(), op.tab.size(), hipMemcpyHostToDevice));
        }
        op.uploaded = true;
    }
    const bool prof = profiling(E);
    if (op.mark >= 0 && !op.mark_ev) CK(hipEventCreateWithFlags(&op.mark_ev, hipEventDisableTiming));
    if (prof)
        while (op.ev.size() < 2 * op.steps.size()) {
            hipEvent_t e;
            CK(hipEventCreate(&e));
            op.ev.push_back(e);
        }
    if (prof || !E.graphs || !E.cache) {
        for (size_t i = 0; i < op.steps.size(); ++i) {
            if (prof) CK(hipEventRecord(op.ev[2 * i], E.s));
            CK(op.steps[i].fn(E.s, op.dtab));
            if (prof) CK(hipEventRecord(op.ev[2 * i + 1], E.s));
            if ((int)i == op.mark) CK(hipEventRecord(op.mark_ev, E.s));
        }
        return MG_OK;
    }
    if (!op.exec) CKS(op_capture(E, op, &op.exec));
    CK(hipGraphLaunch(op.exec, E.s));
    return MG_OK;
}

// Timings of the last profiled run of op (the stream has passed it); live:
// Arnoldi steps (or cycles) each item took in that run, null = all items.
mg_status op_collect(Exec& E, const Op& op, const std::vector<int>* live) {
    if (!profiling(E) || op.ev.size() < 2 * op.steps.size()) return MG_OK;
    for (size_t i = 0; i < op.steps.size(); ++i) {
        const Step& st = op.steps[i];
        float ms = 0.0f;
        CK(hipEventElapsedTime(&ms, op.ev[2 * i], op.ev[2 * i + 1]));
        E.prof->ms[st.cls] += ms;
        E.prof->cnt[st.cls] += 1;
        E.prof->bytes[st.cls] += step_bytes(st, live);
    }
    return MG_OK;
}

template <typename F>
mg_status cached(OpCache& cache, const std::vector<uintptr_t>& key, Op** out, F record) {
    auto f = cache.ops.find(key);
    if (f != cache.ops.end()) {
        *out = f->second;
        return MG_OK;
    }
    Op* op = new (std::nothrow) Op();
    if (!op) return MG_E_NOMEM;
    const mg_status st = record(*op);
    if (st != MG_OK) {
        op_free(op);
        return st;
    }
    cache.ops.emplace(key, op);
    *out = op;
    return MG_OK;
}

// Recording context.
struct Rec {
    Op* op;
    Work* w;
    int dim;
    bool mixed;
    int tag;
};

void add(Rec& R, int cls, std::vector<ItemBytes> ib, std::function<hipError_t(hipStream_t, const char*)> fn) {
    R.op->steps.push_back(Step{std::move(fn), cls, R.tag, std::move(ib)});
}

// One right-hand side of one problem.
struct Item {
    mg_ctx* c;
    int rhs;
};

// Gates: which device flag of an item lets a slot run.
enum Gate { G_NONE = 0, G_LIVE = 1, G_FIN = 2, G_ZERO = 3 };

const int* gate_of(const Rec& R, int gk, int k) {
    mg::GmFlags* f = R.w->gfl + k;
    switch (gk) {
        case G_LIVE: return &f->live;
        case G_FIN: return &f->fin;
        case G_ZERO: return &f->zero;
        default: return nullptr;
    }
}

// Level-0 inputs and outputs of one item's cycle.
struct L0 {
    const void* f;            // right-hand side (complex double)
    double fs;                // scale applied to f
    const double* fsp;        // device scale of f (overrides fs) or null
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
const mg::SmoothBufs* sbuf(const mg_ctx* c, int l, int rhs) { return c->sb_d + (size_t)rhs * c->L + l; }
cx<double>* gcoef_of(const mg_ctx* c, int l, int rhs, int phase) {
    return c->gcoef + ((size_t)rhs * c->L + l) * 8 + 4 * phase;
}

// Shape of a launch at depth d: the one tuned for the largest level in it.
int launch_shape(const std::vector<Item>& it, const std::vector<int>& who, int d) {
    long long best = -1;
    int shape = 0;
    for (int k : who) {
        const Level& V = it[k].c->lv[d];
        if (V.N > best) {
            best = V.N;
            shape = V.shape;
        }
    }
    return shape;
}

// Shape ids of a context: omega-Jacobi: the tile shapes, then the
// plane-sweep configurations of the zero-guess fused kernels; GMRES(3): the
// row-marching strips (2D) or the tile shapes (3D).
int num_shapes(const mg_ctx* c) {
    if (c->gsmooth) return c->dim == 2 ? mg::NUM_MARCH_SHAPES : mg::NUM_TILE_SHAPES;
    return mg::NUM_TILE_SHAPES + mg::NUM_SWEEP_SHAPES;
}

// Sweep configuration of an omega-Jacobi launch (-1: tiles) and its tile
// shape; the sweeps serve the zero-guess kernels only.
void split_shape(int shape, bool zero, int* sweep, int* tile) {
    const bool sw = shape >= mg::NUM_TILE_SHAPES;
    *sweep = sw && zero ? shape - mg::NUM_TILE_SHAPES : -1;
    *tile = sw ? 0 : shape;
}

void fused_counts(int dim, int sweep, int tile, const int n[3], int nt[3]) {
    if (sweep >= 0)
        mg::sweep_counts(dim, sweep, n, nt);
    else
        mg::tile_counts(dim, tile, n, nt);
}

std::vector<int> above_tail(const std::vector<Item>& it, int d) {
    std::vector<int> who;
    for (int k = 0; k < (int)it.size(); ++k)
        if (d < it[k].c->lt) who.push_back(k);
    return who;
}

// ---------------------------------------------------------------------------
// V-cycle pieces (Sec. 3.1)
// ---------------------------------------------------------------------------

// K_A (omega-Jacobi) at depth d for the items that have a coarser level
// below d.  With norm (level 0 with incoming iterates) the partials of
// ||f - A u||^2 of item k land in rpart[k * bstride + tile], (*cnt)[k] tiles.
mg_status rec_ka(Rec& R, int dir, const std::vector<Item>& it, int gk, const std::vector<L0>* l0, int d,
                 bool norm, std::vector<int>* cnt) {
    const std::vector<int> who = above_tail(it, d);
    if (who.empty()) return MG_OK;
    const bool zero = !(d == 0 && l0 && (*l0)[0].u);
    norm = norm && !zero;
    if (norm && who.size() != it.size()) return MG_E_STATE;
    int sweep, shape;
    split_shape(launch_shape(it, who, d), zero, &sweep, &shape);
    const double ct = R.mixed ? 8.0 : 16.0, sk = R.mixed ? 4.0 : 8.0;
    std::vector<mg::CycleSlot> sl(who.size());
    std::vector<ItemBytes> ib;
    if (cnt) cnt->assign(it.size(), 0);
    int tiles = 0;
    for (size_t q = 0; q < who.size(); ++q) {
        const int k = who[q];
        const Item& I = it[k];
        mg_ctx* c = I.c;
        mg::CycleSlot& s = sl[q];
        s = mg::CycleSlot{};
        s.lv = view_ptr(c, dir, d);
        if (d == 0) {
            const L0& z = (*l0)[k];
            s.f = z.f;
            s.fscale = z.fs;
            s.fsp = z.fsp;
            s.u = z.u;
            s.u1 = z.u ? (void*)(c->U1 + (size_t)I.rhs * c->lv[0].N) : nullptr;
        } else {
            s.f = lvec(c, c->lv[d].F, d, I.rhs);
            s.fscale = 1.0;
        }
        s.c = lvec(c, c->lv[d + 1].F, d + 1, I.rhs);
        s.gate = gate_of(R, gk, k);
        s.tile0 = tiles;
        int nt[3];
        fused_counts(R.dim, sweep, shape, c->lv[d].n, nt);
        const int n = nt[0] * nt[1] * nt[2];
        if (norm && n > R.w->bstride) return MG_E_STATE;
        if (cnt) (*cnt)[k] = n;
        tiles += n;
        double by = c->lv[d].N * ((d == 0 ? 16.0 : ct) + sk) + c->lv[d + 1].N * ct;
        if (!zero) by += c->lv[0].N * 2.0 * ct;
        ib.push_back({k, by, 0.0});
    }
    mg::CycleArgs a{};
    a.st.n = (int)sl.size();
    a.st.ntiles = tiles;
    a.norm_part = norm ? R.w->rpart : nullptr;
    a.pstride = R.w->bstride;
    const size_t off = put(*R.op, sl);
    const int dim = R.dim;
    const bool mixed = R.mixed;
    add(R, d == 0 ? MG_K_SMOOTH_RESTRICT_FINE : MG_K_COARSE_LEVELS, ib, [=](hipStream_t s, const char* base) {
        mg::CycleArgs b = a;
        b.st.s = (const mg::CycleSlot*)(base + off);
        if (sweep >= 0) return mg::launch_sweep_sr(dim, mixed, d == 0, sweep, b, s);
        return mg::launch_smooth_restrict(dim, mixed, d == 0, zero, shape, b, s);
    });
    return MG_OK;
}

// K_B (omega-Jacobi) at depth d.
mg_status rec_kb(Rec& R, int dir, const std::vector<Item>& it, int gk, const std::vector<L0>* l0, int d, bool acc) {
    const std::vector<int> who = above_tail(it, d);
    if (who.empty()) return MG_OK;
    const bool zero = !(d == 0 && l0 && (*l0)[0].u);
    int sweep, shape;
    split_shape(launch_shape(it, who, d), zero, &sweep, &shape);
    const double ct = R.mixed ? 8.0 : 16.0, sk = R.mixed ? 4.0 : 8.0;
    std::vector<mg::CycleSlot> sl(who.size());
    std::vector<ItemBytes> ib;
    int tiles = 0;
    for (size_t q = 0; q < who.size(); ++q) {
        const int k = who[q];
        const Item& I = it[k];
        mg_ctx* c = I.c;
        mg::CycleSlot& s = sl[q];
        s = mg::CycleSlot{};
        s.lv = view_ptr(c, dir, d);
        if (d == 0) {
            const L0& z = (*l0)[k];
            s.f = z.f;
            s.fscale = z.fs;
            s.fsp = z.fsp;
            s.u1 = z.u ? (void*)(c->U1 + (size_t)I.rhs * c->lv[0].N) : nullptr;
            s.out = z.out;
        } else {
            s.f = lvec(c, c->lv[d].F, d, I.rhs);
            s.fscale = 1.0;
            s.out = lvec(c, c->lv[d].E, d, I.rhs);
        }
        s.c = lvec(c, c->lv[d + 1].E, d + 1, I.rhs);
        s.gate = gate_of(R, gk, k);
        s.tile0 = tiles;
        int nt[3];
        fused_counts(R.dim, sweep, shape, c->lv[d].n, nt);
        tiles += nt[0] * nt[1] * nt[2];
        const double cf = d == 0 ? 16.0 : ct;
        double by = c->lv[d].N * (cf + sk + cf) + c->lv[d + 1].N * ct;
        if (!zero) by += c->lv[0].N * ct;
        if (d == 0 && acc) by += c->lv[0].N * 16.0;
        ib.push_back({k, by, 0.0});
    }
    mg::CycleArgs a{};
    a.st.n = (int)sl.size();
    a.st.ntiles = tiles;
    const size_t off = put(*R.op, sl);
    const int dim = R.dim;
    const bool mixed = R.mixed;
    const bool ac = d == 0 && acc;
    add(R, d == 0 ? MG_K_PROLONG_SMOOTH_FINE : MG_K_COARSE_LEVELS, ib, [=](hipStream_t s, const char* base) {
        mg::CycleArgs b = a;
        b.st.s = (const mg::CycleSlot*)(base + off);
        if (sweep >= 0) return mg::launch_sweep_ps(dim, mixed, d == 0, ac, sweep, b, s);
        return mg::launch_prolong_smooth(dim, mixed, d == 0, zero, ac, shape, b, s);
    });
    return MG_OK;
}

// The coarse tail of every item (levels lt..L-1 and the coarsest solve),
// one workgroup per item: its correction lands in E_lt.
mg_status rec_tail(Rec& R, int dir, const std::vector<Item>& it, int gk) {
    std::vector<mg::TailSlot> sl(it.size());
    std::vector<ItemBytes> ib;
    for (size_t k = 0; k < it.size(); ++k) {
        const Item& I = it[k];
        mg_ctx* c = I.c;
        mg::TailSlot& s = sl[k];
        s = mg::TailSlot{};
        s.lv = view_ptr(c, dir, c->lt);
        s.sb = sbuf(c, c->lt, I.rhs);
        s.nlev = c->L - c->lt;
        s.gate = gate_of(R, gk, (int)k);
        double by = 0.0;
        for (int l = c->lt; l < c->L; ++l) by += 2.0 * c->lv[l].N * (R.mixed ? 8.0 : 16.0);
        ib.push_back({(int)k, by, 0.0});
    }
    mg::TailArgs a{};
    a.n = (int)sl.size();
    a.gmres = it[0].c->gsmooth ? 1 : 0;
    a.brk = R.mixed ? 1e-5 : 1e-13;
    const size_t off = put(*R.op, sl);
    const int dim = R.dim;
    const bool mixed = R.mixed;
    add(R, MG_K_COARSEST_SOLVE, ib, [=](hipStream_t s, const char* base) {
        mg::TailArgs b = a;
        b.s = (const mg::TailSlot*)(base + off);
        return mg::launch_tail(dim, mixed, b, s);
    });
    return MG_OK;
}

// ---------------------------------------------------------------------------
// Vector passes on level 0 (residual, norm, Arnoldi passes, combination)
// ---------------------------------------------------------------------------
enum Blk { B_VEC = 0, B_DOT = 1, B_MV = 2 };

// Chunks per slot of the Arnoldi passes: vper points per thread per
// workgroup when every slot is live, so chunks of vper / ARN_SPLIT.
int chunks_of(const mg_ctx* c, int bk) {
    return mg::arnoldi_chunks(bk == B_MV, c->dim, c->lv[0].n, c->lv[0].N, c->vper / mg::ARN_SPLIT);
}

int blocks_of(const mg_ctx* c, int bk) {
    if (bk == B_DOT || bk == B_MV) return (chunks_of(c, bk) + mg::ARN_SPLIT - 1) / mg::ARN_SPLIT;
    return mg::vec_blocks(c->lv[0].N);
}

// One vector launch over every item: fill(k, slot, bytes) completes the
// slots; (*cnt)[k] = workgroups of item k (= its partials).
template <typename F, typename L>
mg_status rec_vec(Rec& R, int dir, const std::vector<Item>& it, int gk, int bk, int cls, std::vector<int>* cnt,
                  F fill, L launch) {
    std::vector<mg::VecSlot> sl(it.size());
    std::vector<ItemBytes> ib;
    if (cnt) cnt->assign(it.size(), 0);
    int blocks = 0;
    for (size_t k = 0; k < it.size(); ++k) {
        const Item& I = it[k];
        mg::VecSlot& s = sl[k];
        s = mg::VecSlot{};
        s.lv = I.c->outer_d[dir];
        s.block0 = blocks;
        s.gate = gate_of(R, gk, (int)k);
        const int nb = blocks_of(I.c, bk);
        // partial sums per slot: one per chunk of the Arnoldi passes, else
        // one per workgroup
        const int np = (bk == B_DOT || bk == B_MV) ? chunks_of(I.c, bk) : nb;
        s.nc = np;
        if (np > R.w->bstride) return MG_E_STATE;
        if (cnt) (*cnt)[k] = np;
        blocks += nb;
        ItemBytes b{(int)k, 0.0, 0.0};
        fill((int)k, s, b);
        ib.push_back(b);
    }
    mg::VecArgs a{};
    a.st.n = (int)sl.size();
    a.st.nblocks = blocks;
    a.part = R.w->part;
    a.rpart = R.w->rpart;
    a.pstride = HSTRIDE;
    a.bstride = R.w->bstride;
    const size_t off = put(*R.op, sl);
    add(R, cls, ib, [=](hipStream_t s, const char* base) {
        mg::VecArgs b = a;
        b.st.s = (const mg::VecSlot*)(base + off);
        return launch(b, s);
    });
    return MG_OK;
}

// y_k = f_k - A x_k (f_k null: A x_k) on level 0, with ||y_k||^2 partials.
mg_status rec_residual(Rec& R, int dir, const std::vector<Item>& it, int gk, const std::vector<const cx<double>*>& x,
                       const std::vector<const cx<double>*>& f, const std::vector<cx<double>*>& y, bool norm,
                       std::vector<int>* cnt) {
    const int dim = R.dim;
    return rec_vec(
        R, dir, it, gk, B_VEC, MG_K_RESIDUAL, cnt,
        [&](int k, mg::VecSlot& s, ItemBytes& b) {
            s.x = x[k];
            s.f = f[k];
            s.y = y[k];
            b.base = it[k].c->lv[0].N * (40.0 + (f[k] ? 16.0 : 0.0));
        },
        [=](mg::VecArgs b, hipStream_t s) {
            if (!norm) b.rpart = nullptr;
            return mg::launch_residual(dim, b, s);
        });
}

mg_status rec_norm(Rec& R, const std::vector<Item>& it, int gk, const std::vector<const cx<double>*>& x,
                   std::vector<int>* cnt) {
    return rec_vec(
        R, 0, it, gk, B_VEC, MG_K_OTHER, cnt,
        [&](int k, mg::VecSlot& s, ItemBytes& b) {
            s.x = x[k];
            b.base = it[k].c->lv[0].N * 16.0;
        },
        [](const mg::VecArgs& b, hipStream_t s) { return mg::launch_norm(b, s); });
}

mg_status rec_vzero(Rec& R, const std::vector<Item>& it, int gk, const std::vector<cx<double>*>& y) {
    return rec_vec(
        R, 0, it, gk, B_VEC, MG_K_OTHER, nullptr,
        [&](int k, mg::VecSlot& s, ItemBytes& b) {
            s.y = y[k];
            b.base = it[k].c->lv[0].N * 16.0;
        },
        [](const mg::VecArgs& b, hipStream_t s) { return mg::launch_vzero(b, s); });
}

// Fixed-order sum of the real partials of each item into w->rtot[k].
mg_status rec_reduce_real(Rec& R, const std::vector<int>& cnt) {
    const size_t off = put(*R.op, cnt);
    mg::ReduceArgs a{};
    a.rpart = R.w->rpart;
    a.rout = R.w->rtot;
    a.bstride = R.w->bstride;
    const int n = (int)cnt.size();
    add(R, MG_K_REDUCE, {}, [=](hipStream_t s, const char* base) {
        mg::ReduceArgs b = a;
        b.cnt = (const int*)(base + off);
        return mg::launch_reduce(b, n, true, s);
    });
    return MG_OK;
}

// Krylov control kernels, one workgroup per item; cnt: partials per item of
// the producing launch (slot k = item k).
mg_status rec_gm(Rec& R, int which, const std::vector<Item>& it, const std::vector<int>* cnt, int j) {
    std::vector<mg::GmItem> t(it.size());
    for (size_t k = 0; k < it.size(); ++k) {
        const Item& I = it[k];
        mg::GmItem& g = t[k];
        g.st = R.w->gst + k;
        g.fl = R.w->gfl + k;
        g.scale = I.c->scale_d + (size_t)I.rhs * HSTRIDE;
        g.coef = I.c->coef_d + (size_t)I.rhs * HSTRIDE;
        g.cnt = cnt ? (*cnt)[k] : 0;
        g.slot = (int)k;
    }
    mg::GmArgs a{};
    a.prm = R.w->prm;
    a.part = R.w->part;
    a.rpart = R.w->rpart;
    a.pstride = HSTRIDE;
    a.bstride = R.w->bstride;
    a.j = j;
    const size_t off = put(*R.op, t);
    const int n = (int)t.size();
    add(R, MG_K_REDUCE, {}, [=](hipStream_t s, const char* base) {
        mg::GmArgs b = a;
        b.it = (const mg::GmItem*)(base + off);
        return mg::launch_gm(which, n, b, s);
    });
    return MG_OK;
}

// ---------------------------------------------------------------------------
// GMRES(3) smoothing (Sec. 3.2.2): pre-smoothing at depth d ends in the
// restriction of its residual, post-smoothing starts from u1 + P e.
// ---------------------------------------------------------------------------

// Coefficient solve of slots of a Gram launch (partials per slot: cnt; the
// q-th slot solved is slot pslot[q] of the Gram launch, q itself when
// pslot is null).
void rec_coef(Rec& R, int d, int phase, const std::vector<Item>& it, const std::vector<int>& who,
              const std::vector<int>& cnt, int gk, const std::vector<int>* pslot = nullptr) {
    std::vector<mg::CoefSlot> cs(who.size());
    for (size_t q = 0; q < who.size(); ++q) {
        const Item& I = it[who[q]];
        cs[q].coef = gcoef_of(I.c, d, I.rhs, phase);
        cs[q].cnt = cnt[q];
        cs[q].pslot = pslot ? (*pslot)[q] : (int)q;
        cs[q].gate = gate_of(R, gk, who[q]);
    }
    mg::SmCoefArgs a{};
    a.part = R.w->part;
    a.pstride = HSTRIDE;
    a.bstride = R.w->bstride;
    const size_t off = put(*R.op, cs);
    const bool mixed = R.mixed;
    const int n = (int)cs.size();
    add(R, d == 0 ? MG_K_REDUCE : MG_K_COARSE_LEVELS, {}, [=](hipStream_t s, const char* base) {
        mg::SmCoefArgs b = a;
        b.s = (const mg::CoefSlot*)(base + off);
        return mg::launch_sm_coef(mixed, b, n, s);
    });
}

// Slot table of the pointwise 3D smoother passes; (*cnt)[q] partials.
mg_status sm_slots(Rec& R, int dir, int d, const std::vector<Item>& it, const std::vector<int>& who, int gk,
                   std::vector<mg::SmSlot>& sl, std::vector<int>& cnt, int& blocks) {
    sl.assign(who.size(), mg::SmSlot{});
    cnt.assign(who.size(), 0);
    blocks = 0;
    for (size_t q = 0; q < who.size(); ++q) {
        const Item& I = it[who[q]];
        mg::SmSlot& s = sl[q];
        s.lv = view_ptr(I.c, dir, d);
        s.sb = sbuf(I.c, d, I.rhs);
        s.gate = gate_of(R, gk, who[q]);
        s.block0 = blocks;
        const int nb = mg::vec_blocks(I.c->lv[d].N);
        if (nb > R.w->bstride) return MG_E_STATE;
        cnt[q] = nb;
        blocks += nb;
    }
    return MG_OK;
}

// 3D: powers, Gram partials and coefficients of one smoothing step (q0
// given by the slots' f or the q0 buffer).
mg_status rec_smooth_coef(Rec& R, int d, int phase, const std::vector<Item>& it, const std::vector<int>& who,
                          const std::vector<mg::SmSlot>& sl, const std::vector<int>& cnt, int blocks, bool q0f,
                          int gk) {
    const bool fine = d == 0;
    const double ct = R.mixed ? 8.0 : 16.0, sk = R.mixed ? 4.0 : 8.0;
    const double q0b = (fine && q0f) ? 16.0 : ct;
    std::vector<ItemBytes> ib1, ib2, ibg;
    for (int k : who) {
        const double n = (double)it[k].c->lv[d].N;
        ib1.push_back({k, n * (q0b + sk + ct), 0.0});
        ib2.push_back({k, n * (ct + sk + ct), 0.0});
        ibg.push_back({k, n * (q0b + 2.0 * ct + sk), 0.0});
    }
    mg::SmArgs a{};
    a.st.n = (int)sl.size();
    a.st.nblocks = blocks;
    a.part = R.w->part;
    a.pstride = HSTRIDE;
    a.bstride = R.w->bstride;
    const size_t off = put(*R.op, sl);
    const int dim = R.dim;
    const bool mixed = R.mixed;
    if (fine && dim == 3) {
        // the finest 3D level marches along z: its own workgroup count (and
        // Gram partial count) per slot
        std::vector<mg::SmSlot> slz(sl);
        std::vector<int> cz(who.size());
        int nbz = 0;
        for (size_t q = 0; q < who.size(); ++q) {
            slz[q].block0 = nbz;
            cz[q] = mg::power_z_tiles(it[who[q]].c->lv[d].n);
            if (cz[q] > R.w->bstride) return MG_E_STATE;
            nbz += cz[q];
        }
        mg::SmArgs az = a;
        az.st.nblocks = nbz;
        const size_t offz = put(*R.op, slz);
        for (int stage = 1; stage <= 2; ++stage)
            add(R, MG_K_SMOOTH_POWER_FINE, stage == 1 ? ib1 : ib2, [=](hipStream_t s, const char* base) {
                mg::SmArgs b = az;
                b.st.s = (const mg::SmSlot*)(base + offz);
                return mg::launch_sm_power_z(mixed, true, stage, b, s);
            });
        add(R, phase ? MG_K_SMOOTH_GRAM_POST_FINE : MG_K_SMOOTH_GRAM_FINE, ibg, [=](hipStream_t s, const char* base) {
            mg::SmArgs b = az;
            b.st.s = (const mg::SmSlot*)(base + offz);
            return mg::launch_sm_gram_z(mixed, true, b, s);
        });
        rec_coef(R, d, phase, it, who, cz, gk);
        return MG_OK;
    }
    for (int stage = 1; stage <= 2; ++stage)
        add(R, fine ? MG_K_SMOOTH_POWER_FINE : MG_K_COARSE_LEVELS, stage == 1 ? ib1 : ib2,
            [=](hipStream_t s, const char* base) {
                mg::SmArgs b = a;
                b.st.s = (const mg::SmSlot*)(base + off);
                return mg::launch_sm_power(dim, mixed, fine, stage, b, s);
            });
    add(R, fine ? (phase ? MG_K_SMOOTH_GRAM_POST_FINE : MG_K_SMOOTH_GRAM_FINE) : MG_K_COARSE_LEVELS, ibg,
        [=](hipStream_t s, const char* base) {
            mg::SmArgs b = a;
            b.st.s = (const mg::SmSlot*)(base + off);
            return mg::launch_sm_gram(dim, mixed, fine, b, s);
        });
    rec_coef(R, d, phase, it, who, cnt, gk);
    return MG_OK;
}

// 2D fused passes (mg_march2d.hip): Gram pass, coefficient solve, apply pass.
// On coarse levels with few tiles per rhs the apply pass forms the
// coefficients itself from the Gram partials (no separate solve launch).
// (The choice is per slot -- by its own tile count -- so that a batch
// launch forms every slot's coefficients as the single-context one does.)
bool fused_coef(int d, const std::vector<int>& cnt) {
    if (d == 0) return false;
    for (int n : cnt)
        if (n <= mg::FUSED_COEF_TILES) return true;
    return false;
}

// The coefficient solve launch for the slots the apply pass does not serve.
void rec_coef_rest(Rec& R, int d, int phase, const std::vector<Item>& it, const std::vector<int>& who,
                   const std::vector<int>& cnt, int gk) {
    std::vector<int> w2, c2, p2;
    for (size_t q = 0; q < who.size(); ++q)
        if (cnt[q] > mg::FUSED_COEF_TILES) {
            w2.push_back(who[q]);
            c2.push_back(cnt[q]);
            p2.push_back((int)q);
        }
    if (!w2.empty()) rec_coef(R, d, phase, it, w2, c2, gk, &p2);
}

void set_fused_coef(mg::CycleArgs& a, const Rec& R) {
    a.gpart = R.w->part;
    a.gpstride = HSTRIDE;
    a.gbstride = R.w->bstride;
    // an exhausted Krylov space shows as a relative Cholesky pivot at the
    // rounding level of the vectors' precision (as in the solve launch)
    a.gbrk = R.mixed ? 1e-5 : 1e-13;
}
mg_status rec_pre_2d(Rec& R, int dir, const std::vector<Item>& it, int gk, const std::vector<L0>* l0, int d,
                     bool nz, const std::vector<int>& who) {
    const int shape = launch_shape(it, who, d);
    const double ct = R.mixed ? 8.0 : 16.0, sk = R.mixed ? 4.0 : 8.0;
    std::vector<mg::CycleSlot> sl(who.size());
    std::vector<int> cnt(who.size());
    std::vector<ItemBytes> ibg, iba;
    int tiles = 0;
    for (size_t q = 0; q < who.size(); ++q) {
        const int k = who[q];
        const Item& I = it[k];
        mg_ctx* c = I.c;
        mg::CycleSlot& s = sl[q];
        s = mg::CycleSlot{};
        s.lv = view_ptr(c, dir, d);
        if (nz) {
            s.f = nullptr;
            s.fscale = 1.0;
            s.u = (*l0)[k].u;
        } else if (d == 0) {
            s.f = (*l0)[k].f;
            s.fscale = (*l0)[k].fs;
            s.fsp = (*l0)[k].fsp;
        } else {
            s.f = lvec(c, c->lv[d].F, d, I.rhs);
            s.fscale = 1.0;
        }
        s.c = lvec(c, c->lv[d + 1].F, d + 1, I.rhs);
        s.sb = sbuf(c, d, I.rhs);
        s.gate = gate_of(R, gk, k);
        s.tile0 = tiles;
        int nt[3];
        mg::march_counts(shape, c->lv[d].n, nt);
        cnt[q] = nt[0] * nt[1];
        if (cnt[q] > R.w->bstride) return MG_E_STATE;
        tiles += cnt[q];
        const double q0b = (d == 0 && !nz) ? 16.0 : ct;
        ibg.push_back({k, c->lv[d].N * (q0b + sk), 0.0});
        iba.push_back({k, c->lv[d].N * (q0b + sk + ct + (nz ? 16.0 : 0.0)) + c->lv[d + 1].N * ct, 0.0});
    }
    mg::CycleArgs a{};
    a.st.n = (int)sl.size();
    a.st.ntiles = tiles;
    const size_t off = put(*R.op, sl);
    const bool mixed = R.mixed;
    cx<double>* part = R.w->part;
    const int bstride = R.w->bstride;
    add(R, d == 0 ? MG_K_SMOOTH_GRAM_FINE : MG_K_COARSE_LEVELS, ibg, [=](hipStream_t s, const char* base) {
        mg::CycleArgs b = a;
        b.st.s = (const mg::CycleSlot*)(base + off);
        return mg::launch_sm2_gram(mixed, d == 0, false, shape, b, part, HSTRIDE, bstride, s);
    });
    mg::CycleArgs aa = a;
    if (fused_coef(d, cnt)) {
        set_fused_coef(aa, R);
        rec_coef_rest(R, d, 0, it, who, cnt, gk);
    } else {
        rec_coef(R, d, 0, it, who, cnt, gk);
    }
    add(R, d == 0 ? MG_K_SMOOTH_RESTRICT_FINE : MG_K_COARSE_LEVELS, iba, [=](hipStream_t s, const char* base) {
        mg::CycleArgs b = aa;
        b.st.s = (const mg::CycleSlot*)(base + off);
        return mg::launch_sm2_apply_restrict(mixed, d == 0, nz, shape, b, s);
    });
    return MG_OK;
}

mg_status rec_post_2d(Rec& R, int dir, const std::vector<Item>& it, int gk, const std::vector<L0>* l0, int d,
                      bool acc, const std::vector<int>& who) {
    const int shape = launch_shape(it, who, d);
    const double ct = R.mixed ? 8.0 : 16.0, sk = R.mixed ? 4.0 : 8.0;
    std::vector<mg::CycleSlot> sl(who.size());
    std::vector<int> cnt(who.size());
    std::vector<ItemBytes> ibg, iba;
    int tiles = 0;
    for (size_t q = 0; q < who.size(); ++q) {
        const int k = who[q];
        const Item& I = it[k];
        mg_ctx* c = I.c;
        mg::CycleSlot& s = sl[q];
        s = mg::CycleSlot{};
        s.lv = view_ptr(c, dir, d);
        if (d == 0) {
            s.f = (*l0)[k].f;
            s.fscale = (*l0)[k].fs;
            s.fsp = (*l0)[k].fsp;
            s.out = (*l0)[k].out;
        } else {
            s.f = lvec(c, c->lv[d].F, d, I.rhs);
            s.fscale = 1.0;
            s.out = lvec(c, c->lv[d].E, d, I.rhs);
        }
        s.c = lvec(c, c->lv[d + 1].E, d + 1, I.rhs);
        s.sb = sbuf(c, d, I.rhs);
        s.gate = gate_of(R, gk, k);
        s.tile0 = tiles;
        int nt[3];
        mg::march_counts(shape, c->lv[d].n, nt);
        cnt[q] = nt[0] * nt[1];
        if (cnt[q] > R.w->bstride) return MG_E_STATE;
        tiles += cnt[q];
        const double fb = d == 0 ? 16.0 : ct;
        ibg.push_back({k, c->lv[d].N * (ct + fb + sk) + c->lv[d + 1].N * ct, 0.0});
        iba.push_back({k, c->lv[d].N * (ct + fb + sk + fb + (d == 0 && acc ? 16.0 : 0.0)) + c->lv[d + 1].N * ct, 0.0});
    }
    mg::CycleArgs a{};
    a.st.n = (int)sl.size();
    a.st.ntiles = tiles;
    const size_t off = put(*R.op, sl);
    const bool mixed = R.mixed;
    cx<double>* part = R.w->part;
    const int bstride = R.w->bstride;
    const bool ac = d == 0 && acc;
    add(R, d == 0 ? MG_K_SMOOTH_GRAM_POST_FINE : MG_K_COARSE_LEVELS, ibg, [=](hipStream_t s, const char* base) {
        mg::CycleArgs b = a;
        b.st.s = (const mg::CycleSlot*)(base + off);
        return mg::launch_sm2_gram(mixed, d == 0, true, shape, b, part, HSTRIDE, bstride, s);
    });
    mg::CycleArgs aa = a;
    if (fused_coef(d, cnt)) {
        set_fused_coef(aa, R);
        rec_coef_rest(R, d, 1, it, who, cnt, gk);
    } else {
        rec_coef(R, d, 1, it, who, cnt, gk);
    }
    add(R, d == 0 ? MG_K_PROLONG_SMOOTH_FINE : MG_K_COARSE_LEVELS, iba, [=](hipStream_t s, const char* base) {
        mg::CycleArgs b = aa;
        b.st.s = (const mg::CycleSlot*)(base + off);
        return mg::launch_sm2_apply_out(mixed, d == 0, ac, shape, b, s);
    });
    return MG_OK;
}

// Pre-smoothing at depth d and restriction of its residual to depth d + 1.
// Level 0 with incoming iterates (FP64 only): q0 = f - A u by the FP64
// residual kernel, whose ||q0||^2 partials of item k land in rpart (cnt).
mg_status rec_pre_g(Rec& R, int dir, const std::vector<Item>& it, int gk, const std::vector<L0>* l0, int d,
                    bool norm, std::vector<int>* cnt) {
    const std::vector<int> who = above_tail(it, d);
    if (who.empty()) return MG_OK;
    const bool nz = d == 0 && l0 && (*l0)[0].u;
    if (nz && R.mixed) return MG_E_STATE;
    if (nz) {
        if (who.size() != it.size()) return MG_E_STATE;
        std::vector<const cx<double>*> xs(it.size()), fs(it.size());
        std::vector<cx<double>*> ys(it.size());
        for (size_t k = 0; k < it.size(); ++k) {
            const L0& z = (*l0)[k];
            if (z.fs != 1.0 || z.fsp) return MG_E_STATE;
            xs[k] = z.u;
            fs[k] = (const cx<double>*)z.f;
            ys[k] = (cx<double>*)lvec(it[k].c, it[k].c->lv[0].Q[0], 0, it[k].rhs);
        }
        CKS(rec_residual(R, dir, it, gk, xs, fs, ys, norm, cnt));
    }
    if (R.dim == 2) return rec_pre_2d(R, dir, it, gk, l0, d, nz, who);
    std::vector<mg::SmSlot> ss;
    std::vector<int> scnt;
    int blocks = 0;
    CKS(sm_slots(R, dir, d, it, who, gk, ss, scnt, blocks));
    for (size_t q = 0; q < who.size(); ++q) {
        const int k = who[q];
        const Item& I = it[k];
        mg::SmSlot& s = ss[q];
        if (nz) {
            s.f = nullptr;
            s.fscale = 1.0;
        } else if (d == 0) {
            s.f = (*l0)[k].f;
            s.fscale = (*l0)[k].fs;
            s.fsp = (*l0)[k].fsp;
        } else {
            s.f = lvec(I.c, I.c->lv[d].F, d, I.rhs);
            s.fscale = 1.0;
        }
    }
    CKS(rec_smooth_coef(R, d, 0, it, who, ss, scnt, blocks, !nz, gk));
    const int shape = launch_shape(it, who, d);
    const double ct = R.mixed ? 8.0 : 16.0, sk = R.mixed ? 4.0 : 8.0;
    std::vector<mg::CycleSlot> sl(who.size());
    std::vector<ItemBytes> ib;
    int tiles = 0;
    for (size_t q = 0; q < who.size(); ++q) {
        const int k = who[q];
        const Item& I = it[k];
        mg_ctx* c = I.c;
        mg::CycleSlot& s = sl[q];
        s = mg::CycleSlot{};
        s.lv = ss[q].lv;
        s.f = ss[q].f;
        s.fscale = ss[q].fscale;
        s.fsp = ss[q].fsp;
        s.u = nz ? (const void*)(*l0)[k].u : nullptr;
        s.c = lvec(c, c->lv[d + 1].F, d + 1, I.rhs);
        s.sb = sbuf(c, d, I.rhs);
        s.gate = ss[q].gate;
        s.tile0 = tiles;
        if (d == 0) {   // the finest level marches along z
            tiles += mg::power_z_tiles(c->lv[d].n);
        } else {
            int nt[3];
            mg::tile_counts(R.dim, shape, c->lv[d].n, nt);
            tiles += nt[0] * nt[1] * nt[2];
        }
        const double q0b = (d == 0 && !nz) ? 16.0 : ct;
        ib.push_back({k, c->lv[d].N * (q0b + 3.0 * ct + sk + (nz ? 16.0 : 0.0)) + c->lv[d + 1].N * ct, 0.0});
    }
    mg::CycleArgs a{};
    a.st.n = (int)sl.size();
    a.st.ntiles = tiles;
    const size_t off = put(*R.op, sl);
    const int dim = R.dim;
    const bool mixed = R.mixed;
    add(R, d == 0 ? MG_K_SMOOTH_RESTRICT_FINE : MG_K_COARSE_LEVELS, ib, [=](hipStream_t s, const char* base) {
        mg::CycleArgs b = a;
        b.st.s = (const mg::CycleSlot*)(base + off);
        if (d == 0) return mg::launch_sm_apply_restrict_z(mixed, nz, b, s);
        return mg::launch_sm_apply_restrict(dim, mixed, d == 0, nz, shape, b, s);
    });
    return MG_OK;
}

// Coarse-grid correction and post-smoothing at depth d.
mg_status rec_post_g(Rec& R, int dir, const std::vector<Item>& it, int gk, const std::vector<L0>* l0, int d,
                     bool acc) {
    const std::vector<int> who = above_tail(it, d);
    if (who.empty()) return MG_OK;
    if (R.dim == 2) return rec_post_2d(R, dir, it, gk, l0, d, acc, who);
    const int shape = launch_shape(it, who, d);
    const double ct = R.mixed ? 8.0 : 16.0, sk = R.mixed ? 4.0 : 8.0;
    std::vector<mg::CycleSlot> sl(who.size());
    std::vector<ItemBytes> ib;
    int tiles = 0;
    for (size_t q = 0; q < who.size(); ++q) {
        const int k = who[q];
        const Item& I = it[k];
        mg_ctx* c = I.c;
        mg::CycleSlot& s = sl[q];
        s = mg::CycleSlot{};
        s.lv = view_ptr(c, dir, d);
        if (d == 0) {
            s.f = (*l0)[k].f;
            s.fscale = (*l0)[k].fs;
            s.fsp = (*l0)[k].fsp;
        } else {
            s.f = lvec(c, c->lv[d].F, d, I.rhs);
            s.fscale = 1.0;
        }
        s.c = lvec(c, c->lv[d + 1].E, d + 1, I.rhs);
        s.sb = sbuf(c, d, I.rhs);
        s.gate = gate_of(R, gk, k);
        s.tile0 = tiles;
        int nt[3];
        mg::tile_counts(R.dim, shape, c->lv[d].n, nt);
        tiles += nt[0] * nt[1] * nt[2];
        ib.push_back({k, c->lv[d].N * (ct + (d == 0 ? 16.0 : ct) + sk + 2.0 * ct) + c->lv[d + 1].N * ct, 0.0});
    }
    mg::CycleArgs a{};
    a.st.n = (int)sl.size();
    a.st.ntiles = tiles;
    const size_t off = put(*R.op, sl);
    const int dim = R.dim;
    const bool mixed = R.mixed;
    add(R, d == 0 ? MG_K_PROLONG_SMOOTH_FINE : MG_K_COARSE_LEVELS, ib, [=](hipStream_t s, const char* base) {
        mg::CycleArgs b = a;
        b.st.s = (const mg::CycleSlot*)(base + off);
        return mg::launch_sm_prolong_resid(dim, mixed, d == 0, shape, b, s);
    });
    std::vector<mg::SmSlot> ss;
    std::vector<int> scnt;
    int blocks = 0;
    CKS(sm_slots(R, dir, d, it, who, gk, ss, scnt, blocks));
    CKS(rec_smooth_coef(R, d, 1, it, who, ss, scnt, blocks, false, gk));
    std::vector<ItemBytes> ibo;
    for (size_t q = 0; q < who.size(); ++q) {
        const int k = who[q];
        const Item& I = it[k];
        mg_ctx* c = I.c;
        ss[q].out = d == 0 ? (void*)(*l0)[k].out : lvec(c, c->lv[d].E, d, I.rhs);
        ibo.push_back({k, c->lv[d].N * (4.0 * ct + (d == 0 ? 16.0 : ct) + (d == 0 && acc ? 16.0 : 0.0)), 0.0});
    }
    mg::SmArgs sa{};
    sa.st.n = (int)ss.size();
    sa.st.nblocks = blocks;
    const size_t off2 = put(*R.op, ss);
    const bool ac = d == 0 && acc;
    add(R, d == 0 ? MG_K_PROLONG_SMOOTH_FINE : MG_K_COARSE_LEVELS, ibo, [=](hipStream_t s, const char* base) {
        mg::SmArgs b = sa;
        b.st.s = (const mg::SmSlot*)(base + off2);
        return mg::launch_sm_apply_out(mixed, d == 0, ac, b, s);
    });
    return MG_OK;
}

// The descending / ascending halves of one level's cycle work.
mg_status rec_down(Rec& R, int dir, const std::vector<Item>& it, int gk, const std::vector<L0>* l0, int d, bool norm,
                   std::vector<int>* cnt) {
    return it[0].c->gsmooth ? rec_pre_g(R, dir, it, gk, l0, d, norm, cnt) : rec_ka(R, dir, it, gk, l0, d, norm, cnt);
}
mg_status rec_up(Rec& R, int dir, const std::vector<Item>& it, int gk, const std::vector<L0>* l0, int d, bool acc) {
    return it[0].c->gsmooth ? rec_post_g(R, dir, it, gk, l0, d, acc) : rec_kb(R, dir, it, gk, l0, d, acc);
}

// One V(1,1) cycle for the items, gated by gk.  With norms (and incoming
// iterates) the ||f - A u||^2 partials of item k land in rpart, (*cnt)[k].
mg_status rec_cycle(Rec& R, int dir, const std::vector<Item>& it, int gk, const std::vector<L0>& l0, bool acc,
                    bool norms, std::vector<int>* cnt) {
    if (R.mixed && l0[0].u) return MG_E_STATE;
    int maxT = 0;
    for (const Item& I : it) maxT = std::max(maxT, I.c->lt);
    CKS(rec_down(R, dir, it, gk, &l0, 0, norms, cnt));
    for (int d = 1; d < maxT; ++d) CKS(rec_down(R, dir, it, gk, nullptr, d, false, nullptr));
    CKS(rec_tail(R, dir, it, gk));
    for (int d = maxT - 1; d >= 1; --d) CKS(rec_up(R, dir, it, gk, nullptr, d, false));
    CKS(rec_up(R, dir, it, gk, &l0, 0, acc));
    return MG_OK;
}
// ---------------------------------------------------------------------------
// Arnoldi passes (Sec. 4.1: one cycle per outer step)
// ---------------------------------------------------------------------------
cx<double>* basis(const Item& I, int i) {
    mg_ctx* c = I.c;
    return c->V + ((size_t)I.rhs * c->vstride + i) * c->lv[0].N;
}
cx<double>* zbasis(const Item& I, int i) {
    mg_ctx* c = I.c;
    return c->Zb + ((size_t)I.rhs * c->zstride + i) * c->lv[0].N;
}
cx<double>* wvec(const Item& I) { return I.c->W + (size_t)I.rhs * I.c->lv[0].N; }
cx<double>* zvec(const Item& I) { return I.c->Z + (size_t)I.rhs * I.c->lv[0].N; }
double* scale_of(const Item& I) { return I.c->scale_d + (size_t)I.rhs * HSTRIDE; }

// Pass 1 of step j: w = A z, partials of h1 = V^H w.
mg_status rec_matvec_dot(Rec& R, int dir, const std::vector<Item>& it, int gk, bool flexible, int j,
                         std::vector<int>* cnt) {
    const int dim = R.dim;
    return rec_vec(
        R, dir, it, gk, B_MV, MG_K_MATVEC_DOT, cnt,
        [&](int k, mg::VecSlot& s, ItemBytes& b) {
            const Item& I = it[k];
            s.x = flexible ? zbasis(I, j) : zvec(I);
            s.y = wvec(I);
            s.V = basis(I, 0);
            s.scale = scale_of(I);
            s.j = j;
            const double N = (double)I.c->lv[0].N;
            b.base = N * (16.0 * (j + 1) + 16.0 + 8.0 + 16.0);
        },
        [=](const mg::VecArgs& b, hipStream_t s) { return mg::launch_matvec_dot(dim, j + 1, b, s); });
}

// Pass 2 of step j: V_{j+1} = w - V h, partials of V^H V_{j+1}, ||V_{j+1}||^2.
mg_status rec_update_gram(Rec& R, int dir, const std::vector<Item>& it, int gk, int j, std::vector<int>* cnt) {
    return rec_vec(
        R, dir, it, gk, B_DOT, MG_K_UPDATE_DOT, cnt,
        [&](int k, mg::VecSlot& s, ItemBytes& b) {
            const Item& I = it[k];
            s.y = wvec(I);
            s.V = basis(I, 0);
            s.scale = scale_of(I);
            s.hin = R.w->gst[k].h;
            s.j = j;
            const double N = (double)I.c->lv[0].N;
            b.base = N * (16.0 * (j + 1) + 16.0 + 16.0);
        },
        [=](const mg::VecArgs& b, hipStream_t s) { return mg::launch_update_gram(j + 1, b, s); });
}

// End of a restart cycle: t = sum_i coef_i V_i into W (flexible: x +=
// sum_i coef_i Z_i), over the basis vectors the cycle built.
mg_status rec_combine(Rec& R, const std::vector<Item>& it, int gk, const std::vector<cx<double>*>& X, bool flexible,
                      int m) {
    return rec_vec(
        R, 0, it, gk, B_VEC, MG_K_COMBINE, nullptr,
        [&](int k, mg::VecSlot& s, ItemBytes& b) {
            const Item& I = it[k];
            s.V = flexible ? zbasis(I, 0) : basis(I, 0);
            s.coef = I.c->coef_d + (size_t)I.rhs * HSTRIDE;
            s.y = flexible ? X[k] : wvec(I);
            s.jp = &R.w->gfl[k].kk;
            const double N = (double)I.c->lv[0].N;
            b.base = N * (16.0 + (flexible ? 16.0 : 0.0));
            b.per = N * 16.0;
        },
        [=](const mg::VecArgs& b, hipStream_t s) { return mg::launch_combine(m, flexible, b, s); });
}

// ---------------------------------------------------------------------------
// Solver operations.  GMRES: an initial operation (||f||, zero right-hand
// sides, first residual) and one restart cycle (m steps for every item,
// items that stop early gated off, then the solution update and the new
// residual).  Standalone: an initial operation and a chunk of cycles with
// the stop test after each.
// ---------------------------------------------------------------------------
mg_status rec_gmres_init(Rec& R, int dir, const std::vector<Item>& it, const std::vector<cx<double>*>& X,
                         const std::vector<const cx<double>*>& F) {
    R.tag = TAG_ALWAYS;
    std::vector<int> c1, c2;
    CKS(rec_norm(R, it, G_NONE, F, &c1));
    CKS(rec_gm(R, mg::GM_INIT, it, &c1, 0));
    CKS(rec_vzero(R, it, G_ZERO, X));
    std::vector<const cx<double>*> xs(X.begin(), X.end());
    std::vector<cx<double>*> v0(it.size());
    for (size_t k = 0; k < it.size(); ++k) v0[k] = basis(it[k], 0);
    CKS(rec_residual(R, dir, it, G_FIN, xs, F, v0, true, &c2));
    CKS(rec_gm(R, mg::GM_RESTART, it, &c2, 0));
    return MG_OK;
}

mg_status rec_gmres_cycle(Rec& R, int dir, const std::vector<Item>& it, const std::vector<cx<double>*>& X,
                          const std::vector<const cx<double>*>& F, int m, bool flexible) {
    const size_t n = it.size();
    for (int j = 0; j < m; ++j) {
        R.tag = j;
        std::vector<L0> l0(n);
        for (size_t k = 0; k < n; ++k)
            l0[k] = L0{basis(it[k], j), 1.0, scale_of(it[k]) + j, nullptr, flexible ? zbasis(it[k], j) : zvec(it[k])};
        CKS(rec_cycle(R, dir, it, G_LIVE, l0, false, false, nullptr));
        if (j == 0) R.op->mark = (int)R.op->steps.size() - 1;
        std::vector<int> c1, c2;
        CKS(rec_matvec_dot(R, dir, it, G_LIVE, flexible, j, &c1));
        CKS(rec_gm(R, mg::GM_H, it, &c1, j));
        CKS(rec_update_gram(R, dir, it, G_LIVE, j, &c2));
        CKS(rec_gm(R, mg::GM_COL, it, &c2, j));
    }
    R.tag = TAG_FIN;
    CKS(rec_combine(R, it, G_FIN, X, flexible, m));
    if (!flexible) {
        std::vector<L0> l0(n);
        for (size_t k = 0; k < n; ++k) l0[k] = L0{wvec(it[k]), 1.0, nullptr, nullptr, X[k]};
        CKS(rec_cycle(R, dir, it, G_FIN, l0, true, false, nullptr));
    }
    std::vector<const cx<double>*> xs(X.begin(), X.end());
    std::vector<cx<double>*> v0(n);
    for (size_t k = 0; k < n; ++k) v0[k] = basis(it[k], 0);
    std::vector<int> c3;
    CKS(rec_residual(R, dir, it, G_FIN, xs, F, v0, true, &c3));
    CKS(rec_gm(R, mg::GM_RESTART, it, &c3, 0));
    return MG_OK;
}

mg_status rec_sa_init(Rec& R, const std::vector<Item>& it, const std::vector<cx<double>*>& U,
                      const std::vector<const cx<double>*>& F) {
    R.tag = TAG_ALWAYS;
    std::vector<int> c1;
    CKS(rec_norm(R, it, G_NONE, F, &c1));
    CKS(rec_gm(R, mg::SA_INIT, it, &c1, 0));
    CKS(rec_vzero(R, it, G_ZERO, U));
    return MG_OK;
}

// Standalone (Sec. 4.1, LVL-MG): the residual of the incoming iterate is
// formed inside the first fused kernel of each cycle (FP64), or by the FP64
// residual of the refinement step u <- u + M (f - A u) (mixed precision,
// fixed-shift cycle); the stop test follows the cycle.
mg_status rec_sa_chunk(Rec& R, int dir, const std::vector<Item>& it, const std::vector<cx<double>*>& U,
                       const std::vector<const cx<double>*>& F, int K) {
    const size_t n = it.size();
    const bool direct = !R.mixed && !it[0].c->shifted0;
    for (int q = 0; q < K; ++q) {
        R.tag = q;
        std::vector<int> cnt;
        std::vector<L0> l0(n);
        if (direct) {
            for (size_t k = 0; k < n; ++k) l0[k] = L0{F[k], 1.0, nullptr, U[k], U[k]};
            CKS(rec_cycle(R, dir, it, G_LIVE, l0, false, true, &cnt));
        } else {
            std::vector<const cx<double>*> xs(U.begin(), U.end());
            std::vector<cx<double>*> ws(n);
            for (size_t k = 0; k < n; ++k) ws[k] = wvec(it[k]);
            CKS(rec_residual(R, dir, it, G_LIVE, xs, F, ws, true, &cnt));
            for (size_t k = 0; k < n; ++k) l0[k] = L0{ws[k], 1.0, nullptr, nullptr, U[k]};
            CKS(rec_cycle(R, dir, it, G_LIVE, l0, true, false, nullptr));
        }
        CKS(rec_gm(R, mg::SA_STEP, it, &cnt, 0));
    }
    return MG_OK;
}

mg_status ensure_basis(mg_ctx* c, int restart, bool flexible) {
    if (!c->V || c->vstride < restart + 1) {
        CK(hipStreamSynchronize(c->stream));
        dfree(c->V);
        c->vstride = 0;
        const size_t bytes = (size_t)c->nrhs * (restart + 1) * c->lv[0].N * sizeof(cx<double>);
        CKS(dalloc(&c->V, bytes));
        c->vstride = restart + 1;
        c->gen++;
        cache_clear(c->cache);
    }
    if (flexible && (!c->Zb || c->zstride < restart)) {
        CK(hipStreamSynchronize(c->stream));
        dfree(c->Zb);
        c->zstride = 0;
        const size_t bytes = (size_t)c->nrhs * restart * c->lv[0].N * sizeof(cx<double>);
        CKS(dalloc(&c->Zb, bytes));
        c->zstride = restart;
        c->gen++;
        cache_clear(c->cache);
    }
    return MG_OK;
}

// Sweep schedule of the Arnoldi passes: points per thread (so workgroups
// per right-hand side), picked by timing both passes at a mid-restart step
// on the context's own basis.  The choice depends on the context only, so a
// batch reduces in the same order as a single solve.
mg_status tune_arnoldi(mg_ctx* c, int m) {
    if (c->vtuned) return MG_OK;
    c->vtuned = true;
    const int j = std::min(8, m - 1);
    static const int cand[3] = {64, 32, 16};
    std::vector<Item> it;
    for (int r = 0; r < c->nrhs; ++r) it.push_back(Item{c, r});
    hipEvent_t e0, e1;
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    Exec E{c->stream, nullptr, nullptr, false};
    float best = 1e30f;
    int pick = c->vper;
    mg_status st = MG_OK;
    for (int per : cand) {
        c->vper = per;
        Op op;
        Rec R{&op, &c->work, c->dim, c->mixed, TAG_ALWAYS};
        st = rec_matvec_dot(R, 0, it, G_NONE, c->Zb != nullptr && c->zstride > j, j, nullptr);
        if (st == MG_OK) st = rec_update_gram(R, 0, it, G_NONE, j, nullptr);
        if (st != MG_OK) {   // the work space does not hold this split
            st = MG_OK;
            op_release(op);
            continue;
        }
        float tot = 0.0f;
        for (int rep = 0; rep < 4 && st == MG_OK; ++rep) {
            if (hipEventRecord(e0, c->stream) != hipSuccess) st = MG_E_DEVICE;
            if (st == MG_OK) st = op_run(E, op);
            if (st == MG_OK && hipEventRecord(e1, c->stream) != hipSuccess) st = MG_E_DEVICE;
            if (st == MG_OK && hipEventSynchronize(e1) != hipSuccess) st = MG_E_DEVICE;
            float ms = 0.0f;
            if (st == MG_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = MG_E_DEVICE;
            if (rep > 0) tot += ms;
        }
        op_release(op);
        if (st != MG_OK) break;
        if (tot < 0.97f * best) {
            best = tot;
            pick = per;
        }
    }
    c->vper = pick;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

std::vector<uintptr_t> item_key(int kind, int dir, const std::vector<Item>& it, const std::vector<cx<double>*>& U,
                                const std::vector<const cx<double>*>& F) {
    std::vector<uintptr_t> key{(uintptr_t)kind, (uintptr_t)dir};
    for (size_t k = 0; k < it.size(); ++k) {
        key.push_back((uintptr_t)it[k].c);
        key.push_back((uintptr_t)it[k].rhs);
        key.push_back((uintptr_t)it[k].c->gen);
        key.push_back((uintptr_t)it[k].c->vper);
        key.push_back((uintptr_t)U[k]);
        key.push_back((uintptr_t)F[k]);
    }
    return key;
}

enum OpKind { K_GM_INIT = 1, K_GM_CYCLE = 2, K_SA_INIT = 3, K_SA_CHUNK = 4, K_CYCLE = 5, K_APPLY = 6 };
constexpr int SA_CHUNK = 8;   // standalone cycles per operation

mg_status read_flags(Exec& E, Work& w, int n) {
    CK(hipMemcpyAsync(w.gfl_h, w.gfl, (size_t)n * sizeof(mg::GmFlags), hipMemcpyDeviceToHost, E.s));
    CK(hipStreamSynchronize(E.s));
    return MG_OK;
}

// Items of a solve that share a work space and a stream.  Several groups
// of one solve run concurrently, each on its own stream: the body of group
// g > 0 starts once group g - 1 has finished the first cycle of its restart
// cycle, so one group's latency-bound coarse levels overlap another's
// bandwidth-bound Arnoldi passes.  Every launch of a group covers only its
// items, and each item's sums keep their order (partials per item), so the
// results do not depend on the grouping.
struct Group {
    Exec E;
    Work* w;
    std::vector<Item> it;
    std::vector<cx<double>*> U;
    std::vector<const cx<double>*> F;
    int off = 0;   // position of the group's first item among the solve's items
    Op* init = nullptr;
    Op* body = nullptr;
};

// Solve for the items: device-driven (F)GMRES(m) or standalone cycles.
mg_status solve_groups(std::vector<Group>& G, int dir, int mode, double rtol, int maxit, int restart, int* iters,
                       double* hist) {
    if (maxit < 0 || !(rtol >= 0.0)) return MG_E_INVAL;
    if (G.empty() || G[0].it.empty()) return MG_E_INVAL;
    const bool gm = mode == MG_MODE_GMRES || mode == MG_MODE_FGMRES;
    if (!gm && mode != MG_MODE_STANDALONE) return MG_E_INVAL;
    if (gm && (restart < 1 || restart > MAX_RESTART)) return MG_E_INVAL;
    for (const Group& g : G) {
        if ((int)g.it.size() > g.w->items || g.it.empty()) return MG_E_STATE;
        if (G.size() > 1 && (profiling(g.E) || !g.E.graphs)) return MG_E_STATE;
    }
    const Item& I0 = G[0].it[0];
    const bool flexible = gm && (mode == MG_MODE_FGMRES || I0.c->gsmooth);
    const int dim = I0.c->dim;
    const bool mixed = I0.c->mixed;
    for (const Group& g : G) CK(hipStreamSynchronize(g.E.s));
    if (gm)
        for (const Group& g : G)
            for (const Item& I : g.it) {
                CKS(ensure_basis(I.c, restart, flexible));
                CKS(tune_arnoldi(I.c, restart));
            }
    const size_t hstride = (size_t)maxit + 1;
    for (Group& g : G) {
        Work& w = *g.w;
        const int n = (int)g.it.size();
        CKS(ensure_hist(w, (size_t)n * hstride));
        *w.prm_h = mg::GmParams{rtol, w.hist, (int)hstride, maxit, gm ? restart : 0, flexible ? 1 : 0};
        CK(hipMemcpyAsync(w.prm, w.prm_h, sizeof(mg::GmParams), hipMemcpyHostToDevice, g.E.s));
        std::vector<uintptr_t> k0 = item_key(gm ? K_GM_INIT : K_SA_INIT, dir, g.it, g.U, g.F);
        std::vector<uintptr_t> k1 = item_key(gm ? K_GM_CYCLE : K_SA_CHUNK, dir, g.it, g.U, g.F);
        if (gm) {
            k1.push_back((uintptr_t)restart);
            k1.push_back((uintptr_t)flexible);
        }
        CKS(cached(*g.E.cache, k0, &g.init, [&](Op& op) {
            Rec R{&op, &w, dim, mixed, TAG_ALWAYS};
            return gm ? rec_gmres_init(R, dir, g.it, g.U, g.F) : rec_sa_init(R, g.it, g.U, g.F);
        }));
        CKS(cached(*g.E.cache, k1, &g.body, [&](Op& op) {
            Rec R{&op, &w, dim, mixed, TAG_ALWAYS};
            return gm ? rec_gmres_cycle(R, dir, g.it, g.U, g.F, restart, flexible)
                      : rec_sa_chunk(R, dir, g.it, g.U, g.F, SA_CHUNK);
        }));
    }
    for (Group& g : G) CKS(op_run(g.E, *g.init));
    for (Group& g : G) CKS(read_flags(g.E, *g.w, (int)g.it.size()));
    if (G.size() == 1) {
        std::vector<int> live(G[0].it.size(), 0);
        CKS(op_collect(G[0].E, *G[0].init, &live));
    }
    std::vector<int> before, live, sbefore;
    // every run of the bodies advances each running item by at least one step
    const long long guard = (long long)maxit + 2;
    for (long long run = 0;; ++run) {
        std::vector<char> act(G.size(), 0);
        bool any = false;
        for (size_t q = 0; q < G.size(); ++q)
            for (size_t k = 0; k < G[q].it.size(); ++k) {
                const mg::GmFlags& f = G[q].w->gfl_h[k];
                if (gm ? f.state == 0 : f.live != 0) act[q] = 1;
            }
        for (char a : act) any = any || a;
        if (!any) break;
        if (run >= guard) return MG_E_STATE;
        if (G.size() == 1) {
            const Group& g = G[0];
            const int n = (int)g.it.size();
            before.assign(n, 0);
            sbefore.assign(n, 0);
            for (int k = 0; k < n; ++k) {
                before[k] = g.w->gfl_h[k].its;
                sbefore[k] = g.w->gfl_h[k].state;
            }
        }
        for (size_t q = 0; q < G.size(); ++q) {
            if (!act[q]) continue;
            if (q > 0 && act[q - 1] && G[q - 1].body->mark_ev)
                CK(hipStreamWaitEvent(G[q].E.s, G[q - 1].body->mark_ev, 0));
            CKS(op_run(G[q].E, *G[q].body));
        }
        for (Group& g : G) CKS(read_flags(g.E, *g.w, (int)g.it.size()));
        if (G.size() == 1 && profiling(G[0].E)) {
            Group& g = G[0];
            const int n = (int)g.it.size();
            live.assign(n, 0);
            for (int k = 0; k < n; ++k) {
                const mg::GmFlags& f = g.w->gfl_h[k];
                live[k] = f.its - before[k];
                if (!gm && sbefore[k] == 0 && (f.state == 1 || f.state == 3)) live[k]++;
            }
            CKS(op_collect(g.E, *g.body, &live));
        }
    }
    for (Group& g : G)
        if (hist)
            CK(hipMemcpyAsync(hist + (size_t)g.off * hstride, g.w->hist, g.it.size() * hstride * sizeof(double),
                              hipMemcpyDeviceToHost, g.E.s));
    for (Group& g : G) CK(hipStreamSynchronize(g.E.s));
    mg_status ret = MG_OK;
    for (const Group& g : G)
        for (size_t k = 0; k < g.it.size(); ++k) {
            const mg::GmFlags& f = g.w->gfl_h[k];
            if (iters) iters[g.off + k] = f.its;
            const int state = (!gm && f.state == 0) ? 2 : f.state;
            if (state == 3) ret = MG_E_DIVERGED;
            else if (state == 2 && ret == MG_OK) ret = MG_NOT_CONVERGED;
        }
    return ret;
}

mg_status solve_items(Exec& E, Work& w, int dir, const std::vector<Item>& it, const std::vector<cx<double>*>& U,
                      const std::vector<const cx<double>*>& F, int mode, double rtol, int maxit, int restart,
                      int* iters, double* hist) {
    std::vector<Group> G(1, Group{E, &w, it, U, F, 0, nullptr, nullptr});
    return solve_groups(G, dir, mode, rtol, maxit, restart, iters, hist);
}

// Splits the items of a multi-rhs (F)GMRES solve into up to SOLVE_GROUPS
// groups of about equal points, in order; group 0 runs on E with w, group
// g > 0 on streamg[g - 1] with workg[g - 1] (both created or grown here).
mg_status make_groups(const Exec& E, Work& w, Work* workg, hipStream_t* streamg, const std::vector<Item>& it,
                      const std::vector<cx<double>*>& U, const std::vector<const cx<double>*>& F,
                      std::vector<Group>& G) {
    const int n = (int)it.size();
    const int ng = std::min(n, SOLVE_GROUPS);
    double tot = 0.0;
    for (const Item& I : it) tot += (double)I.c->lv[0].N;
    std::vector<int> cut(ng + 1, n);
    cut[0] = 0;
    double acc = 0.0;
    int g = 1;
    for (int k = 0; k < n && g < ng; ++k) {
        acc += (double)it[k].c->lv[0].N;
        // close group g - 1 after item k once it holds its share, leaving
        // at least one item for each later group
        if (acc >= tot * g / ng - 0.5 && n - (k + 1) >= ng - g) cut[g++] = k + 1;
    }
    for (; g < ng; ++g) cut[g] = std::max(cut[g - 1] + 1, n - (ng - g));
    for (int q = 0; q < ng; ++q) {
        const int lo = cut[q], hi = cut[q + 1];
        if (hi <= lo) return MG_E_STATE;
        Exec Eg = E;
        Work* wg = &w;
        if (q > 0) {
            hipStream_t& sg = streamg[q - 1];
            Work& wq = workg[q - 1];
            if (!sg) CK(hipStreamCreateWithFlags(&sg, hipStreamNonBlocking));
            if (wq.items < hi - lo || wq.bstride != w.bstride) {
                CK(hipStreamSynchronize(sg));
                work_free(wq);
                CKS(work_alloc(wq, hi - lo, w.bstride));
            }
            Eg.s = sg;
            wg = &wq;
        }
        G.push_back(Group{Eg, wg, std::vector<Item>(it.begin() + lo, it.begin() + hi),
                          std::vector<cx<double>*>(U.begin() + lo, U.begin() + hi),
                          std::vector<const cx<double>*>(F.begin() + lo, F.begin() + hi), lo, nullptr, nullptr});
    }
    return MG_OK;
}

Exec ctx_exec(mg_ctx* c) { return Exec{c->stream, &c->prof, &c->cache, true}; }

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
    Exec E = ctx_exec(c);
    const bool gm = mode == MG_MODE_GMRES || mode == MG_MODE_FGMRES;
    if (!gm || c->nrhs < 2 || profiling(E))
        return solve_items(E, c->work, dir, it, U, F, mode, rtol, maxit, restart, iters, hist);
    std::vector<Group> G;
    CKS(make_groups(E, c->work, c->workg, c->streamg, it, U, F, G));
    return solve_groups(G, dir, mode, rtol, maxit, restart, iters, hist);
}
// The GMRES(3) smoother's buffer table of a context (pointers per rhs and
// level).
std::vector<mg::SmoothBufs> smooth_table(const mg_ctx* c) {
    const int L = c->L;
    std::vector<mg::SmoothBufs> sb((size_t)c->nrhs * L);
    for (int l = 0; l < L; ++l) {
        const Level& V = c->lv[l];
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
    return sb;
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free cycle: one file-scope device array per GPU
// (kept until the process ends).  Host code uses the address obtained from
// hipGetSymbolAddress on that device, never the array's name.
// ---------------------------------------------------------------------------
constexpr size_t SCRATCH_BYTES = (size_t)64 << 20;
constexpr size_t STAGE_BYTES = (size_t)1 << 20;
constexpr int MAX_DEVICES = 64;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];
void* scratch_ptr[MAX_DEVICES] = {};

// Address of this device's scratch (the device is current).
mg_status scratch_init(int dev) {
    if (dev < 0 || dev >= MAX_DEVICES) return MG_E_DEVICE;
    if (scratch_ptr[dev]) return MG_OK;
    void* p = nullptr;
    CK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return MG_E_DEVICE;
    scratch_ptr[dev] = p;
    return MG_OK;
}

// ---------------------------------------------------------------------------
// Set-up
// ---------------------------------------------------------------------------
void release(mg_ctx* c) {
    if (!c) return;
    cache_free(c->cache);
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
        dfree(c->cinv[d]);
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
    hfree(c->stage);
    if (c->stage_ev) (void)hipEventDestroy(c->stage_ev);
    c->stage_ev = nullptr;
    work_free(c->work);
    for (int g = 0; g < SOLVE_GROUPS - 1; ++g) {
        work_free(c->workg[g]);
        if (c->streamg[g]) (void)hipStreamDestroy(c->streamg[g]);
        c->streamg[g] = nullptr;
    }
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
                a.cinv = b.cinv = c->cinv[dir];
            }
        }
        CKS(dalloc(&c->views_d[dir], vd.size() * sizeof(LevelView<double>)));
        CK(hipMemcpy(c->views_d[dir], vd.data(), vd.size() * sizeof(LevelView<double>), hipMemcpyHostToDevice));
        LevelView<double> outer = vd[0];   // residuals and Krylov steps: the problem's own operator
        outer.sigma = mg::mk(1.0, 0.0);
        outer.cinv = nullptr;
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
// passes of the level (zero-guess variants, all right-hand sides) for every
// shape, launched one by one.
mg_status autotune(mg_ctx* c) {
    const long long N0 = c->lv[0].N;
    if (N0 < AUTOTUNE_MIN_POINTS) return MG_OK;
    std::vector<Item> it;
    std::vector<L0> l0;
    CK(mg::launch_fill_zero(c->Z, (long long)c->nrhs * N0 * sizeof(cx<double>), c->stream));
    for (int r = 0; r < c->nrhs; ++r) {
        it.push_back(Item{c, r});
        l0.push_back(L0{c->Z + (size_t)r * N0, 1.0, nullptr, nullptr, c->W + (size_t)r * N0});
    }
    for (int l = 1; l < c->L; ++l) {
        CK(mg::launch_fill_zero(c->lv[l].F, (long long)c->nrhs * c->lv[l].N * elem(c), c->stream));
        CK(mg::launch_fill_zero(c->lv[l].E, (long long)c->nrhs * c->lv[l].N * elem(c), c->stream));
    }
    hipEvent_t e0, e1;
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    // the level's passes replayed as a graph (as the cycle runs them), so
    // that the comparison of shapes on small levels is not one of host
    // launch overheads: one replay to warm up, then REPS timed back to back
    constexpr int REPS = 6;
    Exec E{c->stream, nullptr, &c->cache, true};
    mg_status st = MG_OK;
    for (int l = 0; l < c->lt && st == MG_OK; ++l) {
        if (c->lv[l].N < AUTOTUNE_MIN_POINTS) break;
        float best = 1e30f;
        int best_shape = 0;
        for (int shape = 0; shape < num_shapes(c) && st == MG_OK; ++shape) {
            c->lv[l].shape = shape;
            Op op;
            Rec R{&op, &c->work, c->dim, c->mixed, TAG_ALWAYS};
            st = rec_down(R, 0, it, G_NONE, &l0, l, false, nullptr);
            if (st == MG_OK) st = rec_up(R, 0, it, G_NONE, &l0, l, false);
            if (st == MG_OK) st = op_run(E, op);
            if (st == MG_OK && hipEventRecord(e0, c->stream) != hipSuccess) st = MG_E_DEVICE;
            for (int rep = 0; rep < REPS && st == MG_OK; ++rep) st = op_run(E, op);
            if (st == MG_OK && hipEventRecord(e1, c->stream) != hipSuccess) st = MG_E_DEVICE;
            if (st == MG_OK && hipEventSynchronize(e1) != hipSuccess) st = MG_E_DEVICE;
            float tot = 0.0f;
            if (st == MG_OK && hipEventElapsedTime(&tot, e0, e1) != hipSuccess) st = MG_E_DEVICE;
            op_release(op);
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

// Workgroups per right-hand side that any launch of this context may use
// (so the partial sums it writes fit the work space).
int max_blocks(const mg_ctx* c) {
    int m = mg::vec_blocks(c->lv[0].N);
    for (int shape = 0; shape < mg::NUM_TILE_SHAPES; ++shape) {
        int nt[3];
        mg::tile_counts(c->dim, shape, c->lv[0].n, nt);
        m = std::max(m, nt[0] * nt[1] * nt[2]);
    }
    if (c->dim == 2)
        for (int shape = 0; shape < mg::NUM_MARCH_SHAPES; ++shape) {
            int nt[3];
            mg::march_counts(shape, c->lv[0].n, nt);
            m = std::max(m, nt[0] * nt[1]);
        }
    for (int sweep = 0; sweep < mg::NUM_SWEEP_SHAPES; ++sweep) {
        int nt[3];
        mg::sweep_counts(c->dim, sweep, c->lv[0].n, nt);
        m = std::max(m, nt[0] * nt[1] * nt[2]);
    }
    if (c->dim == 3) m = std::max(m, mg::power_z_tiles(c->lv[0].n));
    for (int per : {16, 32, 64})
        for (bool mv : {false, true})
            m = std::max(m, mg::arnoldi_chunks(mv, c->dim, c->lv[0].n, c->lv[0].N, per / mg::ARN_SPLIT));
    return m;
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
            // the direct solve on the coarsest level applies the inverse,
            // formed column by column from the LU factors in FP64
            std::vector<cx<double>> inv((size_t)nc * nc);
            std::vector<cd> col(nc);
            for (int j = 0; j < nc; ++j) {
                std::fill(col.begin(), col.end(), cd(0.0));
                col[j] = 1.0;
                lu_solve(M, piv, nc, col);
                for (int i = 0; i < nc; ++i) inv[(size_t)i * nc + j] = tocx(col[i]);
            }
            CKS(dalloc(&c->cinv[dir], inv.size() * sizeof(cx<double>)));
            CK(hipMemcpy(c->cinv[dir], inv.data(), inv.size() * sizeof(cx<double>), hipMemcpyHostToDevice));
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
    // (2D GMRES(3): SMALL_POINTS, the marching passes being faster than the
    // tail's global-memory level)
    c->lt = L - 1;
    const long long tail_max = (c->gsmooth && c->dim == 2) ? mg::SMALL_POINTS : mg::TAIL_POINTS;
    for (int l = 1; l < L; ++l)
        if (c->lv[l].N <= tail_max) {
            c->lt = l;
            break;
        }
    {   // the levels of the tail with at most SMALL_POINTS points share its LDS
        long long small = 0;
        for (int l = c->lt; l < L; ++l)
            if (c->lv[l].N <= mg::SMALL_POINTS || l == L - 1) small += c->lv[l].N;
        if (c->lv[c->lt].N > mg::TAIL_POINTS || small > mg::TAIL_LDS || c->lv[L - 1].N > mg::SMALL_POINTS)
            return MG_E_INVAL;
        // only the first tail level may keep its vectors in global memory
        for (int l = c->lt + 1; l < L; ++l)
            if (c->lv[l].N > mg::SMALL_POINTS) return MG_E_INVAL;
    }
    {
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
        }
        const std::vector<mg::SmoothBufs> sb = smooth_table(c);
        CKS(dalloc(&c->sb_d, sb.size() * sizeof(mg::SmoothBufs)));
        CK(hipMemcpy(c->sb_d, sb.data(), sb.size() * sizeof(mg::SmoothBufs), hipMemcpyHostToDevice));
    }
    const size_t vbytes = (size_t)c->nrhs * c->lv[0].N * sizeof(cx<double>);
    if (!c->mixed) CKS(dalloc(&c->U1, vbytes));
    CKS(dalloc(&c->Z, vbytes));
    CKS(dalloc(&c->W, vbytes));
    CKS(work_alloc(c->work, c->nrhs, max_blocks(c)));
    CKS(dalloc(&c->scale_d, (size_t)c->nrhs * HSTRIDE * sizeof(double)));
    CKS(dalloc(&c->coef_d, (size_t)c->nrhs * HSTRIDE * sizeof(cx<double>)));
    // the allocation-free cycle: this device's scratch, pinned table staging
    CK(hipGetDevice(&c->device));
    CKS(scratch_init(c->device));
    CKS(halloc(&c->stage, STAGE_BYTES));
    CK(hipEventCreate(&c->stage_ev));
    CK(hipEventRecord(c->stage_ev, c->stream));
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
    const int n = c->nrhs;
    std::vector<Item> it;
    std::vector<cx<double>*> U;
    std::vector<const cx<double>*> F;
    for (int r = 0; r < n; ++r) {
        it.push_back(Item{c, r});
        U.push_back((cx<double>*)u + (size_t)r * N);
        F.push_back((const cx<double>*)f + (size_t)r * N);
    }
    const bool want = res_before != nullptr;
    const bool direct = !c->mixed && !c->shifted0;
    std::vector<uintptr_t> key = item_key(K_CYCLE, 0, it, U, F);
    key.push_back(want ? 1 : 0);
    Op* op = nullptr;
    CKS(cached(c->cache, key, &op, [&](Op& o) -> mg_status {
        Rec R{&o, &c->work, c->dim, c->mixed, TAG_ALWAYS};
        std::vector<int> cnt;
        std::vector<L0> l0(n);
        if (direct) {
            for (int r = 0; r < n; ++r) l0[r] = L0{F[r], 1.0, nullptr, U[r], U[r]};
            CKS(rec_cycle(R, 0, it, G_NONE, l0, false, want, &cnt));
            if (want) CKS(rec_reduce_real(R, cnt));
        } else {
            std::vector<const cx<double>*> xs(U.begin(), U.end());
            std::vector<cx<double>*> ws(n);
            for (int r = 0; r < n; ++r) ws[r] = wvec(it[r]);
            CKS(rec_residual(R, 0, it, G_NONE, xs, F, ws, want, &cnt));
            if (want) CKS(rec_reduce_real(R, cnt));
            for (int r = 0; r < n; ++r) l0[r] = L0{ws[r], 1.0, nullptr, nullptr, U[r]};
            CKS(rec_cycle(R, 0, it, G_NONE, l0, true, false, nullptr));
        }
        return MG_OK;
    }));
    Exec E = ctx_exec(c);
    CKS(op_run(E, *op));
    if (profiling(E)) {
        CK(hipStreamSynchronize(c->stream));
        CKS(op_collect(E, *op, nullptr));
    }
    if (want) {
        CK(hipMemcpyAsync(c->work.rtot_h, c->work.rtot, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        CK(hipStreamSynchronize(c->stream));
        for (int r = 0; r < n; ++r) res_before[r] = std::sqrt(c->work.rtot_h[r]);
    }
    return MG_OK;
}

// Allocation-free form of mg_cycle: the same recorded launches, with every
// work vector, reduction buffer and table in this device's scratch.
mg_status mg_cycle_noalloc(mg_ctx* c, double* u, const double* f, double* res_before) {
    if (!c || !u || !f) return MG_E_INVAL;
    int dev = -1;
    CK(hipGetDevice(&dev));
    if (dev != c->device || dev < 0 || dev >= MAX_DEVICES || !scratch_ptr[dev]) return MG_E_STATE;
    char* base = (char*)scratch_ptr[dev];
    size_t used = 0;
    auto take = [&](size_t bytes) -> char* {
        used = (used + 255) & ~(size_t)255;
        char* p = base + used;
        used += bytes;
        return p;
    };
    // a shadow of the context whose work space lies in the scratch
    mg_ctx sh;
    sh.p = c->p;
    sh.dim = c->dim;
    sh.L = c->L;
    sh.mixed = c->mixed;
    sh.nrhs = c->nrhs;
    sh.stream = c->stream;
    sh.lv = c->lv;
    sh.ncoarse = c->ncoarse;
    for (int d = 0; d < 2; ++d) {
        sh.cinv[d] = c->cinv[d];
        sh.views_d[d] = c->views_d[d];
        sh.outer_d[d] = c->outer_d[d];
        sh.views_f[d] = c->views_f[d];
    }
    sh.shifted0 = c->shifted0;
    sh.gsmooth = c->gsmooth;
    sh.lt = c->lt;
    const size_t esz = elem(c);
    for (int l = 0; l < c->L; ++l) {
        Level& V = sh.lv[l];
        const size_t bytes = (size_t)c->nrhs * V.N * esz;
        if (V.F) V.F = take(bytes);
        if (V.E) V.E = take(bytes);
        for (int i = 0; i < 3; ++i)
            if (V.Q[i]) V.Q[i] = take(bytes);
        if (V.SU1) V.SU1 = take(bytes);
        if (V.SU2) V.SU2 = take(bytes);
    }
    const size_t vbytes = (size_t)c->nrhs * c->lv[0].N * sizeof(cx<double>);
    if (c->U1) sh.U1 = (cx<double>*)take(vbytes);
    sh.W = (cx<double>*)take(vbytes);
    sh.gcoef = (cx<double>*)take((size_t)c->nrhs * c->L * 8 * sizeof(cx<double>));
    sh.sb_d = (mg::SmoothBufs*)take((size_t)c->nrhs * c->L * sizeof(mg::SmoothBufs));
    Work w;
    w.items = c->nrhs;
    w.bstride = c->work.bstride;
    w.part = (cx<double>*)take((size_t)c->nrhs * HSTRIDE * w.bstride * sizeof(cx<double>));
    w.rpart = (double*)take((size_t)c->nrhs * w.bstride * sizeof(double));
    w.rtot = (double*)take((size_t)c->nrhs * sizeof(double));
    if (used > SCRATCH_BYTES) return MG_E_INVAL;

    const long long N = c->lv[0].N;
    const int n = c->nrhs;
    std::vector<Item> it;
    std::vector<cx<double>*> U;
    std::vector<const cx<double>*> F;
    for (int r = 0; r < n; ++r) {
        it.push_back(Item{&sh, r});
        U.push_back((cx<double>*)u + (size_t)r * N);
        F.push_back((const cx<double>*)f + (size_t)r * N);
    }
    const bool want = res_before != nullptr;
    Op op;
    {
        Rec R{&op, &w, c->dim, c->mixed, TAG_ALWAYS};
        std::vector<int> cnt;
        std::vector<L0> l0(n);
        if (!c->mixed && !c->shifted0) {
            for (int r = 0; r < n; ++r) l0[r] = L0{F[r], 1.0, nullptr, U[r], U[r]};
            CKS(rec_cycle(R, 0, it, G_NONE, l0, false, want, &cnt));
            if (want) CKS(rec_reduce_real(R, cnt));
        } else {
            std::vector<const cx<double>*> xs(U.begin(), U.end());
            std::vector<cx<double>*> ws(n);
            for (int r = 0; r < n; ++r) ws[r] = wvec(it[r]);
            CKS(rec_residual(R, 0, it, G_NONE, xs, F, ws, want, &cnt));
            if (want) CKS(rec_reduce_real(R, cnt));
            for (int r = 0; r < n; ++r) l0[r] = L0{ws[r], 1.0, nullptr, nullptr, U[r]};
            CKS(rec_cycle(R, 0, it, G_NONE, l0, true, false, nullptr));
        }
    }
    char* dtab = take(op.tab.size());
    if (used > SCRATCH_BYTES) return MG_E_INVAL;
    const std::vector<mg::SmoothBufs> sb = smooth_table(&sh);
    const size_t sbb = sb.size() * sizeof(mg::SmoothBufs);
    if (sbb + op.tab.size() > STAGE_BYTES) return MG_E_INVAL;
    // the staging buffer is free once the previous call's copies are done
    CK(hipEventSynchronize(c->stage_ev));
    std::memcpy(c->stage, sb.data(), sbb);
    if (!op.tab.empty()) std::memcpy(c->stage + sbb, op.tab.data(), op.tab.size());
    CK(hipMemcpyAsync(sh.sb_d, c->stage, sbb, hipMemcpyHostToDevice, c->stream));
    if (!op.tab.empty())
        CK(hipMemcpyAsync(dtab, c->stage + sbb, op.tab.size(), hipMemcpyHostToDevice, c->stream));
    CK(hipEventRecord(c->stage_ev, c->stream));
    for (const Step& st : op.steps) CK(st.fn(c->stream, dtab));
    if (want) {
        CK(hipMemcpyAsync(c->work.rtot_h, w.rtot, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        CK(hipStreamSynchronize(c->stream));
        for (int r = 0; r < n; ++r) res_before[r] = std::sqrt(c->work.rtot_h[r]);
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
    CK(mg::launch_grad_k2((const cx<double>*)u, (const cx<double>*)lam, c->nrhs, c->lv[0].N, grad, c->stream));
    return MG_OK;
}

mg_status mg_apply(mg_ctx* c, int level, int adjoint, const double* x, double* y) {
    if (!c || !x || !y || level < 0 || level >= c->L) return MG_E_INVAL;
    const long long N = c->lv[level].N;
    const int dir = adjoint ? 1 : 0;
    std::vector<uintptr_t> key{(uintptr_t)K_APPLY, (uintptr_t)level, (uintptr_t)dir, (uintptr_t)x, (uintptr_t)y};
    Op* op = nullptr;
    CKS(cached(c->cache, key, &op, [&](Op& o) -> mg_status {
        std::vector<VecSlot> sl(c->nrhs);
        int blocks = 0;
        for (int r = 0; r < c->nrhs; ++r) {
            VecSlot& s = sl[r];
            s = VecSlot{};
            s.lv = c->views_d[dir] + level;
            s.x = (const cx<double>*)x + (size_t)r * N;
            s.y = (cx<double>*)y + (size_t)r * N;
            s.block0 = blocks;
            blocks += mg::vec_blocks(N);
        }
        VecArgs a{};
        a.st.n = c->nrhs;
        a.st.nblocks = blocks;
        const size_t off = put(o, sl);
        const int dim = c->dim;
        o.steps.push_back(Step{[=](hipStream_t s, const char* base) {
                                   VecArgs b = a;
                                   b.st.s = (const VecSlot*)(base + off);
                                   return mg::launch_residual(dim, b, s);
                               },
                               MG_K_OTHER, TAG_ALWAYS, {}});
        return MG_OK;
    }));
    Exec E = ctx_exec(c);
    CKS(op_run(E, *op));
    if (profiling(E)) {
        CK(hipStreamSynchronize(c->stream));
        CKS(op_collect(E, *op, nullptr));
    }
    return MG_OK;
}

int mg_tile_shape(mg_ctx* c, int level, int shape) {
    if (!c || level < 0 || level >= c->L) return MG_E_INVAL;
    if (shape >= num_shapes(c)) return MG_E_INVAL;
    if (shape >= 0) {
        if (hipStreamSynchronize(c->stream) != hipSuccess) return MG_E_DEVICE;
        c->lv[level].shape = shape;
        cache_clear(c->cache);   // recorded operations hold the old shapes
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
    Exec E{c0->stream, &c0->prof, &b->cache, true};
    const bool gm = mode == MG_MODE_GMRES || mode == MG_MODE_FGMRES;
    if (!gm || it.size() < 2 || profiling(E))
        return solve_items(E, b->work, 0, it, U, F, mode, rtol, maxit, restart, iters, hist);
    std::vector<Group> G;
    CKS(make_groups(E, b->work, b->workg, b->streamg, it, U, F, G));
    return solve_groups(G, 0, mode, rtol, maxit, restart, iters, hist);
}

void mg_batch_destroy(mg_batch* b) {
    if (!b) return;
    if (!b->ctxs.empty()) (void)hipStreamSynchronize(b->ctxs[0]->stream);
    cache_free(b->cache);
    work_free(b->work);
    for (int g = 0; g < SOLVE_GROUPS - 1; ++g) {
        if (b->streamg[g]) (void)hipStreamSynchronize(b->streamg[g]);
        work_free(b->workg[g]);
        if (b->streamg[g]) (void)hipStreamDestroy(b->streamg[g]);
    }
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
    c->prof.clear();
    return MG_OK;
}

mg_status mg_profile_read(mg_ctx* c, int which, double* total_ms, long long* count, double* bytes) {
    if (!c || which < 0 || which >= MG_K_NUM_CLASSES) return MG_E_INVAL;
    CK(hipStreamSynchronize(c->stream));
    if (total_ms) *total_ms = c->prof.ms[which];
    if (count) *count = c->prof.cnt[which];
    if (bytes) *bytes = c->prof.bytes[which];
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
