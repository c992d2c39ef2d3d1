// Device-side types and kernel launchers of the level-dependent multigrid.
//
// Everything here is gfx950 (CDNA4, wave64) code.  Grid vectors are
// interleaved complex, x fastest.  A launch covers a list of "slots": one slot
// is one right-hand side of one problem (grid); it carries a pointer to the
// device-resident descriptor of its level (LevelView) and the pointers of the
// vectors it reads and writes, so one launch can serve right-hand sides of
// grids of different sizes.  Slot tables live in device memory (any number of
// slots per launch); the kernel arguments carry their address.  A slot may
// carry a gate: a device flag that, when zero, makes the slot's workgroups
// return at once, so that one recorded sequence of launches (replayed as a
// HIP graph) serves right-hand sides whose iterations stop at different
// steps.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mg {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
    T r, i;
};

template <typename T>
__host__ __device__ __forceinline__ cx<T> mk(T r, T i) {
    cx<T> z;
    z.r = r;
    z.i = i;
    return z;
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return mk(a.r + b.r, a.i + b.i); }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return mk(a.r - b.r, a.i - b.i); }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
    return mk(a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r);
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return mk(s * a.r, s * a.i); }
// conj(a) * b
template <typename T>
__host__ __device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
    return mk(a.r * b.r + a.i * b.i, a.r * b.i - a.i * b.r);
}
template <typename T>
__host__ __device__ __forceinline__ T abs2(cx<T> a) { return a.r * a.r + a.i * a.i; }
template <typename T, typename S>
__host__ __device__ __forceinline__ cx<T> cvt(cx<S> a) { return mk<T>((T)a.r, (T)a.i); }
// a / d via one real division
template <typename T>
__host__ __device__ __forceinline__ cx<T> cdiv(cx<T> a, cx<T> d) {
    T inv = T(1) / abs2(d);
    return mk((a.r * d.r + a.i * d.i) * inv, (a.i * d.r - a.r * d.i) * inv);
}

// Limits.
constexpr int MAX_COARSE = 1024;   // unknowns of the coarsest direct solve
constexpr int MAX_RESTART = 32;    // GMRES restart length
constexpr int HSTRIDE = MAX_RESTART + 1;   // reduction values per slot

__host__ __device__ __forceinline__ bool gated_off(const int* g) { return g && *g == 0; }

// One level of one problem, in compute precision T, resident in device
// memory.  The descriptors of a problem's levels are contiguous, finest
// first, so (this + 1) describes the next coarser level.
template <typename T>
struct LevelView {
    int n[3];                  // interior points per axis (n[2] = 1 in 2D)
    int ntiles[3];             // tiles of the fused kernels on this level
    long long N;               // n[0] n[1] n[2]
    const cx<T>* cm[3];        // per-axis 3-point coefficients
    const cx<T>* c0[3];
    const cx<T>* cp[3];
    const T* k2;               // k^2 sampled on this level
    const cx<double>* cinv;    // coarsest level only: inverse of the level operator (FP64), row-major
    cx<T> sigma;               // shift multiplying k^2
    cx<T> omega;               // Jacobi weight
    T sinv;                    // 1 / s, s the scale of the smoother's power basis
};

// Work vectors of the GMRES(3) smoother for one right-hand side on one level,
// in compute precision, device resident.  With r the residual of the iterate
// being smoothed, q0 = r, q1 = (A/s) q0, q2 = (A/s) q1 (q3 = (A/s) q2 is
// only ever formed on the fly).
struct SmoothBufs {
    void* q[3];
    void* u1;                  // iterate after pre-smoothing
    void* u2;                  // iterate after the coarse-grid correction
    cx<double>* coef;          // [2][4]: c1, c2, c3, (||r||^2, 0) for pre (0) and post (1)
    void* f;                   // the level's right-hand side (levels >= 1)
    void* e;                   // the level's correction (levels >= 1)
};

// The coarse tail: one workgroup per slot runs the cycle from level lt
// (rhs in sb[0].f, zero guess) down to the coarsest and back, leaving the
// correction in sb[0].e, with every vector of those levels in LDS.  lv and
// sb point at level lt; both tables are contiguous by level.
struct TailSlot {
    const void* lv;
    const SmoothBufs* sb;
    int nlev;                  // levels lt .. coarsest
    int pad_;
    const int* gate;
};

struct TailArgs {
    int n;
    int gmres;                 // smoother: 0 omega-Jacobi, 1 GMRES(3)
    double brk;                // relative Cholesky pivot of an exhausted Krylov space
    const TailSlot* s;         // device table of n slots
};
constexpr int TAIL_POINTS = 4096;   // levels of at most this many points go to the tail
constexpr int SMALL_POINTS = 1024;  // tail levels of at most this many points live in LDS
constexpr int TAIL_LDS = 1408;      // points of all LDS tail levels together

// A slot of the two fused cycle kernels and of the coarsest solve.
struct CycleSlot {
    const void* lv;       // LevelView<T>* of this slot's problem at the launch level
    const void* f;        // right-hand side on the launch level (TF at level 0, else T)
    const void* u;        // incoming iterate (standalone level 0), null = zero guess
    void* u1;             // smoothed iterate buffer (standalone level 0) or null
    void* c;              // K_A: coarse right-hand side out; K_B: coarse correction in
    void* out;            // K_B: result; coarsest solve: correction out
    double fscale;        // f is multiplied by this (unless fsp is set)
    int tile0;            // first logical tile of this slot in the launch
    int pad_;
    const SmoothBufs* sb; // GMRES(3) smoother buffers of this slot's rhs on the launch level
    const double* fsp;    // device scale of f, overrides fscale when set
    const int* gate;      // slot skipped when *gate == 0
};

struct CycleSlots {
    int n;
    int ntiles;           // total logical tiles of the launch
    const CycleSlot* s;   // device table of n slots, increasing tile0
};

template <typename S>
__host__ __device__ __forceinline__ double fscale_of(const S& s) {
    return s.fsp ? *s.fsp : s.fscale;
}

// Fused cycle kernels: slots, plus ||f - A u||^2 partials of the incoming
// iterate (standalone level 0) at norm_part[slot * pstride + tile].
struct CycleArgs {
    CycleSlots st;
    double* norm_part;
    int pstride;
    // 2D GMRES(3) apply passes on coarse levels: when gpart is set, each
    // workgroup forms the smoothing coefficients itself from the Gram
    // partials of the preceding Gram pass (value v of the slot's tile b at
    // gpart[(slot * gpstride + v) * gbstride + b]) instead of reading the
    // coefficient record
    const cx<double>* gpart;
    int gpstride, gbstride;
    double gbrk;               // relative pivot of an exhausted Krylov space
};

// Tiles of a coarse level above which the apply passes leave the
// coefficient solve to its own launch.
constexpr int FUSED_COEF_TILES = 128;

// A slot of the vector kernels (residual, norm, GMRES passes, combine).
struct VecSlot {
    const void* lv;             // LevelView<double>* of level 0 (operator, N)
    const cx<double>* x;        // residual / matvec input (z)
    const cx<double>* f;        // residual right-hand side or null
    cx<double>* y;              // residual output / GMRES work vector w / combine output
    cx<double>* V;              // GMRES basis of this rhs: V_i at V + i N
    const double* scale;        // v_i = scale[i] V_i
    const cx<double>* coef;     // combine: t = sum_i coef[i] V_i
    const cx<double>* hin;      // update pass: h_i at hin[i]
    int j;                      // newest basis index (unless jp is set)
    int block0;                 // first workgroup of this slot in the launch
    const int* jp;              // device newest basis index, overrides j when set
    const int* gate;            // slot skipped when *gate == 0
    int nc;                     // Arnoldi passes: chunks of the slot's vector (its partial sums)
};

// Arnoldi passes: each slot's vector is cut into a fixed number of chunks,
// one partial sum each, so the sums do not depend on the launch.  The chunks
// of the slots that are still live are spread evenly over the launch's
// workgroups, of which a slot brings ceil(nc / ARN_SPLIT): with every slot
// live a workgroup takes ARN_SPLIT chunks, and when right-hand sides of a
// batch have converged the others spread over the whole grid.
constexpr int ARN_SPLIT = 4;

struct VecSlots {
    int n;
    int nblocks;                // total workgroups of the launch
    const VecSlot* s;           // device table of n slots, increasing block0
};

// Vector kernels: partial sums at part[(slot * pstride + i) * bstride + b],
// b the workgroup index within its slot.
struct VecArgs {
    VecSlots st;
    cx<double>* part;
    double* rpart;
    int pstride;
    int bstride;
};

// Second reduction stage: out[slot * ostride + v] = sum_{b < cnt[slot]}
// part[(slot * pstride + v) * bstride + b], in a fixed order.
struct ReduceArgs {
    const cx<double>* part;
    const double* rpart;
    cx<double>* out;
    double* rout;
    int nvals, pstride, bstride, ostride;
    const int* cnt;             // device, one count per slot
};

// A slot of the pointwise passes of the GMRES(3) smoother.
struct SmSlot {
    const void* lv;             // LevelView<T>* of the slot's level
    const SmoothBufs* sb;
    const void* f;              // non-null: q0 = fscale f (complex double on level 0, else T)
    void* out;                  // apply pass: result (complex double on level 0, else T)
    double fscale;
    int block0;                 // first workgroup of this slot in the launch
    int pad_;
    const double* fsp;          // device scale of f, overrides fscale when set
    const int* gate;
};

struct SmSlots {
    int n;
    int nblocks;
    const SmSlot* s;            // device table of n slots, increasing block0
};

// Pointwise smoother passes; Gram partials at part[(slot * pstride + v) *
// bstride + b], v < 10 (G00 G11 G22 G33 G01 G02 G03 G12 G13 G23, G_ij =
// sum conj(q_i) q_j).
struct SmArgs {
    SmSlots st;
    cx<double>* part;
    int pstride;
    int bstride;
};

// Gram reduction and coefficient solve: per slot, sum cnt partials in a
// fixed order and write c1, c2, c3, (G00, 0) to coef[0..3].
struct CoefSlot {
    cx<double>* coef;
    int cnt;
    int pslot;                  // the slot's index in the Gram launch (its partials)
    const int* gate;
};
struct SmCoefArgs {
    const cx<double>* part;
    int pstride, bstride;
    const CoefSlot* s;          // device table, one per slot of the Gram launch
};

// ---------------------------------------------------------------------------
// Krylov control on the device.  Per item (one right-hand side of one
// problem): flags read back by the host once per restart cycle, and the
// small dense state of restarted (F)GMRES: Hessenberg columns, Givens
// rotations, the rotated right-hand side g and the Gram matrix of the
// stored basis (used by the one-reduction second Gram-Schmidt pass).
// ---------------------------------------------------------------------------
struct GmFlags {
    int live;      // 1: runs the next Arnoldi step / standalone cycle
    int fin;       // 1: the restart cycle ends (solution update, new residual)
    int zero;      // 1: zero right-hand side, solution 0
    int state;     // 0 running, 1 converged, 2 maxit, 3 diverged
    int its;       // outer steps (GMRES) or cycles (standalone) taken
    int hlen;      // history entries written
    int j;         // newest basis index (GMRES) / cycle counter (standalone)
    int kk;        // index of the last basis vector combined at a restart
};

struct GmState {
    cx<double> H[MAX_RESTART][MAX_RESTART + 1];     // H[col][row], rotated
    cx<double> G[MAX_RESTART + 1][MAX_RESTART + 1]; // G[k][i] = <v_i, v_k>, i <= k
    cx<double> h[MAX_RESTART + 1];                  // column of the step in progress
    cx<double> g[MAX_RESTART + 1];
    cx<double> sn[MAX_RESTART];
    double cs[MAX_RESTART];
    double nf;                                      // ||f||
};

// Solve parameters, device resident (uploaded once per solve).
struct GmParams {
    double rtol;
    double* hist;      // [item][hstride] relative residual histories
    int hstride;       // maxit + 1
    int maxit;
    int m;             // restart length
    int flexible;
};

struct GmItem {
    GmState* st;
    GmFlags* fl;
    double* scale;         // v_i = scale[i] V_i
    cx<double>* coef;      // combination coefficients of a finished restart cycle
    int cnt;               // partials of this item in the producing launch
    int slot;              // slot of this item in the producing launch
};

struct GmArgs {
    const GmItem* it;      // device table, one per workgroup
    const GmParams* prm;
    const cx<double>* part;
    const double* rpart;
    int pstride, bstride;
    int j;                 // Arnoldi step of k_gm_h / k_gm_col
};

// ---------------------------------------------------------------------------
// Launchers (defined in mg_kernels.hip, mg_jacobi.hip and mg_smooth.hip).  All return hipError_t of the launch.
// Tile shape of the fused kernels: a shape id (chosen per level by timing).
// ---------------------------------------------------------------------------
constexpr int NUM_TILE_SHAPES = 3;
void tile_shape(int dim, int shape, int t[3]);
void tile_counts(int dim, int shape, const int n[3], int ntiles[3]);

hipError_t launch_smooth_restrict(int dim, bool f32, bool level0, bool zero, int shape, const CycleArgs& a,
                                  hipStream_t s);
hipError_t launch_prolong_smooth(int dim, bool f32, bool level0, bool zero, bool accumulate, int shape,
                                 const CycleArgs& a, hipStream_t s);
// Plane-sweep variants of the two omega-Jacobi kernels for a zero incoming
// iterate (mg_jacobi.hip): sweep configuration ids 0 .. NUM_SWEEP_SHAPES - 1.
constexpr int NUM_SWEEP_SHAPES = 3;
// Shapes of the 2D GMRES(3) passes: row-marching strips (mg_march2d.hip),
// ids 0 .. MARCH_TILE - 1, and LDS tiles (mg_tile2d.hip), id MARCH_TILE.
constexpr int MARCH_TILE = 4;
constexpr int NUM_MARCH_SHAPES = 5;
void sweep_counts(int dim, int sweep, const int n[3], int ntiles[3]);
hipError_t launch_sweep_sr(int dim, bool f32, bool level0, int sweep, const CycleArgs& a, hipStream_t s);
hipError_t launch_sweep_ps(int dim, bool f32, bool level0, bool accumulate, int sweep, const CycleArgs& a,
                           hipStream_t s);

// number of workgroups a vector kernel uses for N points
// Workgroups per slot of a vector launch over N points: about per points
// per thread, between 1 and 1024.
int vec_blocks(long long N, int per = 8);
// Chunks per slot of the Arnoldi passes on an n[0] x n[1] (x n[2]) grid,
// about per points per thread each.  Matvec pass (mv) in 2D: column blocks
// of NT times row strips of at most per rows, numbered strip-fastest; in
// 3D: the z-march columns of power_z_tiles (per unused); otherwise
// contiguous ranges of the N points, at most 1024 * ARN_SPLIT.
int arnoldi_chunks(bool mv, int dim, const int n[3], long long N, int per);
hipError_t launch_residual(int dim, const VecArgs& a, hipStream_t s);
hipError_t launch_norm(const VecArgs& a, hipStream_t s);
hipError_t launch_matvec_dot(int dim, int jmax, const VecArgs& a, hipStream_t s);
// V_{j+1} = w - sum_i hin_i v_i with partials <v_i, V_{j+1}> (i <= j) and
// ||V_{j+1}||^2 (value j + 1)
hipError_t launch_update_gram(int jmax, const VecArgs& a, hipStream_t s);
// y = 0 for every slot that is not gated off
hipError_t launch_vzero(const VecArgs& a, hipStream_t s);
hipError_t launch_combine(int jmax, bool accumulate, const VecArgs& a, hipStream_t s);
hipError_t launch_reduce(const ReduceArgs& a, int nslots, bool real, hipStream_t s);

// GMRES(3) smoother passes (mg_smooth.hip).  level0: f is complex double.
constexpr int NUM_GRAM = 10;
hipError_t launch_sm_power(int dim, bool f32, bool level0, int stage, const SmArgs& a, hipStream_t s);
// 3D finest level: the same powers as a z-march over columns of PZX x PZY
// points and PZC planes; one workgroup per column piece, power_z_tiles(n)
// per slot (block0 counts them).
constexpr int PZX = 64, PZY = 4, PZC = 32;
constexpr int PZW = PZX + 2, PZH = PZY + 2;   // an LDS plane with its ring
constexpr int PZR = 2 * PZX + 2 * PZH;        // points of the ring
__host__ __device__ inline void pz_counts(const int n[3], int& ntx, int& nty, int& ntz) {
    ntx = (n[0] + PZX - 1) / PZX;
    nty = (n[1] + PZY - 1) / PZY;
    ntz = (n[2] + PZC - 1) / PZC;
}
// ring point r < PZR of a column: its LDS position (x, then y, with the
// ring at 0 and PZW - 1 / PZH - 1)
__host__ __device__ inline void pz_ring(int r, int& lx, int& ly) {
    if (r < PZX) {
        lx = r + 1;
        ly = 0;
    } else if (r < 2 * PZX) {
        lx = r - PZX + 1;
        ly = PZH - 1;
    } else if (r < 2 * PZX + PZH) {
        lx = 0;
        ly = r - 2 * PZX;
    } else {
        lx = PZW - 1;
        ly = r - 2 * PZX - PZH;
    }
}
int power_z_tiles(const int n[3]);
hipError_t launch_sm_power_z(bool f32, bool level0, int stage, const SmArgs& a, hipStream_t s);
// and the Gram partials of that level the same way (one per column piece)
hipError_t launch_sm_gram_z(bool f32, bool level0, const SmArgs& a, hipStream_t s);
hipError_t launch_sm_gram(int dim, bool f32, bool level0, const SmArgs& a, hipStream_t s);
hipError_t launch_sm_coef(bool f32, const SmCoefArgs& a, int nslots, hipStream_t s);
hipError_t launch_sm_apply_restrict(int dim, bool f32, bool level0, bool nonzero, int shape, const CycleArgs& a,
                                    hipStream_t s);
// 3D finest level: the same pass as a z-march over the columns of the power
// passes (power_z_tiles(n) workgroups per slot, tile0 counting them).
hipError_t launch_sm_apply_restrict_z(bool f32, bool nonzero, const CycleArgs& a, hipStream_t s);
hipError_t launch_sm_prolong_resid(int dim, bool f32, bool level0, int shape, const CycleArgs& a, hipStream_t s);
hipError_t launch_sm_apply_out(bool f32, bool level0, bool accumulate, const SmArgs& a, hipStream_t s);
// 2D passes as row-marching wavefronts (mg_march2d.hip): a tile is a strip
// of 56 columns by 32, 16 or 8 rows (shape id 0, 1, 2); Gram partials per strip at
// part[(slot * pstride + v) * bstride + tile].
void march_counts(int shape, const int n[3], int ntiles[3]);
void tile2d_counts(const int n[3], int ntiles[3]);
hipError_t tile2d_gram(bool f32, bool level0, bool post, const CycleArgs& a, cx<double>* part, int pstride,
                       int bstride, hipStream_t s);
hipError_t tile2d_apply_restrict(bool f32, bool level0, bool nonzero, const CycleArgs& a, hipStream_t s);
hipError_t tile2d_apply_out(bool f32, bool level0, bool accumulate, const CycleArgs& a, hipStream_t s);
hipError_t launch_sm2_gram(bool f32, bool level0, bool post, int shape, const CycleArgs& a, cx<double>* part,
                           int pstride, int bstride, hipStream_t s);
hipError_t launch_sm2_apply_restrict(bool f32, bool level0, bool nonzero, int shape, const CycleArgs& a,
                                     hipStream_t s);
hipError_t launch_sm2_apply_out(bool f32, bool level0, bool accumulate, int shape, const CycleArgs& a, hipStream_t s);

hipError_t launch_tail(int dim, bool f32, const TailArgs& a, hipStream_t s);

// Krylov control kernels (mg_krylov.hip), one workgroup per item of a.it:
//   gm_init     ||f|| from the norm partials; zero right-hand sides finish
//               at once; histories set to -1
//   gm_restart  (gated by fin) ||f - A x|| from the residual partials, stop
//               tests, start of a restart cycle
//   gm_h        (gated by live) h = (2 I - G) h1 from the matvec-dot partials
//   gm_col      (gated by live) new basis norm and Gram column, Hessenberg
//               column, Givens rotation, estimate, stop tests, and on a
//               finished restart cycle the coefficients y = R^{-1} g
//   sa_init     standalone: ||f||, zero right-hand sides, histories
//   sa_step     standalone (gated by live): ratio of the incoming iterate
//               from the norm partials, stop tests
hipError_t launch_gm(int which, int nitems, const GmArgs& a, hipStream_t s);
enum { GM_INIT = 0, GM_RESTART = 1, GM_H = 2, GM_COL = 3, SA_INIT = 4, SA_STEP = 5 };

hipError_t launch_inject_k2(int dim, const double* fine, const int nf[3], double* coarse, const int nc[3],
                            hipStream_t s);
hipError_t launch_to_f32(const double* src, float* dst, long long n, hipStream_t s);
hipError_t launch_grad_k2(const cx<double>* u, const cx<double>* lam, int nrhs, long long N, double* grad,
                          hipStream_t s);
hipError_t launch_fill_zero(void* p, long long bytes, hipStream_t s);

}  // namespace mg
