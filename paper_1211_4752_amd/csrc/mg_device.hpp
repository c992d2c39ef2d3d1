// Device-side types and kernel launchers of the level-dependent multigrid.
//
// Everything here is gfx950 (CDNA4, wave64) code.  Grid vectors are
// interleaved complex, x fastest; one workgroup works on one tile of one
// right-hand side ("slot"); slots are described by a small device table so
// that the right-hand sides still iterating can be compacted between steps.
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

// One right-hand side in flight.
struct Slot {
    int rhs;             // index of the right-hand side at the ABI
    int j;               // GMRES: index of the newest basis vector
    int buf;             // index of its internal work vectors
    int pad_;
    long long in_off;    // complex-element offset of the level-0 input vector
    long long out_off;   // complex-element offset of the level-0 output vector
    double in_scale;     // the level-0 input is multiplied by this
};

// Right-hand sides of one launch, passed by value in the kernel arguments.
constexpr int MAX_SLOTS = 32;
// Largest coarsest level (unknowns) of the direct solve.
constexpr int MAX_COARSE = 1024;
struct SlotTable {
    int n;
    Slot s[MAX_SLOTS];
};

// One level of the hierarchy, in compute precision T.
template <typename T>
struct LevelView {
    int n[3];                  // interior points per axis (n[2] = 1 in 2D)
    long long N;               // n[0] n[1] n[2]
    const cx<T>* cm[3];        // per-axis 3-point coefficients
    const cx<T>* c0[3];
    const cx<T>* cp[3];
    const T* k2;               // k^2 sampled on this level
    cx<T> sigma;               // shift multiplying k^2
    cx<T> omega;               // Jacobi weight
};

// Pre-smooth + residual + full weighting (+ norm of the incoming residual).
template <typename T, typename TF>
struct SmoothRestrictArgs {
    LevelView<T> lv;
    int nc[3];                 // coarse sizes
    long long Nc;
    SlotTable st;
    int ntiles[3];
    const cx<T>* u;            // incoming iterate, indexed by rhs (zero guess: null)
    const cx<TF>* f;           // right-hand side: level 0 uses slot.in_off/in_scale,
    bool f_by_slot;            //   coarse levels index by slot (f_by_slot = true)
    cx<T>* u1;                 // smoothed iterate out, indexed by slot (null: skip)
    cx<T>* fc;                 // restricted residual out, indexed by slot
    double* norm_part;         // ||f - A u||^2 per (slot, block) (null: skip)
};

// Prolongation + correction + post-smooth.
template <typename T, typename TF, typename TO>
struct ProlongSmoothArgs {
    LevelView<T> lv;
    int nc[3];
    long long Nc;
    SlotTable st;
    int ntiles[3];
    const cx<T>* u1;           // smoothed iterate by slot (zero guess: null, recomputed)
    const cx<TF>* f;           // right-hand side (as in SmoothRestrictArgs)
    bool f_by_slot;
    const cx<T>* ec;           // coarse correction, indexed by slot
    cx<TO>* out;               // result: level 0 uses slot.out_off, else by slot
    bool out_by_slot;
};

// y = f - A x  or  y = A x, plus ||y||^2 partials.
struct ResidualArgs {
    LevelView<double> lv;
    SlotTable st;
    const cx<double>* x;       // indexed by rhs
    const cx<double>* f;       // indexed by rhs (null: y = A x)
    cx<double>* y;             // y base + slot.out_off
    double* norm_part;         // per (slot, block) (null: skip)
    int nblocks;
};

// GMRES pass kernels: basis V[rhs][i] = Vb + (rhs * vstride + i) * N.
struct OrthoArgs {
    LevelView<double> lv;      // used by the matvec pass
    SlotTable st;
    long long N;
    const cx<double>* z;       // matvec input, by slot
    cx<double>* w;             // work vector, by slot
    cx<double>* Vb;            // basis base
    int vstride;               // restart + 1
    const double* scale;       // scale[rhs * sstride + i]: v_i = scale * V[i]
    int sstride;
    const cx<double>* hin;     // coefficients h_i of the update, [slot * hstride + i]
    int hstride;
    cx<double>* part;          // partial sums [(slot * pstride + i) * nblocks + b]
    int pstride;
    int nblocks;
};

struct CombineArgs {
    SlotTable st;
    long long N;
    const cx<double>* Vb;
    int vstride;
    const cx<double>* coef;    // coef[rhs * sstride + i], applied to V[i] as stored
    int sstride;
    cx<double>* t;             // by slot
};

// ---------------------------------------------------------------------------
// Launchers (defined in mg_kernels.hip).  All return hipError_t of the launch.
// ---------------------------------------------------------------------------
enum class Prec { F64, F32 };

hipError_t launch_smooth_restrict_f64(int dim, bool zero, const SmoothRestrictArgs<double, double>& a,
                                      int* nblocks_out, hipStream_t s);
hipError_t launch_smooth_restrict_f32(int dim, bool level0, const SmoothRestrictArgs<float, double>& a0,
                                      const SmoothRestrictArgs<float, float>& ac, int* nblocks_out,
                                      hipStream_t s);
hipError_t launch_prolong_smooth_f64(int dim, bool zero, bool accumulate,
                                     const ProlongSmoothArgs<double, double, double>& a, hipStream_t s);
hipError_t launch_prolong_smooth_f32(int dim, bool level0, bool accumulate,
                                     const ProlongSmoothArgs<float, double, double>& a0,
                                     const ProlongSmoothArgs<float, float, float>& ac, hipStream_t s);
// number of tiles the two fused kernels use on a level of size n
void tile_counts(int dim, bool f32, const int n[3], int ntiles[3]);

// f / e: coarsest vectors indexed by slot.buf
hipError_t launch_coarse_solve_f64(const cx<double>* lu, const int* piv, int n, const SlotTable& st,
                                   const cx<double>* f, cx<double>* e, hipStream_t s);
hipError_t launch_coarse_solve_f32(const cx<double>* lu, const int* piv, int n, const SlotTable& st,
                                   const cx<float>* f, cx<float>* e, hipStream_t s);

int residual_blocks(long long N);
hipError_t launch_residual(int dim, const ResidualArgs& a, hipStream_t s);
// ||x_r||^2 partials per (local slot, block); x indexed by rhs (by_buf = false) or buf
hipError_t launch_norm(const SlotTable& st, const cx<double>* x, bool by_buf, long long N,
                       double* part, int nblocks, hipStream_t s);

int ortho_blocks(long long N);
hipError_t launch_matvec_dot(int dim, int jmax, const OrthoArgs& a, hipStream_t s);
hipError_t launch_update_dot(int jmax, const OrthoArgs& a, hipStream_t s);
hipError_t launch_update_norm(int jmax, const OrthoArgs& a, hipStream_t s);
hipError_t launch_combine(int jmax, const CombineArgs& a, hipStream_t s);

// out[slot * ostride + v] = sum_b part[(slot * vstride + v) * nblocks + b], v < nvals,
// summed in a fixed order
hipError_t launch_reduce_complex(const cx<double>* part, int nvals, int vstride, int nblocks,
                                 int nslots, cx<double>* out, int ostride, hipStream_t s);
hipError_t launch_reduce_real(const double* part, int nblocks, int nslots, double* out,
                              hipStream_t s);

hipError_t launch_inject_k2(int dim, const double* fine, const int nf[3], double* coarse,
                            const int nc[3], hipStream_t s);
hipError_t launch_to_f32(const double* src, float* dst, long long n, hipStream_t s);
hipError_t launch_grad_k2(const cx<double>* u, const cx<double>* lam, int nrhs, long long N,
                          double* grad, hipStream_t s);
hipError_t launch_fill_zero(void* p, long long bytes, hipStream_t s);

}  // namespace mg
