/*
 * mg.h -- C ABI of the MI355X (gfx950) level-dependent complex-shifted
 * multigrid solver for the indefinite Helmholtz equation
 *
 *     (-Delta^h - k^2) u = f                                   (Sec. 2, eq. HH)
 *
 * after S. Cools, B. Reps, W. Vanroose, "A new level-dependent coarse grid
 * correction scheme for indefinite Helmholtz problems" (NLAA 2013).
 *
 * Method.  Level l (0 = finest, h_l = 2^l h_0) is rediscretised as
 *     A~_l = -Delta^{h_l} - sigma_l k_l^2,   sigma_0 = 1       (Sec. 3.1, eq. cslvariant)
 * with sigma_l = exp(i l theta_max / L) by default (Sec. 3.1: d-theta =
 * theta_max / p, p the number of levels).  One V(1,1) cycle is:
 * omega-Jacobi pre-smoothing (Sec. 3.2.1, eq. wjacobi), residual, full
 * weighting to the next level, recursion with a zero initial guess, a dense
 * direct solve on the coarsest level, (bi/tri)linear interpolation of the
 * correction (Sec. 2.1), omega-Jacobi post-smoothing.  The cycle is used as a
 * solver (Sec. 4.1 "LVL-MG") or as the preconditioner of restarted GMRES,
 * one cycle per outer step (Sec. 4.1, Table 3).
 *
 * Discretisation.  Vertex-centred grid of n[a] interior points per axis with
 * homogeneous Dirichlet ghosts; optional exterior-complex-scaled (ECS)
 * absorbing layers of ecs_lo[a] / ecs_hi[a] cells (Sec. 2.4): node x is
 * mapped to a + (x - a) e^{i phi} left of the layer start a (and likewise on
 * the right), and -d^2/dz^2 is discretised by the 3-point formula on the
 * mapped nodes.  Coarse levels sample k^2 at their own nodes.
 *
 * Layout of every grid vector at this ABI: interleaved complex double
 * (re, im), x fastest, then y, then z, then the right-hand side index:
 *     v[2 * (i_x + n_x (i_y + n_y (i_z + n_z r))) + {0,1}]
 * interior points only.  Real fields (k^2, gradients) use the same order
 * without the (re, im) pair and without the right-hand side index.
 *
 * Memory and streams.  Pointers named *_dev are device pointers on the
 * current HIP device; pointers without the suffix are host memory.  Every
 * call is stream-ordered on the stream given to mg_setup; calls that return
 * host values (iteration counts, histories, res_before) synchronise that
 * stream before returning.  The caller owns all vectors it passes; the
 * context owns the hierarchy and all work space.  Use one context per stream
 * and per host thread.  No exception or abort crosses this ABI; failures are
 * reported by the returned status.
 */
#ifndef MG_H
#define MG_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum mg_status {
    MG_OK = 0,
    MG_NOT_CONVERGED = 1,   /* maxit reached; outputs hold the last iterate */
    MG_E_INVAL = -1,        /* invalid argument or dimensions               */
    MG_E_NOMEM = -2,        /* device or host allocation failed             */
    MG_E_DEVICE = -3,       /* a HIP runtime call failed                    */
    MG_E_DIVERGED = -4,     /* residual ratio above 1e8 or not finite       */
    MG_E_STATE = -5         /* call not valid for this context              */
} mg_status;

enum mg_precision {
    MG_PREC_C128 = 0,       /* every step in complex double                 */
    MG_PREC_MIXED = 1       /* cycle in complex float, coarsest solve, outer
                               residual / correction / GMRES in double       */
};

enum mg_mode {
    MG_MODE_STANDALONE = 0, /* repeated V-cycles (Sec. 4.1, LVL-MG)          */
    MG_MODE_GMRES = 1,      /* restarted GMRES(restart), right-preconditioned
                               by one V-cycle from a zero guess per step;
                               flexible (as MG_MODE_FGMRES) when the smoother
                               is GMRES(3), whose cycle is nonlinear         */
    MG_MODE_FGMRES = 2      /* restarted flexible GMRES (Sec. 3.2.2: the
                               preconditioner may change per step): stores
                               z_j = M v_j, x += Z y                         */
};

enum mg_smoother {
    MG_SMOOTH_JACOBI = 0,   /* omega-Jacobi, weight omega (Sec. 3.2.1)       */
    MG_SMOOTH_GMRES3 = 1    /* one GMRES(3) cycle per smoothing step
                               (Sec. 3.2.2): the iterate of least residual in
                               u + K_3(A~_l, r), coefficients recomputed on
                               every level and application                 */
};

typedef struct mg_params {
    int ndim;               /* 2 or 3                                        */
    int n[3];               /* interior points per axis, x first; each axis
                               must be odd on every level except the last    */
    double h[3];            /* grid spacing per axis                         */
    int nlevels;            /* 0 = automatic: coarsen while every axis is odd
                               and the next size is >= 2                     */
    int ecs_lo[3];          /* ECS cells at the low end of each axis         */
    int ecs_hi[3];          /* ECS cells at the high end of each axis        */
    double ecs_angle;       /* rotation phi of the ECS contour (radians)     */
    const double *sigma;    /* host, 2 * nlevels doubles (re, im) of sigma_l,
                               the shifts of the cycle's level operators;
                               NULL = default schedule (sigma_0 = 1).
                               sigma_0 != 1 makes the cycle a fixed-shift
                               preconditioner (the CSL-preconditioned
                               comparator of Sec. 2.2 / Table 3 with sigma_l =
                               1 + i beta on every level): residuals and
                               Krylov steps keep the problem's operator
                               (sigma = 1); standalone mode and mg_cycle then
                               iterate u <- u + M (f - A u)                  */
    double theta_max;       /* default schedule sigma_l = exp(i l theta_max/L) */
    int nu1, nu2;           /* smoothing sweeps; the library supports 1, 1   */
    double omega[2];        /* complex Jacobi weight (re, im)                */
    int precision;          /* enum mg_precision                             */
    int nrhs;               /* right-hand sides handled by every call (>= 1) */
    int smoother;           /* enum mg_smoother                              */
} mg_params;

typedef struct mg_ctx mg_ctx;

/* Fill *p with the defaults of the paper's setting: V(1,1), omega = 2/3,
 * theta_max = pi/6, phi = pi/4, no ECS, automatic levels, C128, one rhs. */
void mg_params_default(mg_params *p);

/* Build the level hierarchy (Sec. 3.1): per-level spacing, ECS coefficients
 * of the forward and conjugate-transposed operators, sigma_l, k^2 sampled on
 * every level, and the LU factors of the coarsest operator and of its
 * conjugate transpose.  k2_dev: n_x n_y n_z doubles on the device, copied
 * (the caller may free it after the call returns).  stream: a hipStream_t
 * (NULL = the null stream).  Errors: MG_E_INVAL for inconsistent dimensions,
 * unsupported nu1/nu2, nrhs < 1 or a coarsest level above
 * 1024 unknowns; MG_E_NOMEM; MG_E_DEVICE.  *out is NULL on error. */
mg_status mg_setup(const mg_params *p, const double *k2_dev, void *stream,
                   mg_ctx **out);

/* One V(nu1, nu2) cycle for all nrhs right-hand sides, in place on u_dev
 * (A~_0 u = f): the level-dependent cycle of Sec. 3.1 (eq. cslvariant, coarse
 * right-hand side by eq. erreq1 with c = 1).  res_before: NULL or host array
 * of nrhs doubles receiving ||f - A u|| of the incoming u (unscaled 2-norm),
 * computed inside the cycle; when non-NULL the call synchronises.  With
 * mixed precision or a fixed-shift cycle (sigma_0 != 1) the call performs
 * u <- u + M (f - A u) with the residual in FP64. */
mg_status mg_cycle(mg_ctx *c, double *u_dev, const double *f_dev,
                   double *res_before);

/* mg_cycle for callers that cannot allocate memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * kernels and results, with every work vector, reduction buffer and launch
 * table in a fixed device array of the library (64 MiB per GPU, held until
 * the process ends) instead of the context's own work space; the slot
 * tables are staged through a pinned host buffer allocated by mg_setup.
 * Calls no hipMalloc or hipFree.  Errors: MG_E_INVAL when the context needs
 * more than 64 MiB of work space (roughly more than 2M complex128 fine
 * points times right-hand sides), MG_E_STATE when the current device is not
 * the context's.  Every call on a GPU shares that array: calls that overlap
 * on one GPU (other streams, other host threads, other contexts) race; calls
 * ordered on one stream do not.  res_before as in mg_cycle. */
mg_status mg_cycle_noalloc(mg_ctx *c, double *u_dev, const double *f_dev,
                           double *res_before);

/* Solve A u = f for all right-hand sides to ||f - A u|| / ||f|| <= rtol, by
 * repeated cycles (Sec. 4.1, LVL-MG) or restarted right-preconditioned
 * (F)GMRES with one cycle per outer step (Sec. 4.1, Table 3; flexible as
 * Sec. 3.2.2 requires for the GMRES(3) smoother).
 * u_dev holds the initial guess on entry (zeros for a cold start) and the
 * result on exit.  mode: enum mg_mode.  maxit counts V-cycles (standalone)
 * or outer GMRES steps; restart is the GMRES(m) restart length (1..32,
 * ignored in standalone mode).  iters: NULL or host int[nrhs] receiving the
 * count per rhs.  hist: NULL or host double[nrhs * (maxit + 1)] receiving
 * per rhs the relative residual history (standalone: the ratio of the iterate
 * entering each cycle; GMRES: the initial ratio then the estimate after each
 * step), unused tail entries set to -1.  Standalone mode stops after the
 * first cycle whose incoming iterate met rtol.  Returns MG_OK when every rhs
 * converged, MG_NOT_CONVERGED when one reached maxit, MG_E_DIVERGED when
 * one diverged (others still hold their last iterate).  The call waits for
 * the context's stream on entry and returns once all its work is done; a
 * GMRES/FGMRES solve of several right-hand sides runs up to three groups of
 * them concurrently on streams of the library (same results as one group). */
mg_status mg_solve(mg_ctx *c, double *u_dev, const double *f_dev, int mode,
                   double rtol, int maxit, int restart, int *iters,
                   double *hist);

/* Same as mg_solve for the adjoint system A^H lambda = g (extension, not in
 * the paper): the identical cycle on the conjugate-transposed hierarchy
 * {A~_l^H} (shifts conj(sigma_l)). */
mg_status mg_solve_adjoint(mg_ctx *c, double *lam_dev, const double *g_dev,
                           int mode, double rtol, int maxit, int restart,
                           int *iters, double *hist);

/* grad_dev[i] += sum_r Re(conj(lam_r[i]) u_r[i]): the gradient of a real loss
 * with respect to k^2 when lam = A^{-H} dL/d(conj u) (extension).  grad_dev is
 * a real field of n_x n_y n_z doubles. */
mg_status mg_grad_k2(mg_ctx *c, const double *u_dev, const double *lam_dev,
                     double *grad_dev);

/* y = A~_l x (adjoint != 0: A~_l^H x) for all right-hand sides on level l,
 * vectors laid out like the ABI vectors with level-l sizes (mg_level_dims).
 * The level operator of Sec. 3.1; exposed for parity tests. */
mg_status mg_apply(mg_ctx *c, int level, int adjoint, const double *x_dev,
                   double *y_dev);

/* Tile shape of the cycle kernels on one level.  Shape ids 0, 1, 2 are
 * 64x16, 64x8, 128x8 (2D) and 16x8x4, 32x4x2, 16x4x4 (3D) for the
 * omega-Jacobi kernels and the 3D GMRES(3) kernels; 2D GMRES(3) contexts
 * take ids 0..4: row-marching strips of 56 columns by 32, 16, 8, 4 rows,
 * and (id 4) LDS tiles of 32x16 points that form the powers on a shrinking
 * halo.  omega-Jacobi
 * contexts also take ids 3, 4, 5: plane sweeps of the zero-guess kernels
 * (2D: row segments of 256, 512, 256 points sweeping chunks of 16, 16, 32
 * rows with 320, 576, 320 threads; 3D: columns of 64x8, 32x8, 64x4 points
 * sweeping chunks of 16 planes with 768, 448, 384 threads), with tile shape
 * 0 for the kernels that start from a given iterate.  On the finest level of
 * a 3D GMRES(3) context the power, Gram and pre-smoothing apply passes (and
 * in every 3D context the Arnoldi matvec pass) march columns of 64x4 points
 * through 32 planes whatever the shape; the shape sets the tiles of its
 * prolongation pass.
 * mg_setup picks one per level by timing every shape on the level's own
 * arrays, the level's passes
 * replayed as a graph (levels of at least 1024 points above the coarse
 * tail; other levels use shape 0).  The sweep schedule of the two Arnoldi
 * passes (points per thread, so workgroups per right-hand side) is picked
 * the same way at the context's first GMRES solve.
 * shape >= 0 sets it, shape < 0 only queries; returns the shape in force or
 * a negative mg_status. */
int mg_tile_shape(mg_ctx *c, int level, int shape);

/* Batched solves (extension): the right-hand sides of several contexts --
 * grids of different sizes, one stream, one dimension and precision -- are
 * iterated together: every kernel launch covers all of them (any number of
 * right-hand sides), and a whole restart cycle of the batch (m Arnoldi steps
 * with their V-cycles, the solution update and the new residual; in
 * standalone mode, 8 cycles) is one HIP graph captured at the first solve
 * and replayed; right-hand sides that stop early are skipped by device
 * flags, and the host reads those flags once per graph launch.  Every
 * right-hand side follows its own context's iteration: results equal the
 * single-context solves bit for bit when the tile shapes agree.  The batch
 * borrows the contexts; destroy it before them.  u_dev[i], f_dev[i] are context i's
 * vectors; iters and hist are laid out context after context, rhs after rhs
 * (hist: maxit + 1 doubles per rhs).  Same semantics and statuses as
 * mg_solve; MG_E_INVAL if the contexts do not match. */
typedef struct mg_batch mg_batch;
mg_status mg_batch_create(mg_ctx *const *ctxs, int count, mg_batch **out);
mg_status mg_batch_solve(mg_batch *b, double *const *u_dev,
                         const double *const *f_dev, int mode, double rtol,
                         int maxit, int restart, int *iters, double *hist);
void mg_batch_destroy(mg_batch *b);

/* Number of levels and the interior sizes of one level (n[3], x first). */
int mg_num_levels(const mg_ctx *c);
mg_status mg_level_dims(const mg_ctx *c, int level, int n[3]);
/* Copy the per-level shifts into host sigma[2 * nlevels]. */
mg_status mg_get_sigma(const mg_ctx *c, double *sigma);

/* Kernel timing with HIP events on the context's stream.  enable != 0 starts
 * recording (and clears earlier records); mg_profile_read returns the summed
 * milliseconds, the launch count and the summed algorithmic bytes (the
 * compulsory HBM traffic of each launch: every array it must read once and
 * write once, per grid point times points times right-hand sides) of kernel
 * class `which` (enum mg_kernel_class) since then, synchronising the stream.
 * Any of the three out-pointers may be NULL. */
enum mg_kernel_class {
    MG_K_SMOOTH_RESTRICT_FINE = 0,  /* pre-smooth + residual + restriction, level 0
                                       (GMRES(3): the pass applying the polynomial) */
    MG_K_PROLONG_SMOOTH_FINE = 1,   /* prolongation + correction + post-smooth, level 0
                                       (GMRES(3): prolongation + residual, final apply) */
    MG_K_COARSE_LEVELS = 2,         /* every cycle kernel on levels >= 1 */
    MG_K_COARSEST_SOLVE = 3,
    MG_K_RESIDUAL = 4,
    MG_K_MATVEC_DOT = 5,            /* GMRES: w = A z fused with <v_i, w> */
    MG_K_UPDATE_DOT = 6,            /* GMRES: w -= V h fused with <v_i, w> */
    MG_K_UPDATE_NORM = 7,           /* GMRES: w -= V h fused with ||w|| */
    MG_K_REDUCE = 8,
    MG_K_COMBINE = 9,               /* GMRES: t = V y */
    MG_K_OTHER = 10,
    MG_K_SMOOTH_POWER_FINE = 11,    /* GMRES(3) smoother, level 0: q_i = (A/s) q_{i-1} */
    MG_K_SMOOTH_GRAM_FINE = 12,     /* GMRES(3) smoother, level 0, pre-smoothing: Gram
                                       partials of q_0..q_3                          */
    MG_K_SMOOTH_GRAM_POST_FINE = 13,/* the same after the coarse-grid correction     */
    MG_K_NUM_CLASSES = 14
};
mg_status mg_profile(mg_ctx *c, int enable);
mg_status mg_profile_read(mg_ctx *c, int which, double *total_ms,
                          long long *count, double *bytes);

/* Release everything the context owns.  NULL is accepted; calling it twice
 * on the same pointer is not. */
void mg_destroy(mg_ctx *c);

/* Static description of a status code. */
const char *mg_status_str(mg_status s);

#ifdef __cplusplus
}
#endif

#endif /* MG_H */
