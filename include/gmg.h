/*
 * gmg.h -- C ABI of the MI355X (gfx950) geometric-multigrid-preconditioned
 * conjugate-gradient solver for the variable-coefficient diffusion problem
 *
 *        -div(k grad phi) = f        on the unit cube, phi = 0 on the boundary
 *
 * (Eq. 2 of Sec. 1, discretized by the 7-point finite-difference stencil of
 * the structured-grid Laplace workload of Sec. 4.1).  The preconditioner is one
 * multigrid V-cycle (Alg. 1 of Sec. 2.1.1 applied recursively, factor-2
 * coarsening as in Sec. 1) with Chebyshev-Jacobi smoothing and re-discretized
 * coarse operators; the coarsest level is solved exactly (Sec. 1, Sec. 3.3.1).
 * Coarse levels at or below a size threshold are agglomerated onto one
 * workgroup of a persistent kernel: the in-device counterpart of moving coarse
 * levels onto a smaller communicator (Sec. 3.1, Fig. 1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  * N vertices per side, h = 1/(N-1).  Arrays are C order (z, y, x), x fastest:
 *      vertex vectors  (N, N, N)      -- boundary entries are ignored on input
 *                                        and written as 0 on output
 *      kx              (N, N, N-1)    link (i,j,k)-(i+1,j,k)
 *      ky              (N, N-1, N)    link (i,j,k)-(i,j+1,k)
 *      kz              (N-1, N, N)    link (i,j,k)-(i,j,k+1)
 *    A link is active when one of its end points is interior; values on the
 *    other links are never read.
 *  * The operator is (A u)_p = h^-2 sum_{links f of p} k_f (u_p - u_q(f)).
 *  * Every array pointer is a DEVICE pointer (e.g. a torch tensor's data_ptr()),
 *    FP64, contiguous, owned by the caller.  The library copies what it keeps.
 *  * All work is enqueued on the handle's HIP stream (hipStream_t passed as
 *    void*; NULL = the default stream).  Calls return after their results are
 *    complete on that stream unless stated otherwise.
 *  * Nothing aborts and no exception crosses the ABI: every call returns a
 *    gmg_status; gmg_last_error() gives a per-handle message.
 *  * A handle is not thread-safe; distinct handles are independent.
 *  * Launch-shape overrides (read once, in gmg_create; unset or <= 0 keeps the
 *    measured default; results do not change, only timing, except that the
 *    grouping of partial sums in reductions follows the workgroup count):
 *      GMG_TARGET_WGS_V     workgroups targeted by the V-cycle stencil sweeps
 *                           (smoothing, residual; both precisions)
 *      GMG_TARGET_WGS_64    the same for the outer FP64 apply and true residual
 *    A target sets the z-chunk length of a launch (at least 8 planes where
 *    that still yields 1024 workgroups).
 *      GMG_POST_CHUNK       z-chunk length of the one-sweep post-smoother (32)
 *      GMG_PRE_CHUNK        z-chunk length of the one-sweep pre-smoothing and
 *                           residual (64)
 *    Both are shortened on small levels to keep 1024 workgroups.
 *      GMG_APPLY_WIDTH=128  the outer apply in 128 x 4 tiles also on rows of
 *                           384 points or more (default there: 512 x 1)
 *      GMG_PRE_FUSED=0      the separate pre-smoothing and residual sweeps in
 *                           place of the one-sweep kernel (same results to the
 *                           bit; for tests and measurements)
 */
#ifndef GMG_H
#define GMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gmg_handle gmg_handle;

typedef enum {
    GMG_OK = 0,
    GMG_ERR_ARG = 1,           /* null pointer, bad option value, bad level index */
    GMG_ERR_DIMS = 2,          /* N / levels inconsistent, coarsest level too large */
    GMG_ERR_COEFF = 3,         /* a k on an active link is <= 0, NaN or Inf */
    GMG_ERR_NOMEM = 4,         /* device allocation failed */
    GMG_ERR_HIP = 5,           /* a HIP runtime call or kernel launch failed */
    GMG_ERR_NOT_CONVERGED = 6, /* max_it reached; x holds the last iterate */
    GMG_ERR_BREAKDOWN = 7      /* p.Ap <= 0 or a non-finite residual; x holds the last iterate */
} gmg_status;

typedef enum { GMG_FP64 = 0, GMG_MIXED = 1 } gmg_precision;

/* Rule for the coarse link coefficients of the re-discretized coarse operators
 * (the paper uses re-discretized coarse operators, Sec. 4.3, without giving
 * the averaging).  A coarse link spans two fine links in series; the 3x3 lines
 * around it are weighted by (1/4,1/2,1/4) x (1/4,1/2,1/4).  Along the link the
 * two fine values p, q combine as (p+q)/2 (ARITHMETIC) or 2pq/(p+q) (HARMONIC). */
typedef enum { GMG_COARSE_ARITHMETIC = 0, GMG_COARSE_HARMONIC = 1 } gmg_coarse_rule;

typedef struct {
    int32_t n;              /* vertices per side; n >= 3, n <= 5440 and (n-1) % 2^(levels-1) == 0 */
    int32_t levels;         /* >= 1; coarsest level has at most 4096 interior unknowns */
    int32_t cheb_degree;    /* Chebyshev steps per smoothing (pre and post), 1..8; default 2 */
    double cheb_lo;         /* Chebyshev interval of D^-1 A, default [0.25, 2.0] */
    double cheb_hi;
    int32_t switch_n;       /* 0: grid launches on every level.  Else levels with
                               N_l <= switch_n run inside one persistent kernel */
    int32_t persistent_wgs; /* workgroups of the persistent kernel, 1..32 (default 1).  More
                               than one: a co-resident team (cooperative launch) packed
                               onto one XCD when it fits, with a device-wide barrier
                               between sweeps; results are identical for any team size */
    int32_t precision;      /* gmg_precision.  MIXED: V-cycle in FP32 with BF16 link
                               coefficients (round-to-nearest-even from FP64; Galerkin
                               levels FP32); x, r, q = A p, the dot products and the
                               coarsest Cholesky in FP64; the search direction p is
                               formed in FP64 and stored in FP32 */
    int32_t coarse_rule;    /* gmg_coarse_rule, default ARITHMETIC */
    int32_t coeff_is_log;   /* 1: kx/ky/kz hold ln k (natural log) instead of k */
    int32_t check_every;    /* host reads the convergence flag every this many PCG
                               iterations (0 = automatic by grid size) */
    int32_t coarse_solver;  /* 0: exact Cholesky on the coarsest level.  1: truncated
                               hierarchy (the truncation strategy of Sec. 1 / Sec. 3.3.1):
                               the coarsest level, of any size, is solved inexactly by
                               Jacobi-preconditioned CG on grid-wide launches; needs
                               switch_n = 0 */
    double coarse_rtol;     /* coarse CG relative residual target (default 1e-4) */
    int32_t coarse_max_it;  /* coarse CG iteration cap (default 500) */
    int32_t flexible;       /* 1: Polak-Ribiere beta in the outer CG, for preconditioners
                               that change between iterations (inexact coarse solves) */
    int32_t switch2_n;      /* with persistent_wgs > 1: levels with N_l <= switch2_n leave
                               the team for a single workgroup (multi-stage agglomeration,
                               the two-stage repartitioning of Sec. 4.2, Tab. 3); 0 = off */
    int32_t galerkin;       /* g > 0: levels l >= g use the Galerkin operator R A P (trilinear P,
                               R = P^T / 8; 27 coefficients per vertex), each from the level
                               above it; levels below g keep re-discretized links.  g = 1 is
                               Galerkin throughout (Sec. 3.3.2), g > 1 the hybrid construction
                               of Sec. 3.3.3.  0 = re-discretized throughout (default). */
    int32_t persistent_lds; /* 1 (default): with persistent_wgs == 1, the agglomerated levels
                               are copied into the workgroup's LDS for the coarse cycle when they
                               all fit (link levels only); 0: they are swept in HBM/L2.  The
                               result is the same either way. */
    int32_t post_fused;     /* on grid-path link levels with cheb_degree 2: 1 = the
                               post-smoothing runs as one sweep that keeps the first Chebyshev
                               iterate in LDS; 0 = two sweeps through HBM; 2 (default) = the
                               library's choice, currently the one sweep in both precisions
                               (measured at 513^3: FP64 1.7 ms vs 2.9 ms; MIXED 1.02 ms vs
                               1.21 ms, a 3.9 % shorter MIXED solve although the one sweep is
                               instruction-bound at 43 % of HBM peak).  Same values to the bit;
                               only the partial sums of r.z are grouped differently. */
} gmg_options;

typedef struct {
    int32_t iterations;   /* PCG iterations (updates of x) */
    int32_t restarts;     /* MIXED: restarts from the true residual */
    double rel_res;       /* recursive ||r|| / ||f|| at exit */
    double rel_res_true;  /* ||f - A x|| / ||f|| at exit, FP64 */
    double setup_ms;      /* device time of gmg_create / the last gmg_set_coefficients */
    double solve_ms;      /* device time of the solve (HIP events on the stream) */
    int32_t coarse_iterations; /* truncated hierarchy: coarse CG iterations over the solve */
} gmg_info;

/* Fill *opt with the defaults above for n vertices per side and
 * levels = log2(n-1) (coarsest 3^3), FP64, no persistent switch. */
void gmg_default_options(gmg_options *opt, int32_t n);

/* Build the hierarchy (the per-level operators, smoothers and transfers of
 * Sec. 2.1.1): copy k (device, FP64, face shapes) into the library's padded
 * layout, derive the coarse coefficients level by level (re-discretized, or
 * R A P from the galerkin level on, with each Galerkin level's Chebyshev
 * interval), the BF16 copies (MIXED), and the Cholesky factor of the dense
 * coarsest operator.  Allocates every device buffer the solver needs (no
 * allocation happens in gmg_solve).  On success *out owns them until
 * gmg_destroy; on failure *out is NULL and nothing stays allocated.
 * Errors: GMG_ERR_ARG (null pointer, option out of range), GMG_ERR_DIMS,
 * GMG_ERR_COEFF (bad k, or a coarsest operator that is not positive
 * definite), GMG_ERR_NOMEM, GMG_ERR_HIP. */
gmg_status gmg_create(const gmg_options *opt, const double *kx, const double *ky, const double *kz,
                      void *stream, gmg_handle **out);

/* Replace the coefficients (same N, levels, options); rebuilds every derived
 * level and the coarsest factor without reallocating.  Everything, the check
 * of k and of the coarsest factor included, is enqueued on the handle's
 * stream and the call returns without waiting (with Galerkin levels it waits
 * for their Lanczos intervals); k must stay valid until that work has run.
 * A bad k (<= 0, NaN or Inf on an active link) or a coarsest operator that is
 * not positive definite makes the next gmg_solve / gmg_adjoint_gradient, and
 * every one after it until valid coefficients are set, return GMG_ERR_COEFF
 * before any iteration.  Errors here: GMG_ERR_ARG, GMG_ERR_HIP. */
gmg_status gmg_set_coefficients(gmg_handle *h, const double *kx, const double *ky, const double *kz);

/* Change the stream used by later calls. */
gmg_status gmg_set_stream(gmg_handle *h, void *stream);

/* PCG solve of A x = f (Sec. 2.1, CG preconditioned by one V-cycle).  Stops
 * when ||r||_2 <= rtol ||f||_2 (recursive residual; FP64 mode) or when the
 * FP64 true residual also passes (MIXED: otherwise r is replaced by f - A x
 * and CG restarts).  x0 may be NULL (zero initial guess).  f, x, x0: (N,N,N).
 * Returns GMG_OK, GMG_ERR_NOT_CONVERGED or GMG_ERR_BREAKDOWN with x written
 * in every case; info may be NULL. */
gmg_status gmg_solve(gmg_handle *h, const double *f, double *x, const double *x0, double rtol,
                     int32_t max_it, gmg_info *info);

/* Adjoint gradient.  Solves A lambda = dl_dphi with the same PCG (A is
 * symmetric), then for every active link f = (p,q)
 *     g_f = dL/d(ln k_f) = -h^-2 k_f (lambda_p - lambda_q)(phi_p - phi_q)
 * (boundary values are 0); links between two boundary vertices get 0.
 * phi, dl_dphi, lambda: (N,N,N); g_x, g_y, g_z: face shapes.  lambda may be
 * NULL.  Status as gmg_solve. */
gmg_status gmg_adjoint_gradient(gmg_handle *h, const double *phi, const double *dl_dphi, double *g_x,
                                double *g_y, double *g_z, double *lambda, double rtol, int32_t max_it,
                                gmg_info *info);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the solve
 * of gmg_create + gmg_solve + gmg_destroy in one call that allocates nothing.
 * The hierarchy is built in a static device workspace of 64 MiB that each GPU
 * the library runs on holds until the process ends (enough for N <= 65 in
 * either precision at any level count); the handle and its host state
 * records are static too, and no event, pinned buffer or heap object is
 * created.  Options as gmg_create except galerkin, which must be 0.  k, f, x,
 * x0 (may be NULL), rtol, max_it, info as gmg_create / gmg_solve; stream as
 * gmg_create.  Results equal those of gmg_solve with the same options.
 * The workspace keeps the last call's contents and every call clears what it
 * uses; calls that overlap on one GPU (other threads, other streams) race.
 * Errors: GMG_ERR_ARG (null pointer, option out of range, galerkin != 0),
 * GMG_ERR_DIMS (also: the hierarchy does not fit the workspace),
 * GMG_ERR_COEFF, GMG_ERR_HIP, and the solve statuses of gmg_solve;
 * gmg_last_error(NULL) gives the message of the last call on the current
 * device.  Timings in info are host-clock figures. */
gmg_status gmg_solve_static(const gmg_options *opt, const double *kx, const double *ky, const double *kz,
                            const double *f, double *x, const double *x0, double rtol, int32_t max_it, void *stream,
                            gmg_info *info);

/* ---- test hooks: each runs one step of the V-cycle of Sec. 2.1.1 (Alg. 1:
 * smoothing, residual restriction, prolongation and correction, coarse solve)
 * on level `level`, in the handle's V-cycle precision (FP32/BF16 in MIXED
 * mode, with FP64 in and out).  Vectors are (N_l, N_l, N_l) device arrays
 * (natural layout, boundary entries ignored on input, 0 on output).  They use
 * the handle's level buffers, so they must not overlap a solve on the same
 * handle.  GMG_ERR_ARG for a null vector or a level out of range. */
int32_t gmg_level_n(const gmg_handle *h, int32_t level);   /* N_l, or -1 */
/* y = A_l x in the V-cycle precision (Eq. 2 discretized with the 7-point
 * stencil of Sec. 4.1 on level l; the 27-point R A P on Galerkin levels). */
gmg_status gmg_apply_operator(gmg_handle *h, int32_t level, const double *x, double *y);
/* y = A x on level 0 with the FP64 operator of the outer CG (the kernel that
 * forms q = A p in every iteration), in either precision mode.  x, y: (N,N,N). */
gmg_status gmg_apply_outer_operator(gmg_handle *h, const double *x, double *y);
/* x <- Chebyshev-Jacobi smoothing of A_l x = b from x (x0_zero: from 0). */
gmg_status gmg_debug_smooth(gmg_handle *h, int32_t level, const double *b, double *x, int32_t x0_zero);
/* b_c = R (b - A_l x) on level+1 (full weighting). */
gmg_status gmg_debug_residual_restrict(gmg_handle *h, int32_t level, const double *b, const double *x,
                                       double *b_coarse);
/* x += P e, e on level+1 (trilinear). */
gmg_status gmg_debug_prolong(gmg_handle *h, int32_t level, const double *e_coarse, double *x);
/* Coarsest-level solve: x = A_c^-1 b by the FP64 Cholesky factor, or (coarse_solver
 * = 1) the inexact Jacobi-CG of the truncated hierarchy. */
gmg_status gmg_debug_coarse_solve(gmg_handle *h, const double *b, double *x);
/* z = B r, one V-cycle on level 0 (uses the handle's switch level). */
gmg_status gmg_debug_vcycle(gmg_handle *h, const double *r, double *z);
/* Copy level coefficients out in face shapes (MIXED: the BF16 values). */
gmg_status gmg_get_level_coefficients(gmg_handle *h, int32_t level, double *kx, double *ky, double *kz);

/* Dynamic LDS bytes of the one-workgroup persistent kernel when the handle
 * runs its agglomerated levels out of LDS (option persistent_lds), else 0. */
uint64_t gmg_persistent_lds_bytes(const gmg_handle *h);

/* Chebyshev interval [*lo, *hi] of D^-1 A used by the smoother on `level`
 * (host pointers).  The option interval on re-discretized levels; on a
 * smoothed Galerkin level [1.1 lam cheb_lo/cheb_hi, 1.1 lam] with lam the
 * largest Ritz value of 20 Lanczos steps on D^-1 A in the D inner product
 * (the bound 2 of the 7-point operator does not hold for R A P). */
gmg_status gmg_get_level_interval(gmg_handle *h, int32_t level, double *lo, double *hi);

/* Galerkin operator of `level` (>= the handle's galerkin level; GMG_ERR_ARG
 * otherwise) in FP64, written to the device array a27 of N_l^3 * 27 doubles in
 * natural order: a27[((k*N + j)*N + i)*27 + (dz+1)*9 + (dy+1)*3 + (dx+1)] is
 * the coefficient of u(i+dx, j+dy, k+dz) in row (i, j, k); boundary rows and
 * couplings to boundary vertices are 0.  Synchronizes the stream. */
gmg_status gmg_get_level_stencil(gmg_handle *h, int32_t level, double *a27);

/* ---- kernel timing.  While profiling is on, every launch of a class on the
 * FINEST level (plus the coarse-level classes) is bracketed by HIP events on
 * the handle's stream; gmg_profile_get returns the launch count and the summed
 * device time.  Used by the benchmark to measure kernels live. */
typedef enum {
    GMG_K_APPLY_DOT = 0,      /* q = A p and partial p.q (outer FP64 operator) */
    GMG_K_RESIDUAL = 1,       /* r = f - A x (FP64 true residual) */
    GMG_K_UPDATE_R = 2,       /* r -= alpha q, partial r.r (MIXED: and the FP32 copy of r) */
    GMG_K_UPDATE_P = 3,       /* p = z (start of a CG recurrence) */
    GMG_K_CHEB_FIRST = 4,     /* first Chebyshev step from zero (MIXED: converts r) */
    GMG_K_CHEB_STEP = 5,      /* Chebyshev step without previous iterate */
    GMG_K_CHEB_STEP_PREV = 6, /* three-term Chebyshev step (previous iterate) */
    GMG_K_CHEB_STEP_DOT = 7,  /* last post-smoothing step + partial r.z */
    GMG_K_LEVEL_RESIDUAL = 8, /* r = b - A x inside the V-cycle */
    GMG_K_PROLONG = 9,        /* x += P e */
    GMG_K_PERSISTENT = 10,    /* persistent coarse-level kernel (all levels below the switch) */
    GMG_K_COARSE_SOLVE = 11,  /* grid-path coarsest Cholesky solve */
    GMG_K_FACE_GRADIENT = 12, /* adjoint link gradient */
    GMG_K_RESTRICT = 13,      /* b_c = R r (full weighting) */
    GMG_K_UPDATE_XP = 14,     /* x += alpha p, p = z + beta p */
    GMG_K_CHEB_PRE2 = 15,     /* first two Chebyshev steps from zero, fused */
    GMG_K_CHEB_POST2 = 16,    /* post-smoothing, both Chebyshev steps in one sweep (+ partial r.z) */
    GMG_K_PRE2_RES = 17,      /* pre-smoothing (two Chebyshev steps from zero) and the residual in one sweep */
    GMG_K_COUNT = 18
} gmg_kernel_class;
gmg_status gmg_profile_start(gmg_handle *h);  /* clear counters, start recording */
gmg_status gmg_profile_stop(gmg_handle *h);   /* stop recording, wait for the stream */
gmg_status gmg_profile_get(gmg_handle *h, int32_t kclass, int32_t *launches, double *total_ms);
const char *gmg_kernel_class_name(int32_t kclass);

/* Plain device-to-device copy of `bytes` on `stream` with nontemporal 16-byte
 * loads and stores; returns after it completes.  planes = 1: one element per
 * thread.  planes > 1: the buffers are `planes` equal slabs and each thread
 * copies its element of every slab in turn, the access pattern of the
 * z-marching stencil kernels.  GMG_ERR_ARG for null pointers, planes < 1, a
 * size that is not a multiple of 16 * planes or needs more than 2^31 - 1
 * workgroups.  Used to calibrate the profiler's HBM byte counters and to
 * measure achievable copy bandwidth. */
gmg_status gmg_calibration_copy(void *dst, const void *src, uint64_t bytes, int32_t planes, void *stream);

void gmg_destroy(gmg_handle *h);
const char *gmg_status_string(gmg_status s);
/* The message of the handle's last error; with h = NULL, that of the last
 * gmg_solve_static call on the current device. */
const char *gmg_last_error(const gmg_handle *h);

#ifdef __cplusplus
}
#endif
#endif /* GMG_H */
