/*
 * hsweep -- sweeping preconditioner for the 2D Helmholtz equation with PML,
 * Schur complements in hierarchical-matrix form, on one AMD MI355X (gfx950).
 *
 * Method: B. Engquist and L. Ying, "Sweeping preconditioner for the
 * Helmholtz equation: hierarchical matrix representation" (2010).
 *
 *   Problem   Delta u + omega^2 / c(x)^2 u = f on (0,1)^2 with a PML of
 *             width eta on every side and u = 0 on the boundary
 *             (Sec. 1, eq. helm; Sec. 2.1, eq. sigma).
 *   Operator  the symmetric 5-point stencil of Sec. 2.1 (eq. helmd) on the
 *             interior points p_{i,j} = (i h, j h), h = 1/(n+1), unknowns
 *             ordered row by row (x1 index fastest); A = A^t.
 *   Factor    layer-by-layer block LDL^t (eq. Afact) with every Schur
 *             complement S_m = A_{m,m} - A_{m,m-1} S_{m-1}^{-1} A_{m-1,m}
 *             formed and inverted as a weakly admissible H-matrix
 *             (Sec. 2.3; Alg. 2.3).
 *   Apply     the forward/backward sweep with the compressed inverses
 *             T_m ~ S_m^{-1} (Alg. 2.4): the preconditioner M.
 *   Solve     GMRES on the preconditioned system (Sec. 2.4), here
 *             right-preconditioned flexible GMRES in FP64 so that the
 *             stopping test is on the true residual ||f - A u|| / ||f||.
 *
 * Layouts.  A 2D field on the grid is n*n values, index (j-1)*n + (i-1)
 * for p_{i,j} (row j = layer j).  Complex values are interleaved
 * (re, im) pairs of double: "complex128".  A batch of nrhs fields is
 * nrhs consecutive fields.
 *
 * Memory.  c may be a host or a device pointer (detected at run time).
 * f, u, mu and grad passed to apply/solve/grad are DEVICE pointers owned by
 * the caller; the library never keeps them past the call.  The library owns
 * the context, the coefficient arrays, the factor store and its work
 * buffers (device memory, freed by hsweep_destroy).
 *
 * Streams.  `stream` is a hipStream_t (NULL = the default stream).  apply,
 * stencil and grad are asynchronous on that stream; factor, factor_batch,
 * solve and solve_batch synchronize on it before returning (they read pivot
 * status or residuals back to the host).
 *
 * Errors.  Every function returns HSWEEP_OK (0) or a negative code; no
 * exception crosses this interface.  Arguments are validated on the host
 * before any device work.  hsweep_last_error() returns a message for the
 * last failure on the calling thread.  A context is not thread-safe;
 * distinct contexts are independent.
 */
#ifndef HSWEEP_H
#define HSWEEP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HSWEEP_OK          0
#define HSWEEP_EINVAL     -1  /* an argument is out of range */
#define HSWEEP_ESTATE     -2  /* call out of order (e.g. apply before factor) */
#define HSWEEP_ENOMEM     -3  /* device or host allocation failed */
#define HSWEEP_EDEVICE    -4  /* HIP runtime error or no usable GPU */
#define HSWEEP_ESINGULAR  -5  /* zero pivot in a dense leaf or core inverse */
#define HSWEEP_ENOCONV    -6  /* GMRES reached maxit; u holds the last iterate */

#define HSWEEP_C128 0         /* factors and sweeps in complex128 */
#define HSWEEP_C64  1         /* factors and sweeps in complex64, FP64 outer loop */

/* Sweep directions (Sec. 2.4): the layers are the grid rows swept upward
 * (+x2, the paper's presentation) or downward (-x2), or the grid columns
 * swept rightward (+x1) or leftward (-x1).  Fields keep the natural layout
 * whatever the direction.  HSWEEP_DIR_MX1 is currently rejected (EINVAL). */
#define HSWEEP_DIR_PX2 0
#define HSWEEP_DIR_MX2 1
#define HSWEEP_DIR_PX1 2
#define HSWEEP_DIR_MX1 3

/* Edges of the unit square (Dirichlet data, Sec. 2.5). */
#define HSWEEP_EDGE_X1_0 0    /* x1 = 0 */
#define HSWEEP_EDGE_X1_1 1    /* x1 = 1 */
#define HSWEEP_EDGE_X2_0 2    /* x2 = 0 */
#define HSWEEP_EDGE_X2_1 3    /* x2 = 1 */

/* pml_sides entry for a side that carries the second-order absorbing
 * boundary condition of Engquist and Majda (Sec. 3, other boundary
 * conditions) instead of a layer: du/dn = i k u + (i/(2k)) d2u/dt2,
 * k = omega/c, imposed at the half point between the boundary node and the
 * first row of unknowns, which eliminates the boundary value
 * u_b = a u_0 + g D_tt u_0 (a = (2 + ikh)/(2 - ikh), g = ih/(k(2 - ikh)),
 * D_tt the second difference along the side).  That row's diagonal and its
 * couplings along the side change (flux form with one weight per edge, the
 * mean of its two end points, so A = A^t still holds); at an end of the side
 * the flux goes to the corner value, zero next to a side without the
 * condition and dropped next to one with it. */
#define HSWEEP_SIDE_ABC (-2)

/* Admissibility of the layer H-matrices (Sec. 2.3).  WEAK: every
 * off-diagonal block of the bisection is low rank (rank <= `rank`), the
 * inverse kept in a Woodbury form; all precisions and batching.  STRONG:
 * only blocks of well-separated clusters (at least one cluster of the same
 * level between them) are low rank, rank <= `rank` at relative tolerance
 * rank_tol; the near field stays dense down to the leaves, products of two
 * non-low-rank blocks that land on a low-rank block are built by randomized
 * SVD (oversampling 8) and the inverse by recursive 2 x 2 block inversion in
 * that format.  STRONG runs in complex128 only (EINVAL otherwise), one
 * context at a time (EINVAL in the batch calls, hsweep_apply_noalloc and
 * hsweep_factor_profile); n_p = n (no padding). */
#define HSWEEP_ADM_WEAK   0
#define HSWEEP_ADM_STRONG 1

typedef struct hsweep_ctx hsweep_ctx;

/* Options of the factorization and of GMRES (set before hsweep_factor). */
typedef struct hsweep_opts {
    int    leaf;        /* dense leaf size b (power of two, 4..64); the padded
                           layer width is n_p = b * 2^L >= n */
    int    rank;        /* maximum rank r of every off-diagonal block: 2, 4, 8
                           or 16, with 1 + r * levels <= 64 */
    double rank_tol;    /* keep singular values > rank_tol * sigma_1 of the block
                           (0 keeps all up to `rank`) */
    double pml_C;       /* PML constant C of eq. sigma (> 0); default 20 */
    int    precision;   /* HSWEEP_C128 or HSWEEP_C64 */
    int    dense;       /* 1: dense uncompressed Schur complements (leaf = n_p,
                           no low-rank levels) -- the exact Alg. 2.1/2.2 */
    int    restart;     /* GMRES restart length (1..200) */
    int    rhs_group;   /* right-hand sides per sweep workgroup, each layer's
                           factors loaded once for the group: 1, 4 (where a
                           grouped kernel exists for the plan, else 1), or
                           0 = automatic */
    int    direction;   /* sweep direction, HSWEEP_DIR_* */
    int    pml_sides[4];/* absorbing-layer width in grid points on the sides
                           x1 = 0, x1 = 1, x2 = 0, x2 = 1; 0 = zero Dirichlet
                           condition on that side (Sec. 2.5); -1 = the width
                           given to hsweep_setup; HSWEEP_SIDE_ABC = no layer
                           and the absorbing boundary condition.  The two
                           widths of an axis must sum to less than n. */
    int    admissibility; /* HSWEEP_ADM_WEAK (default) or HSWEEP_ADM_STRONG */
} hsweep_opts;

/* Fill `o` with the defaults: leaf 16, rank 8, rank_tol 1e-6, C = 20,
 * complex128, compressed, restart 40, automatic right-hand-side groups,
 * sweep direction +x2, the setup's layer width on every side, weak
 * admissibility. */
void hsweep_default_opts(hsweep_opts* o);

/* Create a context for velocity c (n*n doubles, layout above; every value
 * finite and > 0), angular frequency omega (finite, > 0), PML width `pml`
 * in grid points (eta = pml*h, 0 <= pml and 2*pml < n) and n interior
 * points per side (3 <= n <= 8191).  Builds the PML profile and the
 * stencil coefficients on the device (Sec. 2.1).  On success *out owns the
 * context; on failure *out is NULL.  Validation errors -> HSWEEP_EINVAL. */
int hsweep_setup(const double* c, double omega, int pml, int n, hsweep_ctx** out);

/* Replace the options (EINVAL if out of range).  Invalidates any factor. */
int hsweep_set_opts(hsweep_ctx* ctx, const hsweep_opts* o);
int hsweep_get_opts(const hsweep_ctx* ctx, hsweep_opts* o);

/* Layer width n_p, number of low-rank levels L and bytes of the factor
 * store after hsweep_factor (0 before). */
int hsweep_plan_info(const hsweep_ctx* ctx, int* n_p, int* levels, size_t* factor_bytes);

/* Alg. 2.3 on the device: for m = 1..n form S_m = A_{m,m} - D_m T_{m-1} D_m
 * in H-form (recompressed to rank <= r), invert it, and keep T_m in the
 * factor store.  The layer loop is captured once as a HIP graph and
 * replayed on later calls.  Synchronizes `stream`; ESINGULAR on a zero
 * pivot. */
int hsweep_factor(hsweep_ctx* ctx, void* stream);

/* u = M f for nrhs right-hand sides (Alg. 2.4): f, u are device
 * complex128 arrays of nrhs*n*n entries; f and u may not overlap.
 * Asynchronous on `stream`.  ESTATE before hsweep_factor. */
int hsweep_apply(hsweep_ctx* ctx, const void* f, void* u, int nrhs, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): u = M f as
 * hsweep_apply computes it, with the same kernels, but the sweep's work
 * vectors live in a static device array of HSWEEP_NOALLOC_SCRATCH_BYTES per
 * GPU (its address is taken once per device by hsweep_setup) instead of
 * context memory allocated on first use.  No hipMalloc, hipFree or other
 * allocating call is made.  EINVAL if nrhs * n * n_p * (8 bytes for
 * complex64 factors, 16 for complex128) exceeds HSWEEP_NOALLOC_SCRATCH_BYTES.
 * Every call on one GPU shares that array: calls that overlap in time on
 * one GPU (other streams, other threads, other contexts) race and must be
 * serialized by the caller.  The kernels write every scratch entry they
 * read, so no clearing is needed between calls.  Asynchronous on `stream`;
 * ESTATE before hsweep_factor. */
#define HSWEEP_NOALLOC_SCRATCH_BYTES (32u << 20)
int hsweep_apply_noalloc(hsweep_ctx* ctx, const void* f, void* u, int nrhs, void* stream);

/* y = A x for nrhs fields (the FP64 5-point operator, eq. helmd).  Device
 * complex128 arrays; asynchronous. */
int hsweep_stencil(hsweep_ctx* ctx, const void* x, void* y, int nrhs, void* stream);

/* Flexible GMRES in FP64 with M as right preconditioner, x0 = 0, until
 * ||f_k - A u_k|| <= tol ||f_k|| for every k < nrhs or maxit iterations.
 * iters[k] and relres[k] (host arrays of nrhs, may be NULL) receive the
 * iteration count and the final true relative residual of each right-hand
 * side.  Returns ENOCONV if any right-hand side missed tol (u holds the
 * last iterate).  Synchronizes `stream`. */
int hsweep_solve(hsweep_ctx* ctx, const void* f, void* u, int nrhs, double tol,
                 int maxit, int* iters, double* relres, void* stream);

/* Adjoint solve for the gradient of a real functional J(u) of the solution
 * u = A^{-1} f (configs with a receiver misfit, Sec. 2.1: A = A^t).  g holds
 * dJ/dRe(u) + i dJ/dIm(u) for nrhs fields (device complex128, nrhs*n*n).
 * Solves A mu = conj(g) with the same factorization and flexible GMRES as
 * hsweep_solve (tol, maxit, iters, relres as there) and, when grad_f is not
 * NULL, writes grad_f = conj(mu) = dJ/dRe(f) + i dJ/dIm(f).  The velocity
 * gradient follows from hsweep_grad_c(ctx, u, mu, ...).  g, mu and grad_f
 * must not overlap.  Synchronizes `stream`; ENOCONV as hsweep_solve (mu and
 * grad_f then hold the last iterate). */
int hsweep_solve_adjoint(hsweep_ctx* ctx, const void* g, void* mu, void* grad_f, int nrhs, double tol,
                         int maxit, int* iters, double* relres, void* stream);

/* Device bytes the library allocates for this context with its current
 * options: *factor_bytes for setup and hsweep_factor (coefficients, layer
 * operators, factor store and the factorization's per-layer work) and
 * *solve_bytes for an hsweep_solve of nrhs right-hand sides (sweep work
 * vectors, the GMRES basis and residual fields, small reduction arrays).
 * Either pointer may be NULL.  Host-only; EINVAL if nrhs is out of range.
 * With HSWEEP_ADM_STRONG the factor store is known only after
 * hsweep_factor (0 before) and the factorization's scratch is not counted. */
int hsweep_workspace_bytes(const hsweep_ctx* ctx, int nrhs, size_t* factor_bytes, size_t* solve_bytes);

/* Dirichlet data u = b on one edge (HSWEEP_EDGE_*) moved to the right-hand
 * side (Sec. 2.5, depth extrapolation): for each of nrhs fields, the row of
 * unknowns next to the edge gets f -= (coupling to its boundary neighbour,
 * eq. helmd) * b.  b: device complex128, nrhs * n values along the edge
 * (index i-1 for an x2 edge, j-1 for an x1 edge); f: device complex128,
 * nrhs * n * n, updated in place.  The side of the edge should have no
 * absorbing layer (pml_sides 0 there); EINVAL if it carries the absorbing
 * boundary condition.  Asynchronous on `stream`. */
int hsweep_dirichlet_forcing(hsweep_ctx* ctx, int edge, const void* b, void* f, int nrhs, void* stream);

/* Gradient of a real functional with respect to c through the adjoint
 * fields: grad[p] = sum_k Re( mu_k[p] u_k[p] 2 omega^2 / ((s1 s2)[p] c[p]^3) ),
 * the c-derivative of the diagonal of A (eq. helmd) contracted with the
 * adjoint mu_k = A^{-1} conj(g_k) (A = A^t).  u, mu: device complex128,
 * nrhs*n*n; grad: device double, n*n (overwritten).  Asynchronous.  EINVAL
 * when a side carries the absorbing boundary condition (its rows depend on c
 * through k as well, which this formula leaves out). */
int hsweep_grad_c(hsweep_ctx* ctx, const void* u, const void* mu, int nrhs,
                  void* grad, void* stream);

/* Several independent problems factored together (Alg. 2.3 for each):
 * contexts with the same leaf size and rank form a group, and every layer
 * step of a group is launched once for all its contexts whose layer loop
 * has not finished; groups run one after the other.  All contexts must
 * have the same precision.  Synchronizes `stream`. */
int hsweep_factor_batch(hsweep_ctx** ctxs, int count, void* stream);

/* One flexible-GMRES solve per context (one right-hand side each, Sec. 2.4
 * preconditioned by each context's sweep, Alg. 2.4), all contexts in one
 * iteration loop: every GMRES step launches the sweep once for all
 * contexts with the same leaf size and rank (one workgroup per context),
 * the FP64 vector kernels once for all, and the stencil once per context.
 * Each right-hand side stops on its own true residual.  f[k], u[k]: device
 * complex128 fields of context k (n_k * n_k entries).  iters, relres: host
 * arrays of count.  All contexts factored, same precision and device, no
 * context twice, count <= 4096.  The Krylov work buffers belong to
 * ctxs[0] (its restart length applies).  Synchronizes `stream`. */
int hsweep_solve_batch(hsweep_ctx** ctxs, int count, const void* const* f, void* const* u,
                       double tol, int maxit, int* iters, double* relres, void* stream);

/* Release every resource of the context (NULL is allowed). */
void hsweep_destroy(hsweep_ctx* ctx);

/* Message for the last error on this thread ("" if none). */
const char* hsweep_last_error(void);

/* Factor as hsweep_factor does, but with plain launches (no graph) and HIP
 * events recorded on `stream` around each kernel class, every layer queued
 * before one synchronization.  out[0]: total milliseconds of the layer
 * kernels (recompression and leaves, one launch per layer), out[1]: total
 * milliseconds of the Woodbury kernels (L+1 launches per layer), out[2]:
 * number of layers.  count >= 3.  The factor is usable afterwards.
 * For measurement (Alg. 2.3 timed per kernel); synchronizes `stream`. */
int hsweep_factor_profile(hsweep_ctx* ctx, void* stream, double* out, int count);

/* Per-phase device times in milliseconds of the last factor and solve on
 * this context, measured with HIP events: out[0] factor, out[1] sweep
 * (all applies of the last solve), out[2] stencil, out[3] Krylov vector
 * work, out[4] number of applies in the last solve. */
int hsweep_timings(const hsweep_ctx* ctx, double* out, int count);

/* ---- 3D (Sec. 4): the n x n x n unit-cube grid, h = 1/(n+1), unknowns
 * u[(k-1) n^2 + (j-1) n + (i-1)] at (i h, j h, k h) (x1 fastest, then x2,
 * then x3), absorbing layers of `pml` points on all six sides, the 7-point
 * operator of the equation divided by s1 s2 s3 (each edge coefficient
 * s_a(half node) / (product of the other two s at the node) / h^2, the
 * centre omega^2/(s1 s2 s3 c^2) minus the six couplings), zero Dirichlet
 * values outside.  Swept face by face (faces x3 = const) with strongly
 * admissible H-matrix factors of the face Schur complements on quadtree
 * face clusters (boxes bisected in x1, then x2; boxes of one quadtree
 * level are well separated when they differ by more than one box in x1 or
 * x2).  Complex128; fields are device complex128 arrays of nrhs * n^3.
 * Errors as in 2D, message in hsweep_last_error. */
typedef struct hsweep3_ctx hsweep3_ctx;

/* Context for velocity c (n^3 doubles, host or device, finite and > 0),
 * omega > 0, layer width pml (2 pml < n), 3 <= n <= 255.  Defaults: leaf 16
 * face points, rank 2, rank_tol 1e-6 (the paper's 3D setting), restart 40. */
int hsweep3_setup(const double* c, double omega, int pml, int n, hsweep3_ctx** out);
/* Uses leaf (face points per leaf box, 1..1024), rank (1..64), rank_tol,
 * pml_C and restart of `o`; precision must be HSWEEP_C128 and
 * admissibility HSWEEP_ADM_STRONG (EINVAL otherwise).  Invalidates the
 * factors. */
int hsweep3_set_opts(hsweep3_ctx* ctx, const hsweep_opts* o);
/* The face factors T_m = S_m^{-1} (Alg. 2.3 face by face); synchronizes. */
int hsweep3_factor(hsweep3_ctx* ctx, void* stream);
/* u = M f, the face-by-face sweep (Alg. 2.4), nrhs fields. */
int hsweep3_apply(hsweep3_ctx* ctx, const void* f, void* u, int nrhs, void* stream);
/* y = A x in FP64. */
int hsweep3_stencil(hsweep3_ctx* ctx, const void* x, void* y, int nrhs, void* stream);
/* A u = f by right-preconditioned flexible GMRES as hsweep_solve. */
int hsweep3_solve(hsweep3_ctx* ctx, const void* f, void* u, int nrhs, double tol, int maxit, int* iters,
                  double* relres, void* stream);
/* Binary levels of the face cluster tree and bytes of the stored face
 * factors (0 before hsweep3_factor). */
int hsweep3_plan_info(const hsweep3_ctx* ctx, int* levels, size_t* factor_bytes);
void hsweep3_destroy(hsweep3_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* HSWEEP_H */
