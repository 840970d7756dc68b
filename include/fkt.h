/*
 * fkt.h -- C ABI of the MI355X Fast Kernel Transform library (libfkt.so).
 *
 * The library multiplies an isotropic kernel matrix by vectors,
 *     z_i = sum_j K(|r_i - r_j|) x_j                       (paper eq. nbody),
 * in O(N log N) work with the Fast Kernel Transform (Ryan, Ament, Gomes,
 * Damle, arXiv 2106.04487): a binary space-partition tree (Sec. 3.1), far
 * sets by the distance criterion (eq. accparam), dense near-field blocks
 * and a far field compressed through the truncated expansion of Theorem 3.1
 * (eq. finaltrunc) as source-to-multipole moments followed by
 * multipole-to-target evaluation (Algorithm 1).
 *
 * Conventions for every entry point:
 *   - Nothing throws across this boundary; every call returns a status code
 *     and fkt_last_error() gives a message for the calling thread.
 *   - Arrays are row-major. "host" pointers are read on the CPU during the
 *     call; "device" pointers are HIP device memory on the plan's device.
 *   - Device work is enqueued on the plan's stream and is asynchronous: the
 *     caller synchronises the stream before reading results.
 *   - The caller owns every array it passes; the plan copies what it keeps.
 *   - A plan's tree, lists and tables are fixed by fkt_plan; preconditioner
 *     state (fkt_precond_coarse, fkt_learn_*) is added by later calls. Calls
 *     on one plan must be serialised by the caller: the plan owns one set of
 *     work buffers, and a solve sets plan state (the instance flags of its
 *     masked operator applications) while it runs.
 */
#ifndef FKT_H
#define FKT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fkt_plan_s *fkt_plan_t; /* opaque, owned by the library */

typedef enum {
    FKT_OK = 0,
    FKT_EINVAL = 1,        /* invalid argument (message says which)            */
    FKT_ENOMEM = 2,        /* host or device allocation failed                 */
    FKT_EDEVICE = 3,       /* HIP runtime error, or no device for this plan    */
    FKT_EUNSUPPORTED = 4,  /* valid but not built: dimension/order/kind combo  */
    FKT_ENOTCONV = 5       /* iterative solve hit maxit before rtol            */
} fkt_status;

/* Isotropic kernels K(r), r = |r_i - r_j|; l = lengthscale, s2 = variance. */
typedef enum {
    FKT_GAUSSIAN = 0,    /* s2 exp(-r^2 / (2 l^2))                            */
    FKT_EXPONENTIAL = 1, /* s2 exp(-r / l)              (Matern nu = 1/2)      */
    FKT_MATERN32 = 2,    /* s2 (1 + a r) exp(-a r),      a = sqrt(3) / l       */
    FKT_MATERN52 = 3,    /* s2 (1 + a r + a^2 r^2 / 3) exp(-a r), a = sqrt(5)/l */
    FKT_RATQUAD = 4,     /* s2 (1 + r^2 / (2 alpha l^2))^(-alpha)             */
    FKT_CAUCHY = 5,      /* s2 / (1 + r^2 / l^2)                              */
    FKT_LAPLACE = 6      /* s2 / r, with K(0) taken as 0 (no self term)       */
} fkt_kernel_kind;

typedef struct {
    fkt_kernel_kind kind;
    double lengthscale; /* l > 0 (ignored by FKT_LAPLACE)                     */
    double alpha;       /* rational-quadratic shape, > 0 (FKT_RATQUAD only)   */
    double variance;    /* s2 > 0                                             */
} fkt_kernel;

typedef enum {
    FKT_F64 = 0, /* x, y are double; all device arithmetic in FP64            */
    FKT_F32 = 1  /* x, y are float; near and far field in FP32, tree geometry,
                    node centres and expansion coefficients kept in FP64      */
} fkt_precision;

typedef struct {
    double theta;       /* distance criterion of eq. (accparam), 0 < theta < 1 */
    fkt_precision prec;
    int max_depth;      /* tree depth cap (guards duplicate points), 1..60    */
    int device;         /* HIP device ordinal; -1 builds a host-only plan
                           (tree, lists, tables; fkt_mvm then returns
                           FKT_EDEVICE)                                        */
    void *stream;       /* hipStream_t for all device work; NULL = null stream */
    int profile;        /* nonzero: fkt_mvm records HIP events between its
                           stages (see fkt_plan_stage_times)                   */
    int overlap;        /* nonzero (default): the near field runs on a second,
                           plan-owned stream (default priority) concurrently
                           with the far field, joined back into `stream`
                           before the scatter; 0: every stage in order on
                           `stream`                                            */
    int mrhs;           /* FP32 plans: fkt_mvm with nrhs a multiple of 32 runs
                           each group of 32 columns on the matrix cores. The
                           near field: 1 FP32 MFMA, 2 bf16 MFMA (kernel
                           values and weights rounded to bf16, FP32
                           accumulation). The moments of the 32 columns:
                           FP32 MFMA. The far-field evaluation (basis times
                           moments): bf16 MFMA with both operands split into
                           high and low bf16 parts and three products per
                           tile (about 16 mantissa bits), for either value.
                           0 (default): every column on its own, FP32.      */
    int far_mode;       /* order of the far-field evaluation (multipole to
                           target): 1 block-major (one wave per 64-target
                           block, its pairs packed into jobs whose node
                           moments are staged in LDS, one sum per target);
                           2 node-major (one wave per far node and up to 64
                           of its targets, moments read as wave-uniform
                           scalar operands, one atomic add per pair; plan
                           memory 4 bytes per far pair; above rank 120
                           the moments are staged in LDS); 0 (default)
                           picks node-major except for FP32 plans of
                           expansion rank above 1000.                       */
    int compress;       /* 1: compress the radial expansion (Appendix A.4,
                           eq. f_g) for a kernel with K' = q K, q a Laurent
                           polynomial (FKT_EXPONENTIAL, FKT_LAPLACE,
                           FKT_GAUSSIAN; others: FKT_EINVAL). The exact ranks
                           R_k are found at plan time; where compressed
                           kernels are built (1/r and the exponential in
                           d = 3: R_k = 1 and 2) the far field evaluates
                           sum_k |H_k| R_k terms per node instead of
                           C(p+d, d) (fkt_plan_stats.radial_rank), on the
                           node-major far field (far_mode 1 and mrhs are
                           FKT_EUNSUPPORTED). Elsewhere the plan is the
                           uncompressed one. The result is the same
                           truncated expansion up to rounding. 0: off.      */
    int fuse;           /* 1: the near and far field of each MVM pass run as
                           one persistent launch over a global work queue
                           (far jobs and near units interleaved, one atomic
                           per item; built for d = 3, needs the node-major
                           far field and no compression, else
                           FKT_EUNSUPPORTED). 0 (default): separate launches
                           on two streams.                                  */
} fkt_options;

/* Test hook: with the environment variable FKT_FAIL_ALLOC_AT=k set, the k-th
 * device allocation while a plan is built reports out of memory (fkt_plan
 * then returns FKT_ENOMEM and frees what it had allocated). Unset: no
 * effect. */

/* Defaults: theta 0.5, FKT_F64, max_depth 48, device 0, stream NULL, profile 0,
 * overlap 1, mrhs 0, far_mode 0, compress 0, fuse 0. */
void fkt_default_options(fkt_options *opt);

/*
 * fkt_plan -- build the tree, the near/far partition and the coefficient
 * tables, and upload them to the device (paper Sec. 3.1-3.2, Algorithm 1
 * first line; coefficient tables of Appendix A.2).
 *   points    host, n x d FP64, row-major. Copied; not retained. (Host,
 *             not device: the tree and the near/far lists are built on the
 *             CPU, so a device array would be copied back first; the Python
 *             binding does that copy for device tensors.)
 *   n         number of points, >= 1 (sources and targets are the same set).
 *   d         dimension, 3 <= d <= 5 (d = 2 needs the alpha = 0 Gegenbauer
 *             limit and is FKT_EUNSUPPORTED).
 *   k         kernel and its parameters.
 *   leaf_size maximum points per leaf, >= 1 (a node with more is split).
 *   order     truncation order p of eq. (finaltrunc): radial powers j <= p,
 *             harmonic degrees k <= p; expansion rank C(p+d, d).
 *             Built: 0 <= p <= 8 for d = 3, 4 and 5; other orders return
 *             FKT_EUNSUPPORTED with a message naming the built range.
 *   opt       NULL for defaults.
 *   out       receives the plan on FKT_OK, NULL otherwise.
 * Errors: FKT_EINVAL (bad n, d, leaf_size, order, theta, kernel parameters,
 * non-finite coordinates), FKT_EUNSUPPORTED, FKT_ENOMEM, FKT_EDEVICE.
 */
fkt_status fkt_plan(const double *points, int64_t n, int d, fkt_kernel k, int leaf_size, int order,
                    const fkt_options *opt, fkt_plan_t *out);

/*
 * fkt_mvm -- y = K~ x with K~ the FKT approximation of the kernel matrix
 * (Algorithm 1): near field exact, far field through the truncated
 * expansion about each far node's centre.
 *   x, y      device, n x nrhs row-major, element type double (FKT_F64) or
 *             float (FKT_F32). Must not overlap. y is fully overwritten.
 *   nrhs      number of right-hand sides, 1 <= nrhs <= 64. Plans with the
 *             node-major far field run the columns in passes of four (three
 *             padded to four; one or two column by column), sharing every
 *             kernel value, harmonic and radial function within a pass;
 *             mrhs plans run groups of 32 columns on the matrix cores.
 * Enqueued on the plan's stream; returns before the result is ready.
 * Allocates nothing: the plan's work buffers are allocated by fkt_plan.
 * Errors: FKT_EINVAL (NULL/overlapping pointers, nrhs), FKT_EDEVICE (host-only
 * plan, HIP failure). On error y is unspecified.
 */
fkt_status fkt_mvm(fkt_plan_t p, const void *x, void *y, int nrhs);

/*
 * fkt_cg_solve -- solve (K~ + sigma2 I) x = b by conjugate gradients, each
 * iteration one fkt_mvm. Used for the Gaussian-process posterior mean
 * (paper eq. gp_posterior), whose inference runs through MVMs only.
 *   sigma2    noise variance, >= 0.
 *   b         device, n x nrhs (plan precision element type).
 *   x         device, n x nrhs; on entry the initial guess, on exit the
 *             solution (the last iterate if not converged).
 *   rtol      stop when ||b - A x||_2 <= rtol ||b||_2 for every system.
 *             A system is one column of one instance: for a batched plan
 *             (fkt_plan_batch) the operator is block diagonal, so every
 *             instance and column runs its own CG recurrences (its own step
 *             lengths and stopping test, norms over the instance's rows);
 *             a system that has converged is frozen while the others go on,
 *             and the operator work of an instance whose systems have all
 *             converged is skipped in the following iterations.
 *   maxit     iteration cap, >= 1.
 *   precond   0 none, 1 block-Jacobi (per-leaf dense Cholesky of
 *             K_ll + sigma2 I), 2 the learned per-leaf spectral filter
 *             (fkt_learn_*, current weights; block-Jacobi while its output
 *             layer is zero: initially, or after the judge rejected a filter).
 *             With a trained filter, block-Jacobi is also the fallback: once the residual
 *             exceeds 10 times its best so far, or sets no new best for 250
 *             iterations, CG restarts from the best iterate with block-Jacobi
 *             (one extra fkt_mvm; iterations keep counting; the switch is
 *             reported in fkt_plan_stats.cg_fallback_iter).
 *   iters     host, receives the iteration count (of the slowest system;
 *             may be NULL).
 *   relres    host, receives max over systems of the final relative
 *             residual (may be NULL).
 * Synchronises the plan's stream (it reads residual norms on the host).
 * Errors: as fkt_mvm, FKT_EUNSUPPORTED for an unknown precond, FKT_ENOTCONV
 * when maxit is reached (x holds the last iterate).
 */
fkt_status fkt_cg_solve(fkt_plan_t p, double sigma2, const void *b, void *x, int nrhs, double rtol, int maxit,
                        int precond, int *iters, double *relres);

/*
 * fkt_cg_solve64 -- fkt_cg_solve with b and x in FP64 (device, n x nrhs
 * doubles) whatever the plan's precision. On an FP32 plan this is the
 * mixed-precision solve: the MVMs run in FP32, while b, the CG vectors, the
 * preconditioners and the returned solution stay FP64, so the solution is
 * not rounded to FP32 on the way out. On an FP64 plan it is fkt_cg_solve.
 * Arguments, errors and synchronisation as fkt_cg_solve.
 */
fkt_status fkt_cg_solve64(fkt_plan_t p, double sigma2, const double *b, double *x, int nrhs, double rtol, int maxit,
                          int precond, int *iters, double *relres);

/*
 * fkt_cg_solve_refined -- solve (K~ + sigma2 I) x = b to rtol against the
 * FP64 operator while the CG iterations run on the FP32 one (mixed-precision
 * CG with residual replacement), for the posterior-mean system of the
 * paper's Gaussian-process regression (eq. gp_posterior). CG on an FP32
 * operator alone stops at that operator's own error (about 1e-5 relative).
 * Here CG runs on lo (fkt_cg_solve64: FP32 MVMs, FP64 vectors), and each time
 * its worst residual has dropped tenfold since the last replacement, or has
 * reached rtol, the residual is replaced by r = b - (K~64 + sigma2 I) x from
 * the FP64 plan; the search direction is kept. It stops only when every
 * system's replaced (true FP64) residual is <= rtol.
 *   p       FP64 plan; its stream runs the replacement MVMs.
 *   lo      FP32 plan over the same points (same instances, kernel, order
 *           and device; only n, d, device and instance offsets are checked).
 *           The preconditioner (precond as fkt_cg_solve) is lo's.
 *   b, x    device, n x nrhs doubles; x on entry the initial guess, on exit
 *           the solution (the last iterate if not converged).
 *   maxit   cap on the CG iterations, >= 1.
 *   iters   host, CG iterations (one FP32 fkt_mvm each; may be NULL).
 *   outer   host, residual replacements (one FP64 fkt_mvm each; may be NULL).
 *   relres  host, max over systems of the final relative residual, the FP64
 *           one on success (may be NULL).
 * Errors: as fkt_cg_solve; FKT_EINVAL if the plans' precisions or shapes do
 * not pair up; FKT_ENOTCONV when maxit is reached first.
 */
fkt_status fkt_cg_solve_refined(fkt_plan_t p, fkt_plan_t lo, double sigma2, const double *b, double *x, int nrhs,
                                double rtol, int maxit, int precond, int *iters, int *outer, double *relres);

/*
 * fkt_precond_coarse -- two-level preconditioning for the solves of this plan
 * at noise variance sigma2 (project addition: the paper solves its
 * Gaussian-process systems through MVMs, Sec. 5.3 and eq. gp_posterior, and
 * adds no preconditioner). Per-leaf preconditioners cannot reach the smooth
 * global modes that make long-length-scale kernel systems ill-conditioned,
 * so a Nystrom coarse space is added: with the k landmark points J,
 *     L = K(X, X_J) W,   W = chol(K(X_J, X_J) + sigma2 I)^-T,   K ~ L L^T,
 * and the Woodbury identity joins it to the per-leaf part of the residual
 * leaf blocks R_l = K_ll + sigma2 I - L_l L_l^T = V_l^T diag(lam_l) V_l:
 *     P = (L L^T + D)^-1,   D^-1 = blockdiag(V_l^T diag(h_l) V_l),
 * with h = 1 / lam for precond 1 (block-Jacobi of the residual blocks) and
 * h = exp(o) / lam, the learned filter, for precond 2 (whose features then
 * come from the residual spectra; fkt_learn_* train it through P). precond
 * 0 is unaffected. Afterwards every fkt_cg_solve / fkt_cg_solve64 /
 * fkt_cg_solve_noalloc / fkt_learn_* call on this plan with this sigma2 uses
 * the two-level form; a call with another sigma2 drops it (one-level again).
 *   landmarks  host, k distinct indices into the caller's point order (the
 *              caller draws them; uniform without replacement is the
 *              intended use).
 *   k          number of landmarks, 1..4096; 0 returns to one-level.
 * Builds K(X, X_J) and the factor on the device (FP64), the residual leaf
 * blocks' eigendecompositions on the host, G = V L and the k x k matrices
 * C = I + G^T diag(h) G (inverted on the host) for block-Jacobi; the learned
 * filter's C is rebuilt whenever its weights are used. Device memory: about
 * 8 n k (24 n k while building) + 8 (66 + m) k^2 bytes (m up to 64 row
 * chunks). Synchronises the plan's stream.
 * Errors: FKT_EINVAL (bad sigma2, k or landmarks; a landmark block or a
 * residual leaf block that is not positive definite), FKT_EUNSUPPORTED
 * (leaves over 2048 points), FKT_ENOMEM, FKT_EDEVICE.
 */
fkt_status fkt_precond_coarse(fkt_plan_t p, double sigma2, const int64_t *landmarks, int k);

/*
 * fkt_cg_solve_noalloc -- fkt_cg_solve for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same solve, arguments, results and errors, with
 * the CG work vectors (about 8 n nrhs doubles plus reduction partials) in a
 * fixed scratch array of 64 MiB that the library holds on each GPU it runs
 * on until the process ends. It calls no hipMalloc, hipFree or other
 * allocating routine.
 *   Limits: n * nrhs up to about 1.04e6 on an FP64 plan (0.93e6 with
 *   precond 2) and 1.19e6 on an FP32 plan (1.04e6 with precond 2); larger
 *   problems return FKT_EINVAL naming the bytes needed.
 *   precond 1 needs the block-Jacobi factors of this sigma2, and precond 2
 *   also the learned filter's state for it, built beforehand by
 *   fkt_cg_solve (or fkt_learn_params) on this plan, or else the two-level
 *   state of fkt_precond_coarse for this sigma2; otherwise FKT_EINVAL.
 *   Every call on one GPU shares that GPU's scratch array (which keeps the
 *   last call's contents; the solve initialises every entry it reads), so
 *   calls that overlap in time on one GPU -- from several host threads or on
 *   streams that are not ordered -- race and must be serialised by the
 *   caller.
 */
fkt_status fkt_cg_solve_noalloc(fkt_plan_t p, double sigma2, const void *b, void *x, int nrhs, double rtol, int maxit,
                                int precond, int *iters, double *relres);

/* Release the plan and its device memory (NULL is a no-op). Waits for the
 * plan's stream first. */
void fkt_destroy(fkt_plan_t p);

/* Message for the last failing call on this thread ("" if none). The
 * pointer stays valid until the next call on the same thread. */
const char *fkt_last_error(void);

/* Plan statistics (host-side, available for host-only plans too). */
typedef struct {
    int64_t n, nnodes, nleaves, depth;
    int64_t rank;             /* expansion terms per node, C(p+d, d)           */
    int64_t nblocks;          /* 64-target blocks                              */
    int64_t far_nodes;        /* nodes with a non-empty far set                */
    int64_t near_entries;     /* (target block, source leaf) list entries      */
    int64_t far_entries;      /* (target block, far node) list entries         */
    int64_t near_pairs;       /* sum_l |N_l| |l|: kernel evaluations           */
    int64_t near_lane_pairs;  /* evaluations incl. masked-off lanes            */
    int64_t far_pairs;        /* sum_b |F_b|: (target, node) expansions        */
    int64_t far_lane_pairs;   /* expansions incl. masked-off lanes             */
    int64_t s2m_terms;        /* sum_b |b| over nodes with far sets            */
    double plan_seconds;      /* host wall time of fkt_plan                    */
    int64_t cg_fallback_iter; /* iteration at which the last fkt_cg_solve fell
                                 back from the learned filter to block-Jacobi,
                                 -1 if it did not (or no solve has run)        */
    int64_t radial_rank;      /* far-field terms per node as evaluated: rank,
                                 or sum_k |H_k| R_k with radial compression    */
} fkt_plan_stats;

fkt_status fkt_plan_info(fkt_plan_t p, fkt_plan_stats *s);

/*
 * fkt_radial_compression -- the exact compression of the radial expansion
 * (Appendix A.4, eq. f_g; Table "ranks") for kernel k in d dimensions at
 * order `order` (host only; no plan or device needed).
 *   ranks  host, order + 1 ints (may be NULL): R_k, the rank over the
 *          rationals of degree k's radial functions (Laurent coefficients
 *          carried exactly modulo a 61-bit prime, as the paper's rational
 *          rank-revealing factorisation does with exact fractions).
 *   keep   host (may be NULL): radial rows kept per degree by the library's
 *          compressed kernels for this kernel and d (first min(keep, nj)
 *          rows), 0 when none are built or the rows do not qualify.
 *   coef   host (may be NULL; written only when *keep > 0),
 *          (order+1) * mj * mj doubles, mj = order / 2 + 1:
 *          coef[(k * mj + jj) * mj + i] = c_{jj,i} with
 *          L_{k+2jj}(u) = sum_i c_{jj,i} L_{k+2i}(u), i < min(keep, nj),
 *          jj < nj = (order - k) / 2 + 1, where the radial functions of
 *          Theorem 3.1 read F_kj(r) r^j = K(r) u^j L_j(u) in the scaled
 *          distance u = r / l (u = r for FKT_LAPLACE).
 * Errors: FKT_EINVAL for a kernel without K' = q K (q Laurent), d < 1, or
 * order outside [0, 30].
 */
fkt_status fkt_radial_compression(const fkt_kernel *k, int d, int order, int *ranks, int *keep, double *coef);

/* perm[i] = original index of the point at tree position i (host, n int64). */
fkt_status fkt_plan_perm(fkt_plan_t p, int64_t *perm);

/* Per target (original order, host arrays of n int64, any may be NULL):
 * far nodes, far source points, near leaves, near source points. */
fkt_status fkt_plan_target_counts(fkt_plan_t p, int64_t *far_nodes, int64_t *far_points, int64_t *near_leaves,
                                  int64_t *near_points);

/*
 * The plan's partition per target (Sec. 3.2): the far nodes F (eq. accparam)
 * and near leaves N of each target, as host CSR arrays over the targets in
 * the caller's order. Node ids are the tree's preorder numbers (for a
 * batched plan the instance trees are numbered one after another, in
 * instance order), ascending within each target.
 *   far_off, near_off   n + 1 int64 each (may be NULL).
 *   far_node, near_leaf int64 arrays of *nfar_total and *nnear_total entries;
 *                       pass NULL to query the totals first.
 *   nfar_total, nnear_total  receive the totals (may be NULL).
 * Errors: FKT_EINVAL (NULL plan). */
fkt_status fkt_plan_lists(fkt_plan_t p, int64_t *far_off, int64_t *far_node, int64_t *near_off, int64_t *near_leaf,
                          int64_t *nfar_total, int64_t *nnear_total);

/*
 * Device time of fkt_mvm's stages, summed over the calls made since the plan
 * was built with opt.profile != 0 (or since the last reset): ms[0] gather into
 * tree order, ms[1] source-to-multipole moments (incl. partial sums), ms[2]
 * multipole-to-target far field, ms[3] near field, ms[4] the whole column pass
 * (gather to scatter). Times come from HIP events recorded on the stream each
 * stage runs on; with opt.overlap the near field shares the device with the
 * far field, so ms[3] then includes that sharing and ms[4] < the sum of the
 * stages. Synchronises those events. calls (may be NULL) receives the number
 * of column passes timed. reset != 0 clears the record.
 * Errors: FKT_EINVAL (NULL, plan built without profile), FKT_EDEVICE.
 */
fkt_status fkt_plan_stage_times(fkt_plan_t p, double *ms, int64_t *calls, int reset);

/*
 * fkt_plan_batch -- one plan over ninst independent point sets (a forest):
 * instance i is rows offsets[i] .. offsets[i+1]-1 of points (host, FP64,
 * offsets host int64 [ninst + 1], offsets[0] = 0, non-decreasing; empty
 * instances allowed). Each instance gets its own tree (Sec. 3.1) and its
 * own near/far sets; nothing interacts across instances, so fkt_mvm on the
 * concatenated x computes every instance's K~_i x_i in the same launches
 * (one launch per stage over all instances' work). Arguments, options and
 * errors otherwise as fkt_plan.
 */
fkt_status fkt_plan_batch(const double *points, const int64_t *offsets, int ninst, int d, fkt_kernel k, int leaf_size,
                          int order, const fkt_options *opt, fkt_plan_t *out);

/*
 * A whole fkt_mvm(p, x, y, nrhs) captured once into a HIP graph (the stages
 * as fkt_mvm enqueues them, the near field on its own branch with
 * opt.overlap; x and y are baked in) and replayed with
 * fkt_graph_launch on the plan's stream. The plan must outlive the graph;
 * replays of graphs of one plan must not overlap (they share its work
 * buffers). Errors: FKT_EINVAL, FKT_EDEVICE, FKT_ENOMEM.
 */
typedef struct fkt_graph_s *fkt_graph_t;
fkt_status fkt_graph_create(fkt_plan_t p, const void *x, void *y, int nrhs, fkt_graph_t *out);
fkt_status fkt_graph_launch(fkt_graph_t g);
void fkt_graph_destroy(fkt_graph_t g);

/*
 * Leaf-size autotuner: builds a plan (fkt_plan_batch when offsets is not
 * NULL, else fkt_plan over n points) for each of the ncand candidate leaf
 * sizes, times reps MVMs of nrhs zero columns after one untimed pass (HIP
 * events on the plan's stream) and returns the fastest in *best; ms (host,
 * ncand doubles, may be NULL) receives each candidate's time per MVM.
 * opt->device must be >= 0. Time alone decides: theta and p fix the
 * expansion, and a larger leaf only moves interactions of nodes below the
 * leaf level from the far to the exact near field.
 */
fkt_status fkt_autotune_leaf(const double *points, const int64_t *offsets, int ninst, int64_t n, int d, fkt_kernel k,
                             int order, const fkt_options *opt, const int *candidates, int ncand, int nrhs, int reps,
                             int *best, double *ms);

/*
 * Autotuner over leaf sizes and far-field schedules: as fkt_autotune_leaf
 * for every pair (leaves[i], far_modes[m]) (far_mode values of
 * fkt_options: 0 automatic, 1 block-major, 2 node-major; the two schedules
 * tile the far field differently: 64-target blocks over LDS-staged node
 * moments, or one far node over 64 targets). *best_leaf and *best_mode
 * (may be NULL) receive the fastest pair; ms (host, nleaf * nmodes doubles,
 * row i = leaf i, may be NULL) each pair's time per MVM. Errors: as
 * fkt_autotune_leaf, FKT_EINVAL for a far_mode outside 0..2.
 */
fkt_status fkt_autotune(const double *points, const int64_t *offsets, int ninst, int64_t n, int d, fkt_kernel k,
                        int order, const fkt_options *opt, const int *leaves, int nleaf, const int *far_modes,
                        int nmodes, int nrhs, int reps, int *best_leaf, int *best_mode, double *ms);

/*
 * Learned per-leaf preconditioner (not part of the paper's method; used by
 * fkt_cg_solve with precond = 2). For each leaf l, the near-field diagonal
 * block A_l = K(X_l, X_l) + sigma2 I = V_l^T diag(lam_l) V_l is
 * eigendecomposed on the host, and the preconditioner is
 *     M = blockdiag(V_l^T diag(h_l) V_l),   h_{l,i} = exp(o_{l,i}) / lam_{l,i},
 * with o_{l,i} the output of one MLP, FP32, 4 -> 256 (tanh) -> 256 (tanh) -> 1,
 * applied to the features of eigenvalue i of leaf l:
 *     [log(lam_i / sigma2) / 8, log(lam_max / sigma2) / 8, m_l / leaf_size, (i + 1/2) / m_l]
 * (ascending eigenvalues, m_l points in the leaf). M is symmetric positive
 * definite for any weights; o = 0 (the initial last layer is zero) makes it
 * block-Jacobi. Training minimises L = (1/B) sum_b min_a |a A M v_b - v_b|^2 /
 * |v_b|^2 (invariant to the scale of M, as PCG is) for Gaussian v_b with A =
 * the plan's MVM + sigma2 I, its gradient taking A as symmetric. Needs leaves of at most 2048 points and sigma2 > 0; the first
 * call for a sigma2 builds the spectra (host, O(leaf^3) per leaf).
 *
 * Parameters (FP32, fkt_learn_nparams() of them) in the order W1 [4][256],
 * b1 [256], W2 [256][256] (hidden = tanh(h1 W2 + b2)), b2 [256], w3 [256], b3.
 */
int64_t fkt_learn_nparams(void);

/* params: host buffer of fkt_learn_nparams() floats; set = 0 copies the
 * current weights out, set != 0 replaces them. Errors: FKT_EINVAL,
 * FKT_EUNSUPPORTED (leaves > 2048), FKT_EDEVICE, FKT_ENOMEM. */
fkt_status fkt_learn_params(fkt_plan_t p, double sigma2, float *params, int set);

/* Loss L and its gradient for the given batch. v: device, n x batch FP64
 * row-major, caller's point order (1 <= batch <= 64). loss: host; grad: host
 * buffer of fkt_learn_nparams() floats or NULL. Does not change the weights.
 * Synchronises the plan's stream. */
fkt_status fkt_learn_loss_grad(fkt_plan_t p, double sigma2, const double *v, int batch, double *loss, float *grad);

/* `steps` Adam steps (lr, beta1 0.9, beta2 0.999, eps 1e-8), each on a fresh
 * batch of `batch` Gaussian vectors drawn on the device (SplitMix64 counter
 * hash + Box-Muller, keyed by seed and step). loss_first / loss_last (host,
 * may be NULL) receive the loss of the first and of the last step's batch
 * (before that step's update). With judge_iters > 0, block-Jacobi judges the
 * result: judge_iters CG iterations on one Gaussian right-hand side with each
 * preconditioner, and if the learned filter ends with the larger residual its
 * last layer is zeroed (the filter is then block-Jacobi exactly); accepted
 * (host, may be NULL) receives 1 if the trained weights were kept, else 0.
 * Synchronises the plan's stream. */
fkt_status fkt_learn_train(fkt_plan_t p, double sigma2, int steps, int batch, double lr, uint64_t seed,
                           double *loss_first, double *loss_last, int judge_iters, int *accepted);

/*
 * Training of the learned filter by the condition number of the
 * preconditioned operator (an objective aligned with CG's convergence;
 * fkt_learn_train's one-step residual objective drives the filter toward
 * block-Jacobi or past it). Each of `steps` Adam steps (lr, beta1 0.9, beta2
 * 0.999) runs `lanczos` PCG iterations from zero with the current filter
 * (one- or two-level, as fkt_cg_solve with precond 2 would) on a fresh
 * Gaussian right-hand side (SplitMix64 + Box-Muller, keyed by seed and
 * step); PCG's step lengths are the Lanczos tridiagonal of P A and its
 * preconditioned residuals the Lanczos vectors, so the extreme Ritz pairs
 * (lambda, u), u^T P^-1 u = 1, follow at no further operator cost. The
 * objective is log kappa = log lambda_max - log lambda_min; P^-1 is affine
 * in the block part D = blockdiag(V_l^T diag(1/h_l) V_l), so its gradient in
 * the network outputs is (V u_max)_i^2 / h_i - (V u_min)_i^2 / h_i, then back
 * through the MLP. cond_first / cond_last (host, may be NULL) receive the
 * Ritz estimate of kappa at the first and the last step (before its
 * update). judge_iters and accepted as fkt_learn_train. lanczos in
 * [2, 1000]. Errors: as fkt_learn_train; FKT_EDEVICE on a PCG breakdown.
 * Synchronises the plan's stream.
 */
fkt_status fkt_learn_train_cond(fkt_plan_t p, double sigma2, int steps, int lanczos, double lr, uint64_t seed,
                                double *cond_first, double *cond_last, int judge_iters, int *accepted);

/* The condition-number objective of fkt_learn_train_cond for one right-hand
 * side b (device, n FP64, caller's order; not modified): cond (host)
 * receives the Ritz estimate of kappa, grad (host, fkt_learn_nparams()
 * floats, may be NULL) the gradient of log kappa. Does not change the
 * weights. */
fkt_status fkt_learn_cond_grad(fkt_plan_t p, double sigma2, const double *b, int lanczos, double *cond, float *grad);

#ifdef __cplusplus
}
#endif

#endif /* FKT_H */
