/*
 * kchol.h -- C ABI of the MI355X (gfx950) sparse-Cholesky library.
 *
 * Method: Schaefer, Sullivan, Owhadi, "Compression, inversion, and approximate
 * PCA of dense kernel matrices at near-linear computational complexity"
 * (arXiv:1706.02205).  Given points x_1..x_N, a Matern kernel and rho, the
 * library computes
 *   1. the maximin ordering and the sparsity pattern S_rho      (Section 2.3)
 *   2. the covariance entries Theta_ij on S_rho                  (Section 4.4)
 *   3. the zero fill-in incomplete Cholesky factor ICHOL(0)      (Section 2.2)
 *   4. x = Theta^{-1} b ~ P^T L^{-T} L^{-1} P b                  (Section 1, task (2))
 * Step 1 runs on the host (kc_analyze); steps 2-4 run as HIP kernels.
 *
 * Conventions
 *  - Every pointer argument is owned by the caller; the library never frees
 *    caller memory.  "_dev" pointers are device memory of the current HIP
 *    device, all others host memory.
 *  - Points are row-major N x d float64 in the caller's original order.
 *    Right-hand sides and solutions are row-major N x nrhs float64 (the nrhs
 *    values of one point are contiguous), also in the original order.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *    device work is enqueued asynchronously on it unless stated otherwise.
 *  - Calls return kc_status; KC_OK is 0.  On failure kc_last_error() gives a
 *    thread-local message.  No call aborts the process.
 *  - A nonpositive pivot is not an error: it is counted (Section 4.4 zeroes the
 *    column; KC_PIVOT_SHIFT raises it instead).
 *  - Distinct handles may be used from distinct host threads.
 */
#ifndef KCHOL_H
#define KCHOL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    KC_OK = 0,
    KC_EINVAL = 1,     /* bad argument: n<1, d<1, rho<=0 or non-finite, non-finite coordinate, nrhs<1, unsupported nu */
    KC_ENOMEM = 2,     /* host allocation failed */
    KC_EWORKSPACE = 3, /* device workspace or scratch smaller than required */
    KC_EHIP = 4,       /* a HIP runtime call failed (detail in kc_last_error) */
    KC_ESTATE = 5,     /* call out of order, e.g. solve before factorize */
    KC_ERANGE = 6      /* problem too large for the index types (nnz(S) >= 2^32) */
} kc_status;

/* Pattern rule.  MAX is the paper's S_rho = {(i,j): dist(x_i,x_j) <= rho*max(l_i,l_j)}
 * (Section 2.3).  MIN uses rho*min(l_i,l_j), the pattern of Section 6.2. */
typedef enum { KC_RULE_MAX = 0, KC_RULE_MIN = 1 } kc_rule;

/* Arithmetic of the factorization.  FP64: everything in float64.  MIXED:
 * off-diagonal entries of Theta, their Schur updates and the stored L in
 * float32; diagonal accumulation, square roots and divisions in float64. */
typedef enum { KC_FP64 = 0, KC_MIXED = 1 } kc_prec;

/* Nonpositive pivots.  ZERO (Section 4.4): a pivot p <= 0 zeroes the column of L.
 * SHIFT: a pivot p <= tau*Theta_jj is replaced by tau*Theta_jj. */
typedef enum { KC_PIVOT_ZERO = 0, KC_PIVOT_SHIFT = 1 } kc_pivot;

/* Order in which the factorization launches the work units of one DAG level
 * (the columns of a level are independent, so results are the same in both).
 * SPATIAL: the point cloud's k-d tree order, each XCD taking one contiguous
 * slice of the level (L2 locality).  LONGEST: the unit with the longest walk
 * first, so that the last, partly filled round of a level holds short units;
 * this pays for a single large problem, whose units of one level lie far apart
 * anyway; a batch of small problems does better with SPATIAL. */
typedef enum { KC_ORDER_SPATIAL = 0, KC_ORDER_LONGEST = 1 } kc_unit_order;

/* Matern covariance G_{l,nu}(x,y) of Section 4.4 with unit variance; nu must be
 * 0.5, 1.5 or 2.5 (closed forms), lengthscale > 0. */
typedef struct {
    double nu;
    double lengthscale;
} kc_kernel;

typedef struct kc_plan kc_plan;
typedef struct kc_factor kc_factor;
typedef struct kc_graph kc_graph;

typedef struct {
    int64_t n;
    int32_t d;
    int32_t rule;
    double rho;
    int64_t nnz;          /* entries of S in the lower triangle, diagonal included */
    int64_t max_col;      /* longest column of S */
    int64_t max_row;      /* longest row of S */
    int32_t nlevels;      /* depth of the elimination DAG (forward levels) */
    int32_t nrlevels;     /* depth of the reverse DAG (backward solve) */
    int64_t nunits;       /* 64-entry column chunks scheduled by the factorization */
    double t_order_s;     /* host time of the maximin ordering */
    double t_pattern_s;   /* host time of the pattern (CSC + CSR) */
    double t_schedule_s;  /* host time of levels and work units */
    int32_t ninst;        /* independent problems in the plan (1 unless built by kc_analyze_batched) */
} kc_plan_info_t;

typedef struct {
    int64_t nonpositive;  /* columns zeroed by KC_PIVOT_ZERO */
    int64_t shifted;      /* pivots raised by KC_PIVOT_SHIFT */
    int64_t rank;         /* n - nonpositive */
    int64_t updates;      /* Schur updates applied (only if counting was requested, else -1) */
    int64_t exp_hard;     /* exponentials whose rounding could not be certified (expected 0) */
    int64_t nonfinite;    /* entries of L (diagonal included) that are inf or NaN, e.g. after a
                             KC_PIVOT_SHIFT pivot so small that a division overflows; 0 for a usable factor */
    int64_t match_errors; /* entries whose match masks disagreed with the pattern (expected 0; see
                             kc_factor_match_build) */
} kc_factor_stats_t;

const char *kc_status_string(kc_status s);
const char *kc_last_error(void);

/* ---------------------------------------------------------------- analysis */

/* Maximin ordering and pattern S (Section 2.3; the ordering and pattern of the
 * paper's SortSparse algorithm, computed with k-d tree range searches), plus the
 * level schedule of the elimination DAG.  Host only, synchronous.
 * x: N x d row-major float64.  nthreads <= 0 uses all hardware threads.
 * The first point is original index 0; ties in the maximin argmax go to the
 * lowest original index.  *out is library-owned until kc_plan_destroy. */
kc_status kc_analyze(const double *x, int64_t n, int32_t d, double rho, kc_rule rule, int32_t nthreads,
                     kc_plan **out);
/* A batch of independent problems as one plan: instance i is the next counts[i]
 * rows of x (N_total x d).  Each instance is analysed on its own (the same
 * ordering and pattern as kc_analyze on its points, positions shifted by the
 * points before it); their DAG levels are merged so that one launch per level
 * factors every instance at that depth.  Instances run on separate host threads. */
kc_status kc_analyze_batched(const double *x, const int64_t *counts, int32_t ninst, int32_t d, double rho,
                             kc_rule rule, int32_t nthreads, kc_plan **out);
/* Supernodal ordering and pattern (the supernodal construction of the paper's
 * stability analysis, Section 5): after the maximin ordering and the max-rule
 * pattern S_rho, points are aggregated greedily in maximin order -- an
 * unassigned point k starts a supernode and claims every later unassigned point
 * a with l_a >= l_k/2 within 0.5*rho*l_k -- supernodes are ordered by their
 * first point with members consecutive, and the pattern becomes the block
 * closure: every member pair of supernodes with an S_rho pair between them.
 * Its ICHOL(0) is the supernodal incomplete Cholesky factorization (dense
 * blocks).  kc_plan_export reports the new ordering and pattern. */
kc_status kc_analyze_supernodal(const double *x, int64_t n, int32_t d, double rho, int32_t nthreads,
                                kc_plan **out);
/* Supernode boundaries of a supernodal plan in positions (nsuper + 1 entries,
 * snode_ptr may be NULL to query nsuper); nsuper = 0 for other plans. */
kc_status kc_plan_supernodes(const kc_plan *plan, int64_t *snode_ptr, int64_t *nsuper);
kc_status kc_plan_info(const kc_plan *plan, kc_plan_info_t *info);
/* Copies the ordering and pattern into caller buffers (any may be NULL):
 * perm[N] (maximin position -> original index), l[N], colptr[N+1],
 * rowidx[nnz] (CSC of the lower triangle, rows ascending, diagonal first). */
kc_status kc_plan_export(const kc_plan *plan, int32_t *perm, double *l, int64_t *colptr, int32_t *rowidx);
/* Level of each column in the elimination DAG (column j waits for every i<j with (j,i) in S). */
kc_status kc_plan_levels(const kc_plan *plan, int32_t *level);
/* The factorization reads the column indices of each row of S as 16-bit gaps
 * between consecutive indices; a gap of at least `delta_limit` is kept as a
 * full index in a per-row escape list.  The default, 65536, is the largest
 * gap 16 bits hold.  A smaller limit (1 <= delta_limit <= 65536) re-encodes
 * the plan with more escapes -- every entry for 1 -- and yields the same
 * factor; it exists to exercise the escape path.  Factors created afterwards
 * use the new encoding.  Returns the number of escapes in *nescapes (may be NULL).
 * KC_EINVAL for a limit out of range. */
kc_status kc_plan_set_delta_limit(kc_plan *plan, uint32_t delta_limit, int64_t *nescapes);
void kc_plan_destroy(kc_plan *plan);

/* ---------------------------------------------------------------- factor */

/* Device workspace needed by a factor of `plan` in precision `prec`. */
kc_status kc_factor_bytes(const kc_plan *plan, kc_prec prec, size_t *bytes);

/* Binds a factor to a caller-owned device workspace (>= kc_factor_bytes) and
 * uploads the pattern and schedule into it on `stream`.  The plan may be
 * destroyed afterwards; the workspace must outlive the factor. */
kc_status kc_factor_create(const kc_plan *plan, kc_prec prec, void *ws_dev, size_t ws_bytes, void *stream,
                           kc_factor **out);

/* Theta on S and ICHOL(0) (Sections 4.4 and 2.2), asynchronous on `stream`.
 * x_dev: N x d points in original order.  tau is used by KC_PIVOT_SHIFT only.
 * count_updates != 0 also counts the Schur updates (kc_factor_stats.updates).
 * The FP64 factor reproduces the paper's elimination order entry by entry:
 * each entry receives its updates in ascending eliminated index as one fused
 * multiply-add each, and Theta uses a correctly rounded exponential. */
kc_status kc_factorize(kc_factor *f, const double *x_dev, kc_kernel kernel, kc_pivot pivot, double tau,
                       int32_t count_updates, void *stream);

/* kc_factorize for a batch plan: every instance shares nu, instance i uses the
 * lengthscale ell_dev[i] (device array of ninst doubles, each finite and > 0). */
kc_status kc_factorize_batched(kc_factor *f, const double *x_dev, double nu, const double *ell_dev, kc_pivot pivot,
                               double tau, int32_t count_updates, void *stream);

/* Theta on S alone, in CSC order (nnz float64) -- the entries the
 * factorization starts from.  Requires kc_factor_create. */
kc_status kc_theta(kc_factor *f, const double *x_dev, kc_kernel kernel, double *theta_dev, void *stream);

/* Scratch needed by kc_solve for nrhs right-hand sides. */
kc_status kc_solve_bytes(const kc_factor *f, int32_t nrhs, size_t *bytes);

/* x = P^T L^{-T} L^{-1} P b (Section 1, task (2)).  b_dev, x_dev: N x nrhs
 * row-major float64 in original order (may not alias).  A zeroed column gives
 * solution component 0.  Requires a completed kc_factorize on the same factor.
 * Forward levels of fewer than 1024 rows and the backward sweep over short
 * columns follow the sequential substitution (bitwise); larger forward levels
 * sum each row across a wavefront, and when a column has more than 2048
 * off-diagonal entries, the columns up to the last such one are summed in
 * fixed pieces combined in a fixed order (deterministic, not bitwise the
 * sequential order). */
kc_status kc_solve(const kc_factor *f, const double *b_dev, double *x_dev, int32_t nrhs, void *scratch_dev,
                   size_t scratch_bytes, void *stream);

/* kc_solve for callers that cannot allocate device memory -- code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * same kernels and result as kc_solve (bitwise), but its scratch (the forward
 * sweep's intermediate vector and the backward sweep's partial sums,
 * kc_solve_bytes) lives in one fixed array of 96 MiB that the library holds on
 * each device it runs on until the process ends; no call allocates or frees
 * memory.  A solve needing more than 96 MiB of scratch (N * nrhs * 8 bytes
 * plus the partial sums; e.g. 10^6 points with 8 right-hand sides fits)
 * returns KC_EWORKSPACE before any work.  Every call on one device shares that
 * device's array: calls that overlap on one device (on different streams, or
 * from different threads) race and give wrong results; calls ordered on one
 * stream are safe.  Arguments as for kc_solve. */
kc_status kc_solve_noalloc(const kc_factor *f, const double *b_dev, double *x_dev, int32_t nrhs, void *stream);

/* kc_factorize followed by kc_solve (Section 2.2 and Section 1, task (2)) in one
 * call, with the forward sweep overlapped with the factorization: after the
 * launch covering factor levels [l0, l1) is enqueued on `stream`, a second
 * stream owned by the factor (created on first use, default priority; it waits
 * on an event recorded on `stream`) runs the forward sweep of those levels,
 * while `stream` goes on with the next levels; the backward sweep runs on
 * `stream` after both.  Results are bitwise those of kc_factorize (or
 * kc_factorize_batched) + kc_solve.  Arguments as for those calls (update
 * counting is not offered): for a batch plan pass ell_dev, one lengthscale per
 * instance (kernel.lengthscale is then ignored), else NULL.  All work is
 * ordered after earlier work on `stream`, and later work on `stream` is
 * ordered after it. */
kc_status kc_factorize_solve(kc_factor *f, const double *x_dev, kc_kernel kernel, const double *ell_dev,
                             kc_pivot pivot, double tau, const double *b_dev, double *x_out, int32_t nrhs,
                             void *scratch_dev, size_t scratch_bytes, void *stream);

/* Match masks: symbolic data that speeds up the factorization of this pattern.
 * The elimination of Section 2.2 updates entry (k,j) with every parent i < j
 * that row k and row j share, in ascending order.  Without masks each update
 * is found by merging the column indices of row k (read from HBM) with those of
 * row j.  With masks, two bit strings per entry record the shared parents
 * once: one bit per entry of row k before (k,j) and one per parent of j; the
 * factorization then reads one bit instead of a 16-bit index per entry it
 * walks, stops at the last shared parent, and skips value lines holding none.
 * L is bitwise the same either way (same updates, same order).
 *
 * kc_factor_match_bytes: device bytes the masks need -- an 8-byte word per
 * entry of S plus about (pos + np) / 64 8-byte words per entry, pos being the
 * entries of row k before (k,j) and np the parents of j (some 24 GB for 10^6
 * points at rho = 4).  Counting runs on the device, synchronously on `stream`,
 * once per factor.
 * kc_factor_match_build: builds the masks in the caller-owned buffer buf_dev
 * (>= kc_factor_match_bytes, 256-byte aligned), synchronously on `stream`;
 * later factorizations of this factor use them.  The buffer must stay valid
 * while they are attached; buf_dev = NULL detaches them (back to the index
 * merge).  KC_EWORKSPACE for a short or misaligned buffer, KC_ERANGE if a
 * row is too long to stage (more than about 10,000 entries). */
kc_status kc_factor_match_bytes(kc_factor *f, void *stream, size_t *bytes);
kc_status kc_factor_match_build(kc_factor *f, void *buf_dev, size_t bytes, void *stream);

/* Synchronises the factor's last stream and reports pivot statistics. */
kc_status kc_factor_stats(kc_factor *f, kc_factor_stats_t *stats);

/* Copies L to the host in CSC order of the plan (nnz float64; MIXED values are
 * widened).  Synchronous. */
kc_status kc_factor_export_L(const kc_factor *f, double *vals);

void kc_factor_destroy(kc_factor *f);

/* Schedule of the factorization.  Each DAG level runs as its own launch with
 * `wpb` wavefronts (1, 2 or 4) per workgroup, except that every run of
 * consecutive levels with at most `persist_max` work units (64 entries of a
 * column each) runs as ONE persistent launch: a cooperative grid, resident as a
 * whole, whose wavefronts stride over each level's units with a grid-wide
 * barrier between levels.  persist_max = 0 (the default) launches every level
 * separately; INT64_MAX runs the whole factorization in one persistent launch.
 * `order` is the order of the units within a level.  kc_factor_create picks
 * the defaults: wpb from the mean column length, persist_max 0, and LONGEST
 * for a single problem with a level larger than the device holds at once,
 * else SPATIAL (a batch keeps each problem's units together).  When no level
 * exceeds what the device holds at once, the two orders share one array (order
 * cannot change the speed then); asking for LONGEST on such a factor builds its
 * own array first (a device pass over the pattern and a host sort, synchronous
 * on the stream of the factor's last call).  Results are
 * bitwise identical for every schedule.  KC_EINVAL for wpb not in {1, 2, 4},
 * persist_max < 0, an unknown order, or staged rows that do not fit in LDS.
 * Any pointer of kc_factor_schedule may be NULL. */
kc_status kc_factor_set_schedule(kc_factor *f, int32_t wpb, int64_t persist_max, kc_unit_order order);
kc_status kc_factor_schedule(const kc_factor *f, int32_t *wpb, int64_t *persist_max, kc_unit_order *order);

/* Supernodal groups on the matrix cores (mixed-precision factors of supernodal
 * plans, kc_analyze_supernodal; the default for them).  The block-closed
 * pattern gives every member of a supernode the same row structure (Section 5,
 * the supernodal construction; its factorization is the supernodal incomplete
 * Cholesky of the appendix), so a group of up to 16 consecutive members shares
 * its parents: each row below the group is walked once for the whole group, and
 * the group's Schur update is a dense FP32 product on MFMA
 * (v_mfma_f32_16x16x4f32), followed by the group's dense diagonal block with
 * FP64 pivots.  The levels are those of the group DAG.  Update counting, FP64
 * factors and other plans use the entry-wise factorization.  enable = 0 selects
 * the entry-wise factorization for this factor too (results differ only by
 * FP32 rounding order).  KC_EINVAL when enabling on a factor without groups. */
kc_status kc_factor_use_groups(kc_factor *f, int32_t enable);

/* Rows of S with more than max_parents parents are not staged in LDS: the
 * factorization's wavefronts read such a row's indices and values from device
 * memory (the same merge, the same updates in the same order of Section 2.2's
 * algorithm, so the same L; slower).  Rows that do not fit in LDS take that
 * path anyway, so no pattern is refused for its row lengths; a factor starts
 * with the largest limit the LDS allows, and max_parents = -1 restores it.
 * Supernodal groups and match masks need every row staged: with a longer row
 * the factorization is entry-wise and kc_factor_match_build returns KC_ERANGE;
 * lowering the limit under attached masks returns KC_EINVAL. */
kc_status kc_factor_set_stage_limit(kc_factor *f, int32_t max_parents);

/* Autotuner: times the factorization (reps repetitions after a warm-up) for
 * every schedule in {1, 2, 4} wavefronts per workgroup x level grouping
 * persist_max in {0, 256, 4096, all levels} x unit order {SPATIAL, LONGEST} --
 * skipping those whose staged rows do not fit in LDS or whose persistent grid
 * cannot be resident -- and keeps the fastest for this factor
 * (kc_factor_schedule reports it).  Results are bitwise identical for every
 * choice.  For a batch plan pass ell_dev (and ell is ignored), else NULL. */
kc_status kc_factor_tune(kc_factor *f, const double *x_dev, double nu, double ell, const double *ell_dev,
                         kc_pivot pivot, double tau, int32_t reps, void *stream, int32_t *chosen_wpb);

/* Captures factorize + solve of this factor into a HIP graph (on an internal
 * stream; no memory is allocated by the captured work) so that one
 * kc_graph_launch replays every level launch (with the factor's wavefronts per
 * workgroup, one launch per level).  Arguments are those of
 * kc_factorize/kc_factorize_batched and kc_solve; the pointers are baked into the
 * graph and must stay valid.  Replays on a stream are ordered like any other
 * work on it.  Creating the graph runs nothing: the factor keeps its state
 * (kc_solve still needs a computed factor) until the first kc_graph_launch,
 * after which kc_factor_stats and kc_factor_export_L wait for the latest
 * replay on the stream it was launched on. */
kc_status kc_graph_create(kc_factor *f, const double *x_dev, double nu, double ell, const double *ell_dev,
                          kc_pivot pivot, double tau, const double *b_dev, double *sol_dev, int32_t nrhs,
                          void *scratch_dev, size_t scratch_bytes, kc_graph **out);
/* Number of nodes of the recorded graph, and whether its factorization was
 * recorded with persistent launches (1) or as one launch per level (0).
 * Graphs currently record one launch per level: a persistent launch needs the
 * runtime's cooperative launch path, which is used eagerly only. */
kc_status kc_graph_info(const kc_graph *g, int64_t *nodes, int32_t *persistent);
kc_status kc_graph_launch(kc_graph *g, void *stream);
void kc_graph_destroy(kc_graph *g);

/* ---------------------------------------------------------------- refinement */

typedef struct {
    int32_t iterations;        /* CG iterations performed (products with the search directions) */
    int32_t converged;         /* 1 when every right-hand side's true residual reached tol */
    double max_rel_residual;   /* max over right-hand sides of ||r||/||b||, recursive residual */
    double t_matvec_ms;        /* time in dense Theta products (residual checks included) */
    double t_precond_ms;       /* time in the preconditioner solves */
    double true_rel_residual;  /* max over right-hand sides of ||b - Theta x||/||b||, recomputed with one
                                  dense product once the recursive residual met tol (or at maxit) */
    int32_t restarts;          /* times CG restarted from the true residual because it was above tol */
    int32_t pad;
} kc_pcg_info_t;

/* Y = Theta X with the dense N x N Matern matrix (Section 4.4) generated on the
 * fly: x_dev N x d (d <= 32) points, X_dev/Y_dev N x nrhs row-major, all in the
 * same (any) order.  FP64; X and Y may not alias. */
kc_status kc_dense_matvec(const double *x_dev, int64_t n, int32_t d, kc_kernel kernel, const double *X_dev,
                          double *Y_dev, int32_t nrhs, void *stream);

/* Scratch needed by kc_pcg. */
kc_status kc_pcg_bytes(const kc_factor *f, int32_t nrhs, size_t *bytes);

/* Conjugate gradients on the dense system Theta x = b preconditioned by the
 * factor, M^{-1} = P^T L^{-T} L^{-1} P (the paper suggests CG with the sparse
 * factor as preconditioner, Sections 4.2-4.3).  x0 = 0; each right-hand side
 * stops when its recursively updated ||r||/||b|| <= tol (FP64 residuals).  Then
 * the true residual b - Theta x is computed with one more dense product; where
 * it is still above tol, CG restarts from it (info->restarts) until it meets tol
 * or maxit products have been spent.  b_dev, sol_dev: N x nrhs in the original
 * order; x_dev: the points the factor was computed from.  Blocks the host once
 * per iteration for the convergence test. */
kc_status kc_pcg(kc_factor *f, const double *x_dev, kc_kernel kernel, const double *b_dev, double *sol_dev,
                 int32_t nrhs, double tol, int32_t maxit, void *scratch_dev, size_t scratch_bytes, void *stream,
                 kc_pcg_info_t *info);

/* Number of HIP devices visible (0 if none); for availability checks. */
int32_t kc_device_count(void);

#ifdef __cplusplus
}
#endif
#endif /* KCHOL_H */
