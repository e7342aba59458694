/*
 * pms.h -- C ABI of the MI355X (gfx950) parallel multi-scale reduction of a
 * persistent-homology boundary matrix over F2.
 *
 * Method: Mendoza-Smith & Tanner, "Parallel multi-scale reduction of
 * persistent homology filtrations" (arXiv 1708.04710).  The problem is the
 * one of the paper's introduction and Sec. 2.3: given the boundary matrix
 * d in F2^{m x m} of a compatibly ordered filtration (eq.
 * "def:boundary_matrix"), compute low* (eq. "low": the entrywise minimum of
 * low under left-to-right column additions), and from it the persistence
 * pairs (low*(j), j) and the essential simplices (Sec. 2.3, sets Pos / Neg /
 * Ess).
 *
 * Conventions for every entry point
 *   - Indices are 0-based; -1 stands for the paper's 0 ("no entry").
 *   - Every array argument is a DEVICE pointer unless stated otherwise, owned
 *     by the caller, and is only read (inputs) or written (outputs) on the
 *     context's HIP stream.  The library never frees caller memory.
 *   - The library owns its scratch (column arena, tables, bitmasks).  It is
 *     allocated on first use, kept in the context and grown when a larger
 *     problem arrives; pms_destroy releases it.
 *   - A context is bound to one device and one stream and is not thread
 *     safe: use one context per host thread / stream.
 *   - Errors are reported by the return status; no C++ exception crosses
 *     the ABI.  pms_last_error() gives a message for the last failure.  On
 *     error, output arrays hold unspecified values and counts are 0, except
 *     PMS_ERR_CAPACITY (counts hold the required sizes) and
 *     PMS_ERR_NOT_CONVERGED (low_star holds the pairs known so far).
 *   - Every call returns after its results are complete on the stream and
 *     its host-visible counts are filled in (one small device-to-host copy).
 */
#ifndef PMS_H
#define PMS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PMS_OK = 0,
    PMS_ERR_INVALID_ARG = -1,    /* null pointer, negative size, bad option */
    PMS_ERR_NOT_COMPATIBLE = -2, /* rows not strictly ascending, row >= column,
                                    or dim(row) != dim(column) - 1 */
    PMS_ERR_OOM = -3,            /* device allocation failed */
    PMS_ERR_HIP = -4,            /* a HIP runtime call failed */
    PMS_ERR_NOT_CONVERGED = -5,  /* max_rounds reached before low was injective */
    PMS_ERR_CAPACITY = -6,       /* output buffers too small; counts hold the sizes */
    PMS_ERR_INVARIANT = -7,      /* debug_invariants: a property the theory guarantees
                                    did not hold (a library bug); the message names it */
    PMS_ERR_TOO_LARGE = -8       /* pms_reduce_noalloc: the problem does not fit the
                                    fixed region (use pms_reduce) */
} pms_status;

typedef struct pms_ctx pms_ctx;

/* Create a context on `device` that issues all work on `stream` (a
 * hipStream_t; NULL = the default stream).  *ctx receives the handle. */
pms_status pms_create(pms_ctx **ctx, int device, void *stream);
/* Release the context and the scratch it owns.  NULL is accepted. */
void pms_destroy(pms_ctx *ctx);
/* Message of the last failed call on ctx (owned by ctx, valid until the
 * next call); "" when the last call succeeded.  NULL ctx -> static text. */
const char *pms_last_error(const pms_ctx *ctx);
/* Library version string (static). */
const char *pms_version(void);
/* Checks the device's wave-level primitives (DPP reductions) against
 * reference shuffles on ctx's device, and the debug_invariants detectors on
 * fabricated states that each break one property; PMS_OK when all agree. */
pms_status pms_selftest(pms_ctx *ctx);

/* Boundary matrix d of a filtration in filtration order, CSC:
 *   column j (simplex sigma_j) holds rows[col_ptr[j] .. col_ptr[j+1]) -- the
 *   filtration indices of the codimension-1 faces of sigma_j -- strictly
 *   ascending and < j (eq. "def:boundary_matrix": sparse, binary, upper
 *   triangular).  dim[j] is the dimension of sigma_j (eq. "Kp"); it may be
 *   NULL, in which case the dimension checks are skipped and Phase I treats
 *   all columns as one dimension (still exact, fewer early pivots). */
typedef struct {
    int64_t m;              /* number of simplices (columns), >= 0, < 2^31 - 1 */
    const int64_t *col_ptr; /* [m+1], col_ptr[0] = 0, non-decreasing */
    const int32_t *rows;    /* [col_ptr[m]] */
    const int8_t *dim;      /* [m] or NULL */
    /* Optional, both or neither (NULL): left (Def. "left": the first column
     * holding row i, 2^31 - 1 when none) and beta (Def. "beta": the largest
     * row r of column j with left(r) = j, -1 when none), device [m], as a
     * filtration builder can produce them (Sec. 3, after Alg. "Building
     * beta").  Given, Phase 0 reads them instead of computing them; they must
     * equal the definitions (debug_invariants then checks beta's bounds). */
    const int32_t *left;
    const int32_t *beta;
} pms_boundary;

/* Options.  Zero-initialise and set what you need; pms_default_options()
 * returns the recommended values. */
typedef struct {
    /* Source of each column addition in a round (Phase II, Sec. 3.1):
     *   0 = a colliding column is added the leftmost column with the same low
     *       (a pivot when one is known, else the leftmost unreduced column);
     *   1 = only known pivots are added (Alg. "Parallel multi-scale
     *       reduction" as printed).  Both give the same low* (Sec. 2.3). */
    int32_t variant;
    /* 1 = delete rows of simplices known to be negative (compression,
     *     Sec. 2.4 and Sec. 3.2): such rows never hold a low*.  */
    int32_t compression;
    /* Rounds (outer iterations) before giving up; 0 = unbounded (the
     * iteration converges, Thm. "Convergence"). */
    int32_t max_rounds;
    /* Pivot chaining: a column that is known negative (beta_j > 0, Thm.
     * "Properties of beta_j" P.3) or of top dimension (can never be
     * cleared) keeps adding known pivots within a round while its low has
     * one.  0 = one addition per column per round. */
    int32_t chain;
    /* Below this many active columns every column chains (tail mode). */
    int32_t tail_active;
    /* 1 = check the CSC input (sorted rows, upper triangular, dims). */
    int32_t validate;
    /* > 0: run the rounds as a HIP graph of this many rounds (rounded up to
     * even) captured once and replayed, one host synchronisation per replay
     * instead of one per round; rounds after convergence do nothing.  Used
     * only with max_rounds = 0 and the profiler off.  0 = one round at a time. */
    int32_t graph_rounds;
    /* 1 = record the per-round diagnostics (pms_round_stats_read) and the
     * essential estimate (pms_essential_estimate); runs one round at a time
     * (no graph), with two extra passes over the columns per round. */
    int32_t diagnostics;
    /* Initial capacity of the column arena in int32 entries; 0 = automatic.
     * A non-zero value reallocates the arena to exactly this size (the
     * arena still grows when fill-in exceeds it). */
    int64_t arena_entries;
    /* 1 = check, on the device after Phase 0, after every kernel that writes
     * columns and after every round, the properties the theory guarantees,
     * and fail with PMS_ERR_INVARIANT naming the first one broken:
     *   - lows never increase (Sec. 3.1, "Convergence": additions only
     *     remove the low; compression only deletes rows);
     *   - beta_j <= low(j), and a column with beta_j defined is never zero
     *     (Thm. "Properties of beta_j" P.5 and P.3);
     *   - a pivot column never changes again, and piv / low_star name it;
     *   - no column is written twice by one kernel launch (no two threads
     *     own one column);
     *   - no essential simplex ever leaves the estimate E^l (Lemma
     *     "Essential estimation": Ess is a subset of every E^l), checked
     *     against the final Ess;
     *   - at the end low*(j) is the last low seen and beta_j <= low*(j).
     * Runs one round at a time (no graph) with several extra passes over the
     * columns per round; for testing, not production.  0 = off. */
    int32_t debug_invariants;
    /* 1 = clearing by local compression (Sec. 3.2, Lemma "Clearing by local
     * compression" and its Corollary, the case L_j = {0}) every round, after
     * Phase I: a column j of dimension d >= 1 not known negative (no beta_j)
     * whose low lies below every (d-1)-simplex of its complex that is not
     * yet paired (not known negative and not the low* of a found pivot) is
     * positive, and is cleared without further additions.  With
     * pms_reduce_batched the complex is the instance that holds column j
     * (the matrix is block diagonal, so low*(j) is a row of that block).
     * Needs dim.  0 = off. */
    int32_t c8;
    /* 0 = every dimension reduced at once (the default);
     * 1 = twist order (Alg. "Standard reduction with a twist"): the rounds
     *     run on the columns of the top dimension until they are reduced,
     *     then on the next dimension down, and so on; the pivots found in
     *     dimension d clear (zero) the columns of dimension d-1 that are
     *     their lows before those columns are reduced.  Needs dim. */
    int32_t sweep;
    /* Which colliding columns add in a round when round_budget limits them
     * (Sec. 3.4, fewer processors than colliding columns):
     *   0 = in column order;
     *   1 = the columns of the largest sets N(i) first (the columns whose
     *       low is i: one known pivot serves them all), then column order;
     *   2 = the columns known negative (beta_j defined) first, then column
     *       order (their reduction clears the columns of their low*). */
    int32_t priority;
    /* > 0: at most this many columns make the round's first addition (and
     * chain on, when chaining); the others wait for a later round.
     * 0 = every colliding column adds (no limit). */
    int32_t round_budget;
    int32_t reserved; /* 0 */
} pms_options;

pms_options pms_default_options(void);

/* Results.  low_star is required ([m], caller-allocated).  The pair and
 * essential arrays are optional (NULL with capacity 0 = not wanted); when
 * given they receive, in canonical order,
 *   pairs: (pair_birth[k], pair_death[k]) = (low*(j), j) for every j with
 *          low*(j) >= 0, ascending in j (Sec. 2.3: Neg paired with Pos);
 *   essential: every i with low*(i) = -1 that is no column's low*,
 *          ascending (set Ess of Sec. 2.3).
 * Host-visible outputs are filled by the call. */
typedef struct {
    int32_t *low_star;      /* [m] device */
    int32_t *pair_birth;    /* [cap_pairs] device or NULL */
    int32_t *pair_death;    /* [cap_pairs] device or NULL */
    int64_t cap_pairs;
    int32_t *essential;     /* [cap_essential] device or NULL */
    int64_t cap_essential;
    /* host-visible outputs */
    int64_t n_pairs;
    int64_t n_essential;
    int32_t rounds;         /* outer iterations run (Sec. 4: one Phase I + Phase II) */
    int32_t phase0_pivots;  /* pivots known from beta before any addition (Phase 0) */
    int64_t additions;      /* column additions performed (the paper's cost unit) */
    int64_t xor_entries;    /* entries read by those additions */
    int64_t active_sum;     /* sum over rounds of the round's active columns (the columns
                               the per-round kernels pass over) */
    int64_t addition_bytes; /* sum over the additions t <- t + s of 4 (len t + len s +
                               len(t + s)): the bytes a column addition reads and writes
                               by itself.  Exact for a column's first addition in a round;
                               for the chained additions after it, len t counts the
                               column's pending toggles, and len(t + s) = len t + len s - 2
                               (only the low is known to cancel) */
} pms_result;

/* Reduce one boundary matrix (Alg. "Parallel multi-scale reduction":
 * Phase 0 with beta of Def. "beta", then rounds of Phase I local injections
 * (Alg. "Finding local injections", Thms. "Local injection I/II") and
 * Phase II simultaneous column additions, with clearing and compression). */
pms_status pms_reduce(pms_ctx *ctx, const pms_boundary *bnd, const pms_options *opt, pms_result *res);

/* Allocation-free reduction, for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid
 * it).  The same reduction and outputs as pms_reduce, but every scratch
 * buffer -- per-column state, tables, queues, counters and the column arena
 * -- is carved from one fixed device region of PMS_NOALLOC_BYTES per device,
 * reserved when the library is loaded and held until the process ends; the
 * call makes no device or pinned allocation and frees nothing.
 *   - Limits: the per-column state takes about 100 bytes per column (130
 *     with debug_invariants) and the arena at least 4 nnz + 2^20 entries of
 *     4 bytes; a matrix that does not fit, or whose fill-in outgrows the
 *     arena during the reduction (the arena cannot grow), fails with
 *     PMS_ERR_TOO_LARGE.  About 500 000 columns of a lower-star or
 *     Vietoris-Rips filtration fit.
 *   - Options: graph_rounds, diagnostics and arena_entries must be 0, and
 *     the context's profiler off (PMS_ERR_INVALID_ARG otherwise).
 *   - The region is shared by every context and call on a device and keeps
 *     the last call's contents (each call clears what it needs): calls that
 *     overlap in time on one device, from any context or stream, race and
 *     give undefined results.  Serialise them.
 * Everything else (ownership of inputs / outputs, statuses, synchronisation)
 * is as for pms_reduce. */
#define PMS_NOALLOC_BYTES (128ull << 20)
pms_status pms_reduce_noalloc(pms_ctx *ctx, const pms_boundary *bnd, const pms_options *opt, pms_result *res);

/* Reduce `count` filtrations concatenated block-diagonally (as built by
 * pms_build_vr_*: instance b owns the columns [inst_col_off[b],
 * inst_col_off[b+1]) and its rows stay in that range), in one pms_reduce of
 * the whole matrix; the instances never interact, so each gets its own
 * exact pairs (Sec. 2.3).  inst_col_off: device, count + 1 entries
 * ascending from 0 to m (checked: PMS_ERR_INVALID_ARG otherwise).  Outputs
 * beyond pms_reduce's, each optional (NULL = not wanted), device:
 *   inst_pair_off[b], inst_ess_off[b] (count + 1 entries): where instance
 *     b's pairs / essential simplices start in res's arrays (its pairs are
 *     those whose death column is in its range; they are contiguous since
 *     the arrays ascend);
 *   pair_inst[k] (res->cap_pairs entries): the instance of pair k.
 * The pair / essential arrays of res must be given for the offsets of
 * the pairs / essentials to be meaningful (0 otherwise). */
pms_status pms_reduce_batched(pms_ctx *ctx, int32_t count, const int64_t *inst_col_off, const pms_boundary *bnd,
                              const pms_options *opt, pms_result *res, int64_t *inst_pair_off, int64_t *inst_ess_off,
                              int32_t *pair_inst);

/* ------------------------------------------------------------------------
 * Multi-scale diagnostics (Sec. 4's measurements of the iteration).  With
 * pms_options.diagnostics = 1 a reduction records one entry after Phase 0
 * (round 0: beta known, no column added) and one after every round l,
 * describing low^l, the lows at that point (a column's low with the rows of
 * simplices known negative deleted, compression; -1 for a zero column):
 *   - low_l1 = sum_j (low^l(j) + 1), ||low^l||_1 in the paper's 1-based
 *     indexing.  Lows only decrease and end at low*, so the relative l1-error
 *     of eq. "rel_error" is (low_l1 - ||low*||_1) / ||low*||_1, with
 *     ||low*||_1 the last entry's low_l1 of a converged reduction;
 *   - active: columns not yet reduced (neither a pivot nor zero), the
 *     proportion of unreduced columns times m;
 *   - ess_estimate = |E^l|, eq. "essential_iteration": E^0 = [m] and
 *     E^{l+1} = (E^l minus the indices known paired -- columns known negative
 *     and the lows of the pivots) minus {low^l(j)}.  By Lemma "Essential
 *     estimation" Ess is a subset of every E^l; at convergence E = Ess.
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t round;          /* l (0 = after Phase 0) */
    int32_t active;         /* columns neither pivot nor zero */
    int64_t new_pivots;     /* pivots found in the round */
    int64_t additions;      /* column additions in the round */
    int64_t xor_entries;    /* entries those additions read */
    int64_t low_l1;         /* sum_j (low^l(j) + 1) */
    int64_t ess_estimate;   /* |E^l| */
    int64_t c8_cleared;     /* columns cleared by pms_options.c8 in the round */
} pms_round_stats;

/* The entries recorded by the context's last reduction with diagnostics
 * (host array out[cap]); *count receives their number (cap = 0 to ask). */
pms_status pms_round_stats_read(pms_ctx *ctx, int32_t cap, pms_round_stats *out, int32_t *count);
/* E^l of the last recorded entry as a bitmask: bit i of word i / 32 set iff
 * i is in E^l.  bits: device, (m + 31) / 32 words; m must be the last
 * reduction's.  A reduction stopped by max_rounds leaves the estimate of its
 * last completed round. */
pms_status pms_essential_estimate(pms_ctx *ctx, int64_t m, uint32_t *bits);

/* ------------------------------------------------------------------------
 * Tuning.  Pivot chaining (an addition to Phase II of Sec. 3.1: a column
 * keeps adding the known pivot of its low within a round) runs in lane
 * kernels, one lane per queued column, then, for the columns the lanes
 * hand on, a workgroup kernel that solves each chain by sweeps and a
 * wavefront kernel that walks a chain one addition at a time.  Their launch shapes and
 * hand-over thresholds are a per-context pms_tuning.  Every valid setting
 * gives the same low*, pairs and essential simplices (a reduced matrix's
 * lows are unique, Sec. 2.3); only speed changes, and with it possibly the
 * arena's history and so the round count.
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t lane_blocks;    /* grid of the lane kernel (128-thread blocks), 1..65535 */
    int32_t chain_blocks;   /* grid of the wavefront kernel (256-thread blocks), 1..65535 */
    int32_t lane_steps;     /* additions a lane makes to one column before handing it to
                               the wavefront kernel, when at least lane_many columns are
                               queued in the round; 0..2^30 */
    int32_t lane_steps_few; /* the same when fewer are queued; 0..2^30 */
    int32_t lane_many;      /* queued columns from which the round uses lane_steps; >= 0 */
    int32_t lane_refill;    /* a wave writes back and refills its lanes once this many
                               (or all) are free; 1..64 */
    int32_t lane_flush;     /* a wave merges its lanes' pending entries once this many
                               (or all busy) lanes have a full pending set; 1..64 */
    int32_t wide_blocks;    /* grid of the lane kernel's second pass (64-thread blocks, an
                               80-entry buffer per lane) for the columns too long for the
                               first pass; 1..65535 */
    int32_t lane_cap;       /* entries of the first pass's per-lane buffer in use (longer
                               columns go to the second pass); 0..39 */
    int32_t solve;          /* when the lanes hand on at most this many columns in a
                               round, they are reduced by sweeps of the triangular system
                               their chain solves (one workgroup per column, chain_blocks
                               256-thread blocks; the pivots added are the serial chain's),
                               those that do not fit its LDS table by the wavefront
                               kernel; more columns, or 0, go to the wavefront kernel
                               only; 0..2^30 */
} pms_tuning;

/* The built-in setting: 2048, 512, 128, 0, 65536, 32, 16, 2048, 39, 512. */
pms_tuning pms_default_tuning(void);
/* Make *t the context's setting for later reductions (NULL = the built-in
 * one).  PMS_ERR_INVALID_ARG, setting unchanged, when a field is out of range. */
pms_status pms_set_tuning(pms_ctx *ctx, const pms_tuning *t);
/* The context's current setting into *t (host). */
pms_status pms_get_tuning(pms_ctx *ctx, pms_tuning *t);
/* Time n candidates on one boundary matrix and keep the fastest.
 * Candidate i is (opts[i], tunes[i]) (host arrays of n; opts NULL = the
 * default options for all); each runs pms_reduce once untimed, then `reps`
 * (1..64) times timed by the host clock, and scores the median.  ms[i]
 * (host, optional) receives the scores, *best (host) the winner's index.
 * On success the context keeps tunes[*best] and res holds the outputs of
 * one more reduction with the winner; on failure the context's setting is
 * unchanged and the failing call's status is returned.  The profiler, when
 * on, adds its overhead to every candidate alike. */
pms_status pms_autotune(pms_ctx *ctx, const pms_boundary *bnd, int32_t n, const pms_options *opts,
                        const pms_tuning *tunes, int32_t reps, pms_result *res, double *ms, int32_t *best);

/* ------------------------------------------------------------------------
 * Filtrations built on the device.  A pms_filtration is library-owned
 * device memory holding a filtration in compatible order (Sec. 2.2: the
 * simplices of each sub-complex precede the rest, faces precede cofaces),
 * ordered by the key (value, dimension, lexicographic vertex tuple), with its
 * boundary matrix (eq. "def:boundary_matrix").  Pass *f = NULL to allocate a
 * new one, or an existing one to rebuild in place (its buffers are reused
 * when large enough).  Free it with pms_filtration_free.
 * ------------------------------------------------------------------------ */
typedef struct pms_filtration pms_filtration;

typedef struct {
    int64_t m, nnz;
    const int64_t *col_ptr;   /* [m+1] device */
    const int32_t *rows;      /* [nnz] device, ascending per column */
    const int8_t *dim;        /* [m] device */
    const float *value_f32;   /* [m] device, FP32 filtration values, or NULL */
    const int64_t *value_i64; /* [m] device, int64 values (squared distances), or NULL */
    const int32_t *crit;      /* [2m] device: the vertex (lower-star: the argmax vertex by
                                 (value, id), then -1) or edge endpoints (Vietoris-Rips: the
                                 edge whose length is the simplex's value, latest in the
                                 filtration; -1 -1 for vertices) that fixes each value */
    const int32_t *verts;     /* [4m] device, ascending vertex ids, -1 padded */
    const int32_t *left;      /* [m] device, Def. "left" (2^31 - 1: none), or NULL when the
                                 builder does not produce it (lower-star does) */
    const int32_t *beta;      /* [m] device, Def. "beta" (-1: none), or NULL likewise */
} pms_filtration_view;

/* Lower-star filtration of the Freudenthal triangulation of an
 * nx x ny x nz grid of FP32 values (`grid` device, x fastest: vertex id =
 * x + nx*(y + ny*z)).  Simplices are the chains of grid vertices whose steps
 * are non-zero 0/1 vectors with disjoint supports (6 tetrahedra per cube);
 * the value of a simplex is its largest vertex value.  -0 counts as +0;
 * NaN -> PMS_ERR_INVALID_ARG.  Grids of 2^26 vertices or more are rejected. */
pms_status pms_build_lowerstar(pms_ctx *ctx, const float *grid, int32_t nx, int32_t ny, int32_t nz,
                               pms_filtration **f);
/* Vietoris-Rips filtrations to dimension maxdim (0..3) of `count` point
 * clouds at once (Sec. 2.2: a simplex enters when its diameter is at most
 * 2r, i.e. the value of a simplex is its squared diameter).  Cloud b has
 * n[b] points of D[b] coordinates stored row-major at pts + pt_off[b]
 * (pts: device; n, D, pt_off, thr_sqd: host arrays of `count` entries).
 * thr_sqd[b] < 0 keeps every simplex, else simplices with squared
 * diameter <= thr_sqd[b].  The clouds' filtrations are concatenated
 * block-diagonally: cloud b owns the columns [inst_col_off[b],
 * inst_col_off[b+1]) (host output of count+1 entries, may be NULL), and
 * its rows stay in that range, so one pms_reduce of the whole matrix
 * reduces every cloud exactly.  Vertices ids in `verts` / `crit` are global
 * point numbers (cloud b's point a is sum_{b'<b} n[b'] + a).
 *   _i32: integer coordinates, exact int64 squared distances (< 2^35),
 *         n[b] <= 511;
 *   _f32: FP32 coordinates; the squared distance is rounded step by step
 *         in coordinate order (d = x_a - x_b; s = s + d*d, no fused
 *         multiply-add); n[b] <= 1023.
 * Order within a cloud: (value, dimension, lexicographic vertex tuple).  A
 * tetrahedron's value is the largest squared distance among its four
 * vertices, its critical edge (`crit`) the latest of its six edges in the
 * filtration.  More than 32 bits of simplices in total, or a cloud outside
 * the size limits, gives PMS_ERR_INVALID_ARG. */
pms_status pms_build_vr_i32(pms_ctx *ctx, const int32_t *pts, int32_t count, const int32_t *n, const int32_t *D,
                            const int64_t *pt_off, const int64_t *thr_sqd, int32_t maxdim, pms_filtration **f,
                            int64_t *inst_col_off);
pms_status pms_build_vr_f32(pms_ctx *ctx, const float *pts, int32_t count, const int32_t *n, const int32_t *D,
                            const int64_t *pt_off, const float *thr_sqd, int32_t maxdim, pms_filtration **f,
                            int64_t *inst_col_off);
/* Device pointers of a built filtration (valid until it is rebuilt or freed). */
pms_status pms_filtration_view_get(const pms_filtration *f, pms_filtration_view *v);
/* Copy a built filtration into caller-owned device buffers on ctx's stream
 * (any pointer may be NULL to skip that array; value is float or int64 as
 * the view says; crit holds 2m and verts 4m entries).  Returns after the
 * copies complete. */
pms_status pms_filtration_copy_out(pms_ctx *ctx, const pms_filtration *f, int64_t *col_ptr, int32_t *rows,
                                   int8_t *dim, void *value, int32_t *crit, int32_t *verts);
/* Copy the filtration's left and beta (Defs. "left", "beta"; see
 * pms_filtration_view) into caller-owned device arrays of m entries on ctx's
 * stream (either may be NULL); returns after the copies complete.
 * PMS_ERR_INVALID_ARG when the builder did not produce them. */
pms_status pms_filtration_copy_left_beta(pms_ctx *ctx, const pms_filtration *f, int32_t *left, int32_t *beta);
/* Release a filtration (synchronises its device).  NULL is accepted. */
void pms_filtration_free(pms_filtration *f);

/* ------------------------------------------------------------------------
 * Values of simplices and the backward pass through a fixed pairing.
 * With the pairs fixed, a persistence loss depends on the input only through
 * the values of the paired simplices; each value is the value of one
 * critical vertex (lower-star: the argmax vertex by (value, id)) or the
 * squared length of one critical edge (Vietoris-Rips: the simplex's latest
 * facet edge).  All arrays are device arrays of n entries.
 * ------------------------------------------------------------------------ */
/* values[k] = value of simplex[k] (float or int64 as the filtration's
 * view says; NULL to skip); dims[k] = its dimension (NULL to skip). */
pms_status pms_gather(pms_ctx *ctx, const pms_filtration *f, int64_t n, const int32_t *simplex, void *values,
                      int8_t *dims);
/* grad_grid[v] += sum of grad[k] over the k whose simplex has critical
 * vertex v (grad_grid: n_vertices floats, zeroed by the caller). */
pms_status pms_backward_lowerstar(pms_ctx *ctx, const pms_filtration *f, int64_t n, const int32_t *simplex,
                                  const float *grad, float *grad_grid, int64_t n_vertices);
/* For a filtration built by pms_build_vr_f32 from clouds whose points are
 * stored contiguously (point g at pts + g*D): with (a, b) the critical edge
 * of simplex[k], grad_pts[a] += 2 grad[k] (x_a - x_b) and grad_pts[b] -= the
 * same (grad_pts: n_points * D floats, zeroed by the caller).  Vertices
 * (value 0) contribute nothing.  FP32 atomics: the summation order varies. */
pms_status pms_backward_vr_f32(pms_ctx *ctx, const pms_filtration *f, int64_t n, const int32_t *simplex,
                               const float *grad, const float *pts, int32_t D, int64_t n_points, float *grad_pts);

/* Per-kernel timing, opt-in.  pms_profile_enable(ctx, 1) zeroes the totals
 * and from then on records a HIP event pair on ctx's stream around every
 * kernel launch of the library, with the launch's algorithmic bytes (the
 * bytes the step must move: inputs read once, outputs written once).
 * pms_profile_read() synchronises ctx's stream and returns, for kernel slot
 * k (0 <= k < pms_profile_kernels()), the summed event time in ms, the
 * number of launches and the summed algorithmic bytes.  Enabling adds
 * event overhead; leave it off in production. */
pms_status pms_profile_enable(pms_ctx *ctx, int enable);
int pms_profile_kernels(void);
const char *pms_profile_kernel_name(int k); /* static, NULL when out of range */
pms_status pms_profile_read(pms_ctx *ctx, int k, double *total_ms, int64_t *launches, double *bytes);
/* For the kernels that add columns (0 for the others): the summed bytes of
 * their additions at 4 (len t + len s + len(t + s)) each, as in
 * pms_result.addition_bytes, since pms_profile_enable. */
pms_status pms_profile_read_addition_bytes(pms_ctx *ctx, int k, double *bytes);

#ifdef __cplusplus
}
#endif

#endif /* PMS_H */
