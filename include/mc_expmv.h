/*
 * mc_expmv.h -- C ABI of libmcexpmv, an MI355X (gfx950) implementation of the
 * Monte Carlo estimator of exp(tA) v from J. A. Acebron, "A Monte Carlo method
 * for computing the action of a matrix exponential on a vector"
 * (arXiv:1904.12759).
 *
 * The method (paper Sec. 2-3): write A = D - L where the off-diagonal entries
 * a_ij >= 0 of A are jump rates of a continuous-time Markov chain with
 * generator Q = -L.  For row i
 *     r_i = sum_{j != i} a_ij   (exit rate),   d_i = a_ii + r_i,
 *     k_ij = a_ij / r_i         (jump law, Eq. (paths)).
 * A walker started at node i waits Exp(r_x) in every visited state x, jumps
 * with law k_x., stops at the horizon t, and returns  W * v[X_t]  where W is
 * the multiplicative functional of Theorem 1 (Lemma 1 for one step):
 *     MC_EXACT   W = exp( integral_0^t d(X_s) ds )   (the dt -> 0 limit of the
 *                splittings; unbiased for exp(tA) v itself)
 *     MC_STRANG  W = exp( dt * sum_k c_k d(X_{k dt}) ), c_0 = c_N = 1/2,
 *                unbiased for the Strang product of Eq. (eq_general1)
 *     MC_LIE     W = exp( dt * sum_{k>=1} d(X_{k dt}) ), unbiased for the Lie
 *                product of Eq. (deff).
 * Entry i of the result is the mean of W * v[X_t] over the walkers started at
 * i (Algorithm 1); the full vector is that mean for every start node.
 *
 * Random numbers are Philox4x32-10 (Salmon et al., SC'11) keyed by the seed,
 * with counter (event index, walker ordinal, start node, instance id), so every
 * walker's path is a pure function of (A, t, seed, start node, ordinal,
 * instance id) and of nothing about the launch.
 *
 * Conventions for every entry point:
 *   - Device pointers are HIP device (or managed) pointers on the current
 *     device; host pointers are named as such.  Buffers passed in are owned by
 *     the caller; the handle owns only what it allocates.
 *   - Work is enqueued on opts.stream (NULL = the null stream) and is
 *     asynchronous.  Argument errors are returned at once; errors found on the
 *     device (an entry index out of range, the walk-length cap, a weight that
 *     overflows) are latched in the handle and returned by mc_expmv_sync.
 *   - A handle is not thread safe; use one per host thread.
 *   - No C++ exception crosses this interface.
 *   - Allocation failures return MC_ERR_NO_MEMORY after freeing what the call
 *     allocated.  For testing those paths, MC_EXPMV_FAULT=alloc:K in the
 *     environment makes the K-th device or pinned-host allocation of each call
 *     fail (the count restarts at every entry point that allocates, nested ones
 *     included).
 */
#ifndef MC_EXPMV_H
#define MC_EXPMV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MC_OK = 0,
    MC_ERR_INVALID_ARG = 1,   /* bad pointer, size, shape, column index or option */
    MC_ERR_NOT_METZLER = 2,   /* an off-diagonal entry is negative (not a jump rate) */
    MC_ERR_NONFINITE = 3,     /* NaN or Inf in A, t, dt or a proposal bias */
    MC_ERR_OUT_OF_RANGE = 4,  /* a requested entry index is outside [0, n) */
    MC_ERR_NOT_SYMMETRIC = 5, /* the forward (Algorithm 2) estimator needs A == A^T */
    MC_ERR_NO_MEMORY = 6,     /* a device or host allocation failed */
    MC_ERR_DEVICE = 7,        /* a HIP runtime call failed */
    MC_ERR_WALK_LIMIT = 8,    /* a walker reached opts.max_events holding intervals */
    MC_ERR_OVERFLOW = 9,      /* a walker's weight W * v[X_t] is not finite */
    MC_ERR_TOO_LARGE = 10     /* mc_expmv_entries_noalloc: the run needs more than its
                                 fixed scratch */
} mc_status;

enum { MC_EXACT = 0, MC_STRANG = 1, MC_LIE = 2 };
enum { MC_FP64 = 0, MC_FP32 = 1 };

typedef struct mc_expmv_s *mc_expmv_t;

typedef struct {
    uint32_t struct_size;       /* sizeof(mc_expmv_opts), for versioning */
    int32_t mode;               /* MC_EXACT (default), MC_STRANG or MC_LIE */
    double dt;                  /* requested splitting step; N = ceil(t/dt), dt := t/N.
                                   Ignored in MC_EXACT. Default 0.03125 (paper Sec. 6). */
    int32_t weight_prec;        /* MC_FP64 (default): weights and v in double.
                                   MC_FP32: d, log-weight, exp and v in float; time,
                                   RNG and reductions stay FP64/integer. */
    int32_t relabel;            /* 1: order rows by descending exit rate in device memory
                                   (paths and results are unchanged). Default 0. */
    uint32_t lds_budget;        /* bytes of LDS per block for hot rows (needs relabel);
                                   0 = off (default) */
    uint32_t resort_period;     /* needs relabel: every this many events a wavefront
                                   re-sorts its walkers by current (relabelled) node,
                                   each walker's state moving with it, so that
                                   neighbouring lanes gather neighbouring rows; results
                                   are bitwise unchanged.  0 = never (default). */
    uint32_t walkers_per_block; /* threads per block: 64 (default, one wave), 128 or 256 */
    uint32_t instance_id;       /* fourth Philox counter word. Default 0. */
    uint32_t max_events;        /* cap on holding intervals per walker; 0 = 2^24 */
    void *stream;               /* hipStream_t; NULL = null stream */
    int32_t cond_first_jump;    /* 1: variance reduction by conditioning (a remedy of the
                                   kind Sec. 5 names): every backward walker from a node
                                   with exits is drawn given a jump before t (first
                                   holding time from the exponential law truncated to
                                   [0, t), U in [0,1) from the same 53 bits), and returns
                                   e^{-rt} K + (1 - e^{-rt}) W v[X_t], K the value of a
                                   walker that never leaves; the no-jump event is
                                   integrated exactly, the mean is unchanged.  Backward
                                   estimators only.  Default 0. */
    double cond_max_rt;         /* conditioning applies to start nodes with exits and
                                   r t <= cond_max_rt, decided in FP64 as
                                   t <= cond_max_rt * (1/r); others walk plainly.
                                   Default +inf (every node with exits). */
    uint32_t task_walkers;      /* walkers of consecutive entries packed into one task of
                                   the backward walk kernel, which runs them through its
                                   LDS list in as many passes as their jumping walkers
                                   need; entries with fewer walkers share a task up to
                                   this many (at most 64 entries).  0 (default):
                                   automatic, from 1024 to 8192 walkers aiming at
                                   20480 tasks per run, and no fewer than 5120 tasks
                                   where there are that many entries (for
                                   mc_expmv_entries_multi: chunks of walkers, at most
                                   2048 walkers a task).  A tuning knob only:
                                   estimates do not depend on it, bit for bit. */
    int32_t slot_rows;          /* 1: every alias slot also holds the row records and d of
                                   its two destinations (64-byte slots, 4x the slot
                                   memory), so that a jump is one gather instead of a
                                   slot gather followed by the destination's row; pays
                                   where the tables miss in cache.  -1: separate tables.
                                   0 (default): 1 when rows, d and slots together exceed
                                   64 MiB and the 64-byte slots (64 B per stored entry
                                   of A) fit in 4 GiB.  Estimates do not depend on it,
                                   bit for bit. */
    int32_t qmc_first;          /* 1: randomised quasi-Monte Carlo for the first event of
                                   the backward walks (a variance reduction of the kind
                                   Sec. 5 names): the walker ordinals of an entry form
                                   replicates of B = 1024 (MC_FP32) or 512 (MC_FP64)
                                   consecutive walkers, and walker w's first-event words
                                   are the point j of the Korobov rank-1 lattice
                                   (1, a, a^2 mod B), a = 149 (B = 1024) or 119 (B = 512),
                                   shifted modulo 1 by the Philox draw of the counter
                                   (0xFFFFFFFE, w / B, start node, instance id):
                                   64-bit U word j 2^(64-b) + (o0 2^32 + o1), slot word
                                   j g1 2^(32-b) + o2, alias word j g2 2^(32-b) + o3
                                   (B = 2^b, wrapping; j = the b bits of w mod B
                                   reversed, so the first 2^k walkers of a replicate are
                                   the 2^k-point sub-lattice).  Later events are as
                                   in the plain walk.  Unbiased (every coordinate is a
                                   uniform shift); stderr_ then comes from the R replicate
                                   means, R/(R-1) sum_c (n_c/M)^2 (m_c - est)^2, when an
                                   entry has R >= 2 replicates, else the i.i.d. formula.
                                   Not with cond_first_jump or relabel, and max_events
                                   must stay below 0xFFFFFFFE (MC_ERR_INVALID_ARG
                                   otherwise).
                                   Default 0. */
} mc_expmv_opts;

typedef struct {
    uint64_t walkers;           /* walkers simulated by the last run */
    uint64_t events;            /* holding intervals (= jumps + walkers) */
    uint64_t jumps;
    double ms;                  /* device time of the last run, from HIP events */
    double alg_bytes;           /* algorithmic table/vector bytes of the last run */
} mc_expmv_run_stats;

/* Fill *opts with the defaults listed above. */
void mc_expmv_default_opts(mc_expmv_opts *opts);

/* Human-readable text for a status code (static storage). */
const char *mc_expmv_status_string(mc_status s);

/*
 * Build the walk tables for the n x n matrix A (paper Sec. 2: A = D - L; the
 * row split into r_i, d_i and k_ij is Eq. (paths)).
 *   rowptr  device int64[n+1], rowptr[0] = 0, non-decreasing, rowptr[n] = nnz < 2^32
 *   col     device int32[nnz], 0 <= col < n (any order, duplicates allowed)
 *   val     device double[nnz]; diagonal entries are summed into a_ii, positive
 *           off-diagonal entries become jump slots, zero ones are dropped
 *   t       horizon, finite, >= 0 (the paper's beta)
 *   seed    64-bit Philox key
 *   opts    NULL for defaults
 * Errors: MC_ERR_INVALID_ARG (shape, column index, option), MC_ERR_NONFINITE,
 * MC_ERR_NOT_METZLER (negative off-diagonal).  Column-index and shape errors
 * take precedence over non-finite values, which take precedence over signs.
 * A, once create returns, is no longer referenced.  Synchronous.
 */
mc_status mc_expmv_create(mc_expmv_t *out, int64_t n, int64_t nnz, const int64_t *rowptr,
                          const int32_t *col, const double *val, double t, uint64_t seed,
                          const mc_expmv_opts *opts);

/*
 * A handle for the walk on a 7-point stencil without jump tables (the variable-
 * coefficient diffusion operators of the benchmark's 3-D workload): A is given by
 * its face rates instead of CSR, neighbours come from the node index
 * x = i + nx (j + ny k), and a jump picks the neighbour by inverse CDF over the six
 * face rates in the column
 * order of A's row (-z, -y, -x, +x, +y, +z): the first face whose running sum of
 * rates exceeds u r_x, u = o2 2^-32 from the event's Philox draw (the last face with
 * a rate when rounding leaves u r_x at or above the sum).  r_x is the sum of the
 * face rates in that order, d_x = a_xx + r_x (Sec. 2 split, as for CSR input).
 * The same law as the alias tables of mc_expmv_create, sampled by another rule, so
 * paths differ from a CSR handle's (they match the oracle's inverse-CDF rule).
 *   fx, fy, fz  device double[n], n = nx ny nz: the rate between x and its +x / +y /
 *               +z neighbour (A is symmetric in the stencil's off-diagonals), >= 0,
 *               0 on the last plane of that axis
 *   diag        device double[n]: a_xx
 * Supports entries / entries_multi / full / trace / stats in every weight mode and
 * precision; not the tilted proposal, the forward estimator, relabelling,
 * conditioning or the lattice (MC_ERR_INVALID_ARG).  Errors: MC_ERR_INVALID_ARG
 * (sizes, a positive rate on a last plane, a node whose 1/r_x overflows, options),
 * MC_ERR_NONFINITE, MC_ERR_NOT_METZLER (a negative rate).  The arrays are copied;
 * synchronous.  At create each node's 32-byte state record is built from its faces:
 * 1/r_x, which faces carry a rate, and the rule's thresholds on o2 (for each face
 * with a rate but the last, the largest o2 whose u r_x stays below the running sum
 * up to it), so the walk picks the face by integer comparisons with the same result
 * as the rule.  Device memory per node: that record and d_x in both precisions,
 * 44 B (0.74 GB for 256^3; the faces and a_xx, 32 B per node more, only during
 * create); the CSR form holds 16 B row records, d_x, r_x and a 16 B alias slot per
 * stored entry (2.5 GB for 256^3).
 */
mc_status mc_expmv_create_stencil7(mc_expmv_t *out, int64_t nx, int64_t ny, int64_t nz,
                                   const double *fx, const double *fy, const double *fz,
                                   const double *diag, double t, uint64_t seed,
                                   const mc_expmv_opts *opts);

/*
 * Entries idx[0..k-1] of exp(tA) v, n_walkers walkers each (Algorithm 1 and
 * Theorem 1; sample mean and standard error as in Sec. 5, Eq. (errortotal)).
 *   v        device vector of n values: double (MC_FP64) or float (MC_FP32)
 *   idx      device int64[k]; duplicates give identical estimates
 *   est      device double[k]: mean of W * v[X_t]
 *   stderr_  device double[k] or NULL: sqrt(unbiased sample variance / n_walkers)
 *            (0 when n_walkers = 1)
 * With a proposal installed (mc_expmv_set_proposal) the tilted walk is used.
 * An index outside [0, n) yields NaN in est and MC_ERR_OUT_OF_RANGE at sync.
 */
mc_status mc_expmv_entries(mc_expmv_t h, const void *v, const int64_t *idx, int64_t k,
                           int64_t n_walkers, double *est, double *stderr_);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): exactly
 * mc_expmv_entries (same kernels, same arguments, bitwise the same estimates),
 * but the call allocates nothing.  The (count, mean, M2) partials of entries
 * that span several walker chunks (chunks of 1024 walkers with MC_FP32
 * weights, 512 with MC_FP64) live in a static device array of
 * MC_NOALLOC_SCRATCH_DOUBLES doubles (8 MiB) that each GPU the library runs on
 * holds until the process ends; its address is looked up per device by
 * mc_expmv_create.  A run needs 3 * k * ceil(n_walkers / chunk) doubles when
 * n_walkers exceeds one chunk and none otherwise; larger requests return
 * MC_ERR_TOO_LARGE before anything is enqueued.  Every partial is written
 * before it is read, so nothing needs clearing between calls.  All calls of
 * this function on one GPU share the array: calls that overlap on that GPU
 * (other streams, other handles, other host threads) race, so callers order
 * them (one stream, or events).  The handle itself (tables, counters, status
 * word) is allocated by mc_expmv_create, before.
 */
#define MC_NOALLOC_SCRATCH_DOUBLES (1 << 20)
mc_status mc_expmv_entries_noalloc(mc_expmv_t h, const void *v, const int64_t *idx, int64_t k,
                                   int64_t n_walkers, double *est, double *stderr_);

/*
 * As mc_expmv_entries, with its own walker count for every entry (e.g. the
 * production pass of a two-pass run to a target error, Sec. 5): n_walkers is a
 * HOST int64_t[k] (each in 1 .. 2^32-1); all entries go into one launch.  Entry
 * e's estimate and standard error are bitwise those mc_expmv_entries returns
 * for that entry with n_walkers[e] walkers.
 */
mc_status mc_expmv_entries_multi(mc_expmv_t h, const void *v, const int64_t *idx, int64_t k,
                                 const int64_t *n_walkers, double *est, double *stderr_);

/*
 * Entries to a relative standard error target, both passes on the device (the
 * error model of Sec. 5: the statistical error of M walkers is sigma / sqrt(M)).
 * A pilot of pilot_walkers walkers per entry (ordinals 0 .. pilot-1) gives x_e and
 * sigma_e = se_e sqrt(pilot); entry e then gets
 * N_e = ceil(margin (sigma_e / (target |x_e|))^2) walkers, clamped to
 * [min_walkers, max_walkers] (min_walkers when the pilot saw no spread, max_walkers
 * when x_e = 0 or a value is not finite), walked with the ordinals pilot ..
 * pilot + N_e - 1 (independent of the pilot) in one launch whose task count the
 * device reads, so the host does not wait between the passes.  est, stderr_ are
 * the production run's (entry e's values are those of a run of N_e walkers from
 * ordinal pilot); walkers_out (device int64_t[k], may be NULL) receives N_e.
 *   pilot_walkers  2 .. 2^31 (with opts.qmc_first a multiple of the replicate,
 *                  512 (FP64) or 1024 (FP32), so the production run's replicates
 *                  are whole);  target > 0 finite;  margin >= 1 finite;
 *   2 <= min_walkers <= max_walkers, pilot_walkers + max_walkers <= 2^32
 * Asynchronous on the handle's stream like mc_expmv_entries_multi; device memory
 * for the chunk partials is sized for max_walkers (24 B per chunk of 512 (FP64)
 * or 1024 (FP32) walkers per entry).  Errors: MC_ERR_INVALID_ARG,
 * MC_ERR_NO_MEMORY, and the walk's latched errors at the next mc_expmv_sync.
 */
mc_status mc_expmv_entries_to_target(mc_expmv_t h, const void *v, const int64_t *idx, int64_t k,
                                     int64_t pilot_walkers, double target, double margin,
                                     int64_t min_walkers, int64_t max_walkers, double *est,
                                     double *stderr_, int64_t *walkers_out);

/*
 * Every entry of exp(tA) v with n_per_node walkers started at each node
 * (Algorithm 1 applied at every node; equal to mc_expmv_entries with
 * idx = 0..n-1).  est, stderr_: device double[n] (stderr_ may be NULL).
 */
mc_status mc_expmv_full(mc_expmv_t h, const void *v, int64_t n_per_node, double *est,
                        double *stderr_);

/*
 * The full vector by forward walks (Lemma 2 and Theorem 2, Algorithm 2, with
 * the update credited to the state where each walk ends): n_walkers walkers
 * w = 0 .. M-1 draw their start j with probability |v_j| / V, V = sum_l |v_l|
 * (the first node whose cumulative sum of |v| in node order reaches U V, U
 * from the Philox counter (0, w, 0xFFFFFFFF, instance id)), walk forward with
 * counters (k, w, 0xFFFFFFFF, instance id), k = 1, 2, ..., and contribute
 * Y = V sign(v_j) W to the entry of their state at t.  The STRANG and LIE
 * grid coefficients are read in reverse time order, so every mode estimates
 * the same vector as the backward estimator.  A must be symmetric (checked on
 * the first call of a handle, synchronously; MC_ERR_NOT_SYMMETRIC otherwise):
 * then the forward and backward chains coincide, as the paper notes before
 * Lemma 2.  The tilted proposal, if installed, is not used.
 *   v        device double[n] (float[n] with MC_FP32 weights), any signs
 *   est      device double[n]: (1/M) sum_w Y_w 1{X_t = i}; may be NULL when
 *            sum_out is given (then no per-node work is done)
 *   stderr_  device double[n] or NULL (NULL when est is): sqrt(s_i^2 / M), s_i^2
 *            the sample variance of Y_w 1{X_t = i} over the M walkers
 *   sum_out  device double[2] or NULL: mean of Y (an estimate of sum_i x_i, the
 *            total communicability (1, e^A 1) when t = 1 and v = 1, Eq. (TC))
 *            and its standard error
 * Per-node sums use FP64 atomics: two runs agree to rounding, not bitwise;
 * sum_out is bitwise reproducible.  Device errors as for the other entry points.
 */
mc_status mc_expmv_forward(mc_expmv_t h, const void *v, int64_t n_walkers, double *est,
                           double *stderr_, double *sum_out);

/* Per-walker record of forward walkers w0 .. w0+count-1 (parity checks): start
 * node, end node, holding intervals, jumps and Y, each a device array[count]. */
mc_status mc_expmv_forward_trace(mc_expmv_t h, const void *v, int64_t w0, int64_t count,
                                 int32_t *start, int32_t *end, uint32_t *events, uint32_t *jumps,
                                 double *y);

/*
 * Install a tilted proposal (importance sampling; variance reduction is the
 * remedy the paper names in Sec. 5).  edge_bias: device float[nnz] in CSR order;
 * only positive off-diagonal positions are read.  The walk then jumps with
 * rates a~_ij = a_ij exp(b_ij), uses r~_i = sum_j a~_ij and the weight exponent
 * d~_i = d_i + (r~_i - r_i), and adds -b_ij to the log-weight on every jump
 * over edge ij, so the estimator stays unbiased.  NULL restores the plain walk.
 * MC_EXACT mode only (MC_ERR_INVALID_ARG otherwise).  Synchronous.
 */
mc_status mc_expmv_set_proposal(mc_expmv_t h, const float *edge_bias);

/* Copy the installed proposal's biases (device float[nnz], CSR order) to edge_bias
 * (device float[nnz]); MC_ERR_INVALID_ARG when the plain walk is in use.  Synchronous. */
mc_status mc_expmv_get_proposal(mc_expmv_t h, float *edge_bias);

/* Use `stream` (hipStream_t, NULL = null stream) for the handle's later work; that
 * work is ordered after everything already queued on the previous stream (an event
 * wait, no host synchronisation). */
mc_status mc_expmv_set_stream(mc_expmv_t h, void *stream);

/* Wait for the handle's stream; return (and clear) latched device errors. */
mc_status mc_expmv_sync(mc_expmv_t h);

/* Counters and device time of the last entries/full run (synchronises). */
mc_status mc_expmv_stats(mc_expmv_t h, mc_expmv_run_stats *out);

/*
 * Per-walker record of walkers w0 .. w0+count-1 started at node `start`, from
 * the same kernel that computes estimates: final state X_t, holding intervals,
 * jumps and W * v[X_t] (as double).  All outputs are device arrays of `count`.
 * use_proposal selects the tilted walk.  For parity checks; count <= 2^20.
 */
mc_status mc_expmv_trace(mc_expmv_t h, const void *v, int64_t start, int64_t w0, int64_t count,
                         int32_t use_proposal, int32_t *x_end, uint32_t *events,
                         uint32_t *jumps, double *f);

/*
 * Copy the walk tables to host memory (plain, or tilted when use_proposal),
 * rows in the caller's numbering and slots in CSR order:
 *   r, d, inv_r  host double[n];  deg host int64[n];  begin host int64[n]
 *   (first slot of row i among all slots, i.e. the prefix sum of deg)
 *   col, alias   host int32[nslots];  thr host uint32[nslots]
 * Any pointer may be NULL.  nslots comes from mc_expmv_info.  Synchronous.
 */
mc_status mc_expmv_get_tables(mc_expmv_t h, int32_t use_proposal, double *r, double *d,
                              double *inv_r, int64_t *deg, int64_t *begin, int32_t *col,
                              uint32_t *thr, int32_t *alias);

/*
 * Copy a stencil handle's state records (mc_expmv_create_stencil7) to host memory:
 *   d, inv_r  host double[n]: d_x and 1/r_x (0 for a node without exits)
 *   faces     host uint32[n]: the number k of faces with a rate (bits 0..2) and those
 *             faces in column order, 3 bits each from bit 3 (codes 0..5 for -z, -y,
 *             -x, +x, +y, +z)
 *   thr       host uint32[5 n]: per node, for the j-th face with a rate (j < k) the
 *             largest o2 in [0, 2^32) with (o2 2^-32) r_x below the running sum of
 *             the faces up to it, both products rounded in FP64; 2^32 - 1 from j = k on
 * Any pointer may be NULL.  MC_ERR_INVALID_ARG for a CSR handle.  Synchronous.
 */
mc_status mc_expmv_get_stencil(mc_expmv_t h, double *d, double *inv_r, uint32_t *faces,
                               uint32_t *thr);

/* Sizes of a handle: n, number of jump slots, splitting steps N and dt = t/N. */
mc_status mc_expmv_info(mc_expmv_t h, int64_t *n, int64_t *nslots, int64_t *ngrid, double *dt);

/* Release everything the handle owns (synchronises its stream first). */
void mc_expmv_destroy(mc_expmv_t h);

/* ------------------------------------------------------------------ batches
 * Many instances -- each its own matrix, horizon, weight mode, precision,
 * vector and request (entries or the full vector) -- in one persistent launch
 * replayed from a captured HIP graph.  Each instance's results equal those of
 * a separate handle with the same settings and instance id (Algorithm 1 per
 * instance); the schedule (block size, grid, task grabbing) never changes a
 * result.  The paper runs one matrix at a time (Sec. 6); batching is this
 * library's addition for many small problems.
 */
typedef struct mc_batch_s *mc_batch_t;

typedef struct {
    int64_t n, nnz;
    const int64_t *rowptr;      /* device, as in mc_expmv_create */
    const int32_t *col;         /* device */
    const double *val;          /* device */
    double t;                   /* horizon */
    int32_t mode;               /* MC_EXACT, MC_STRANG or MC_LIE */
    double dt;                  /* splitting step for STRANG / LIE */
    int32_t weight_prec;        /* MC_FP64 or MC_FP32 (then v is float) */
    uint32_t instance_id;       /* fourth Philox counter word */
    const void *v;              /* device vector of n values */
    const int64_t *idx;         /* device int64[k] entries, or NULL for the full vector */
    int64_t k;                  /* number of entries (ignored when idx is NULL) */
    int64_t n_walkers;          /* walkers per entry (per node for the full vector) */
    double *est;                /* device double[k] (or [n]) */
    double *stderr_;            /* device double[k] (or [n]), or NULL */
} mc_instance_desc;

typedef struct {
    uint32_t struct_size;       /* sizeof(mc_batch_opts) */
    uint32_t walkers_per_block; /* 64, 128 or 256; 0 = autotune */
    uint32_t blocks_per_cu;     /* persistent grid = CUs * this (1..128); 0 = autotune */
    uint32_t group;             /* tasks taken per grab from a global counter; 0 = static
                                   stride over the task list */
    int32_t use_graph;          /* 1 (default): capture the launch in a HIP graph */
    uint32_t max_events;        /* walk-length cap per walker; 0 = 2^24 */
    void *stream;               /* caller's hipStream_t, NULL = null stream: runs are
                                   ordered after prior work on it and before later work */
    int32_t slot_rows;          /* as mc_expmv_opts.slot_rows, for every instance */
} mc_batch_opts;

typedef struct {
    uint32_t walkers_per_block, blocks_per_cu, group;
    int64_t tasks;              /* (entry, chunk-of-1024-walkers) tasks per run */
} mc_batch_schedule;

/* Fill *opts with the defaults above. */
void mc_batch_default_opts(mc_batch_opts *opts);

/*
 * Build every instance's tables (as mc_expmv_create), choose the schedule
 * (given in opts, read from the file named by MC_EXPMV_TUNE_CACHE, or timed
 * over a fixed candidate list and then appended to that file) and capture the
 * run in a graph.  All instance buffers (v, idx, est, stderr_) must stay valid
 * until mc_expmv_batch_destroy; A may be freed when this returns.
 * Errors: those of mc_expmv_create for any instance, MC_ERR_INVALID_ARG for
 * n_inst outside 1..1024 or bad options.  Synchronous.
 */
mc_status mc_expmv_batch_create(mc_batch_t *out, int32_t n_inst, const mc_instance_desc *inst,
                                uint64_t seed, const mc_batch_opts *opts);

/* Replay the batch (asynchronous, ordered on the caller's stream). */
mc_status mc_expmv_batch_run(mc_batch_t b);

/* Wait for the batch; return (and clear) latched device errors. */
mc_status mc_expmv_batch_sync(mc_batch_t b);

/* Counters and device time of the last run, and the schedule in use (either may be NULL). */
mc_status mc_expmv_batch_stats(mc_batch_t b, mc_expmv_run_stats *out, mc_batch_schedule *sched);

/* Force a schedule (re-captures the graph).  Results are unchanged by it. */
mc_status mc_expmv_batch_set_schedule(mc_batch_t b, const mc_batch_schedule *sched);

/* Release the batch and every instance's tables. */
void mc_expmv_batch_destroy(mc_batch_t b);

/* ------------------------------------------------------- learned proposal
 * A small network predicts the tilt b_ij of every jump edge for
 * mc_expmv_set_proposal.  Variance reduction is the remedy the paper names for
 * the statistical error (Sec. 5, after Eq. (errortotal)); the tilted walk with
 * its importance weights keeps the estimator unbiased whatever the network
 * predicts, so the plain walk stays both the fallback and the check on bias.
 *
 *   node features  f_i = [log1p deg_i, r_i, v_i, log1p(mean deg of i's jump
 *                  targets)], each standardised over the nodes (population sd)
 *   network        x = [f_i; f_j] -> 64 ReLU -> 64 ReLU -> y, b_ij = 8 tanh(y/8);
 *                  bfloat16 weights, FP32 accumulation, the 64x64 layer on MFMA
 *   training       minimise sum_e p_e (b_e - b*_e)^2 / sum_e p_e over the edges,
 *                  p_e = a_ij / r_i, b*_e = log h_j - log h_i with h = sqrt of the
 *                  per-node second moment of W v[X_t] from plain runs; Adam
 *                  (beta 0.9 / 0.999, eps 1e-8) on FP32 master weights.
 * Parameter vector (kMlpParams = 4801 floats): W1[64][8], b1[64], W2[64][64],
 * b2[64], w3[64], b3.  Gradients are reduced in a fixed order (deterministic).
 */
typedef struct mc_mlp_s *mc_mlp_t;

typedef struct {
    uint32_t struct_size;       /* sizeof(mc_learn_opts) */
    int64_t pilot_walkers;      /* plain walkers per node for the statistics (default 256) */
    int32_t steps;              /* Adam steps (default 400) */
    int64_t batch;              /* edge positions per step (default 65536) */
    float lr;                   /* learning rate (default 3e-3) */
    uint64_t seed;              /* weight initialisation */
    float *params_out;          /* host float[4801] or NULL: receives the trained FP32
                                   parameters, e.g. to install the same network on another
                                   matrix with mc_mlp_set_params and mc_mlp_forward */
} mc_learn_opts;

typedef struct {
    float initial_loss, final_loss;
    int32_t steps;
    double pilot_ms, train_ms;  /* device time: pilot + features, training + inference */
} mc_learn_report;

/* Network with He-uniform initial weights drawn from Philox(seed); work on `stream`. */
mc_status mc_mlp_create(mc_mlp_t *out, uint64_t seed, void *stream);
void mc_mlp_destroy(mc_mlp_t m);
/* Copy the FP32 master parameters to / from host float[4801] (set also resets Adam). */
mc_status mc_mlp_get_params(mc_mlp_t m, float *host);
mc_status mc_mlp_set_params(mc_mlp_t m, const float *host);
/* Standardised node features of handle h's matrix and vector v: device float[n][4]. */
mc_status mc_mlp_features(mc_expmv_t h, const void *v, float *feats);
/* log h_i = 0.5 log(second moment) from a plain run's est/stderr (device double[n])
 * with n_walkers walkers per node: device float[n]. */
mc_status mc_mlp_log_h(mc_expmv_t h, const double *est, const double *stderr_, int64_t n_walkers,
                       float *lh);
/* b for every CSR position (0 off the jump edges): device float[nnz]. */
mc_status mc_mlp_forward(mc_mlp_t m, mc_expmv_t h, const float *feats, float *bias);
/* Gradient (device float[4801]) and loss (device float[1], may be NULL) of the
 * weighted squared error over the jump edges at CSR positions [p0, p1). */
mc_status mc_mlp_gradient(mc_mlp_t m, mc_expmv_t h, const float *feats, const float *lh,
                          int64_t p0, int64_t p1, float *grad, float *loss);
/* One Adam step with gradient `grad` (device float[4801]). */
mc_status mc_mlp_adam_step(mc_mlp_t m, const float *grad, float lr);
/* `steps` Adam steps on batches of `batch` positions spread over the matrix;
 * loss_host (may be NULL): host float[steps].  Synchronous. */
mc_status mc_mlp_train(mc_mlp_t m, mc_expmv_t h, const float *feats, const float *lh,
                       int32_t steps, int64_t batch, float lr, float *loss_host);
void mc_learn_default_opts(mc_learn_opts *opts);
/* Pilot plain run on every node -> targets -> features -> training -> inference
 * -> mc_expmv_set_proposal, all on the GPU.  MC_EXACT handles only.  Synchronous. */
mc_status mc_expmv_learn_proposal(mc_expmv_t h, const void *v, const mc_learn_opts *opts,
                                  mc_learn_report *rep);

/* ---------------------------------------------------------------- rankings */

/*
 * Intersection similarity of the node rankings of two vectors, the measure
 * the paper uses (Sec. 6) to compare a Monte Carlo communicability vector with
 * a reference one:
 *     isim_K(x, y) = (1/K) sum_{i=1..K} |X_i delta Y_i| / (2 i),
 * X_i (Y_i) the i nodes with the largest x (y), delta the symmetric
 * difference; 0 for identical top-K rankings, 1 for disjoint ones.  Ties rank
 * the lower node index first; -0 counts as +0.
 *   n        1 .. 2^31 - 1
 *   x, y     device double[n], finite (MC_ERR_NONFINITE otherwise)
 *   k        1 .. n (the paper reports K = n and K = n/10)
 *   out      host double: the value
 *   stream   hipStream_t or NULL (null stream)
 * Allocates and frees its scratch on every call.  Synchronous.
 * Errors: MC_ERR_INVALID_ARG (null pointer, n or k out of range),
 * MC_ERR_NONFINITE, MC_ERR_NO_MEMORY, MC_ERR_DEVICE.
 */
mc_status mc_isim(int64_t n, const double *x, const double *y, int64_t k, double *out,
                  void *stream);

/* ------------------------------------------------------------- diagnostics */

/*
 * The walk kernels' own FP64 elementary functions on a device array, for
 * checking their accuracy:  fn = MC_FN_LOG: y = log x (the logarithm of the
 * holding time S = -log(U) / r, Eq. (paths); x in (0, 1]), MC_FN_EXP: y = e^x
 * (the FP64 weights W of Theorem 1), MC_FN_ONE_MINUS_EXP_NEG: y = 1 - e^{-x}
 * for x >= 0 (first-jump conditioning), MC_FN_EXP_F32: y = e^x in FP32 for x
 * rounded to FP32 (the FP32 weights; 0 below -104, +inf beyond the range).
 *   x, y     device double[n]
 *   stream   hipStream_t or NULL
 * Errors: MC_ERR_INVALID_ARG (fn, n < 0, null pointer), MC_ERR_DEVICE.
 * Asynchronous on stream.
 */
enum { MC_FN_LOG = 0, MC_FN_EXP = 1, MC_FN_ONE_MINUS_EXP_NEG = 2, MC_FN_EXP_F32 = 3 };
mc_status mc_math_eval(int32_t fn, const double *x, double *y, int64_t n, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* MC_EXPMV_H */
