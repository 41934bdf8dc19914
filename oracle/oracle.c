/*
 * Reference oracle for the Monte Carlo estimator of exp(tA) v
 * (Acebron, "A Monte Carlo method for computing the action of a matrix
 * exponential on a vector", arXiv:1904.12759).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is plain, slow, sequential FP64 C that
 * follows the method step by step.  It shares no code with the HIP library and
 * is used only by the tests, by the smoke check and by the CPU-baseline leg of
 * the benchmark.  Nothing in the product path may call it.
 *
 * What it computes (paper Sec. 2, Lemma 1 / Theorem 1, and Sec. 3, Eq. (paths),
 * Algorithm 1):
 *   A = D - L with L a Laplacian-like matrix: off-diagonal entries of A are the
 *   jump rates of a continuous-time Markov chain with generator Q = -L.  With
 *   our general reading, for row i
 *       r_i   = sum_{j != i} a_ij        (total jump rate, L_ii)
 *       d_i   = a_ii + r_i               (diagonal of D)
 *       k_ij  = a_ij / r_i               (jump law of Eq. (paths))
 *   A walker started at i spends Exp(r_x) holding times in each visited state
 *   x, jumps with law k_x., and stops at the horizon t.  The weight is
 *   exp(integral of d(X_s) ds) evaluated exactly (EXACT, the N -> infinity
 *   limit of the splittings), with the trapezoid rule on the grid k*dt
 *   (STRANG, Eq. (eq_general1) and Theorem 1) or with the right Riemann sum on
 *   the grid (LIE, Eq. (deff)).  The single-entry estimate is the mean over
 *   walkers of weight * v[X_t] (Algorithm 1 with the sample mean taken over the
 *   M walkers, Sec. 5).
 *
 * Conventions fixed where the paper leaves a choice (each is a reading of the
 * paper, the same one the library follows):
 *   - random numbers: Philox4x32-10 (Salmon et al., SC'11), key = seed
 *     (low word first), counter = (event index, walker ordinal, start node,
 *     instance id).  One counter value per holding interval.
 *   - U = (m + 1) * 2^-53 with m = (o0 << 21) | (o1 >> 11), so U in (0, 1];
 *     holding time S = -log(U) / r_x computed as -log(U) * (1/r_x).
 *   - the holding time is drawn in the state it is spent in; a jump happens iff
 *     s + S < t (strict), i.e. the residual holding time at a grid point is
 *     carried over (memorylessness) instead of being redrawn as in the printed
 *     Algorithm 1; the two are equal in law.
 *   - jump target: Vose alias table over the positive off-diagonal entries of
 *     the row (CSR order), slot = floor(o2 * deg / 2^32), "keep the slot's own
 *     column" iff o3 < floor(q * 2^32).  This replaces the row scan of Sec. 4
 *     with an O(1) draw of the same law (up to 2^-32 quantisation).
 *   - grid membership: grid point k belongs to state X(k dt) where the state
 *     entered at time s owns the grid points K(s) <= k < K(next jump), with
 *     K(s) = min(N, ceil(s * (N / t))) evaluated in IEEE FP64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

/* ------------------------------------------------------------------ status */
enum {
    OR_OK = 0,
    OR_ERR_INVALID_ARG = 1,
    OR_ERR_NOT_METZLER = 2,
    OR_ERR_NONFINITE = 3,
    OR_ERR_OUT_OF_RANGE = 4,
    OR_ERR_NO_MEMORY = 6,
    OR_ERR_WALK_LIMIT = 8,
    OR_ERR_OVERFLOW = 9,
};

enum { OR_EXACT = 0, OR_STRANG = 1, OR_LIE = 2 };

/* ---------------------------------------------------------- Philox4x32-10 */
/* Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
 * SC'11: ten rounds of the Philox S-P network with multipliers
 * 0xD2511F53, 0xCD9E8D57 and Weyl key increments 0x9E3779B9, 0xBB67AE85. */
void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 53 random bits from the first two output words. */
static uint64_t bits53(uint32_t o0, uint32_t o1)
{
    return ((uint64_t)o0 << 21) | ((uint64_t)o1 >> 11);
}

/* U in (0,1] and in [0,1) from those bits. */
static double uniform_open0(uint32_t o0, uint32_t o1)
{
    return (double)(bits53(o0, o1) + 1u) * 0x1p-53;
}

static double uniform_open1(uint32_t o0, uint32_t o1)
{
    return (double)bits53(o0, o1) * 0x1p-53;
}

/* ------------------------------------------------------------------ model */
typedef struct {
    /* per row */
    double *a_diag, *r, *d, *inv_r;
    int64_t *deg, *begin;         /* slots of row i: begin[i] .. begin[i]+deg[i]-1 */
    int32_t *uniform;
    /* per slot, in CSR order of the positive off-diagonal entries */
    int32_t *col;
    double *val;
    uint32_t *thr;
    int32_t *alias;
    int32_t *alias_slot;          /* slot (within the row) the alias column comes from */
    double *logcorr;              /* proposal only: -b of the slot's own edge */
} table_set;

typedef struct {
    int64_t n, nnz, nslots;
    double t;
    uint64_t seed;
    int mode;
    int64_t ngrid;                /* N, number of splitting steps */
    double dt;                    /* t / N */
    double inv_dt;                /* N / t */
    uint32_t instance;
    uint32_t max_events;
    table_set plain;
    int has_proposal;
    table_set prop;
    int cond;                     /* condition backward walks on a first jump before t */
    double cond_max_rt;           /* ... from start nodes with t <= cond_max_rt / r */
    int cdf_jump;                 /* jump by inverse CDF over the row instead of the alias table */
    int qmc;                      /* randomised lattice for the first event (see below) */
    int qmc_bits;                 /* replicate size B = 2^qmc_bits walkers */
    int64_t *slot_of_csr;         /* CSR position -> slot index, -1 if none */
} oracle_t;

static void free_tables(table_set *ts)
{
    free(ts->a_diag); free(ts->r); free(ts->d); free(ts->inv_r);
    free(ts->deg); free(ts->begin); free(ts->uniform);
    free(ts->col); free(ts->val); free(ts->thr); free(ts->alias); free(ts->alias_slot);
    free(ts->logcorr);
    memset(ts, 0, sizeof(*ts));
}

void oracle_destroy(oracle_t *o)
{
    if (!o) return;
    free_tables(&o->plain);
    free_tables(&o->prop);
    free(o->slot_of_csr);
    free(o);
}

/* Vose's alias method (M. D. Vose, IEEE TSE 17(9), 1991) for one row.
 * q[s] = p_s * deg are the scaled probabilities; the two work lists are
 * LIFO stacks filled by scanning s = 0 .. deg-1.  Output: per slot the
 * integer threshold floor(q * 2^32) of keeping the slot's own column and the
 * alias column; slots whose final q is >= 1 alias to themselves. */
static int vose_row(int64_t deg, double *q, const int32_t *col, uint32_t *thr, int32_t *alias,
                    int32_t *alias_slot_out)
{
    int64_t *small = (int64_t *)malloc(sizeof(int64_t) * (size_t)deg);
    int64_t *large = (int64_t *)malloc(sizeof(int64_t) * (size_t)deg);
    if (!small || !large) { free(small); free(large); return OR_ERR_NO_MEMORY; }
    int64_t ns = 0, nl = 0;
    int32_t *alias_slot = (int32_t *)malloc(sizeof(int32_t) * (size_t)deg);
    if (!alias_slot) { free(small); free(large); return OR_ERR_NO_MEMORY; }
    for (int64_t s = 0; s < deg; ++s) {
        alias_slot[s] = (int32_t)s;
        if (q[s] < 1.0) small[ns++] = s; else large[nl++] = s;
    }
    double *prob = (double *)malloc(sizeof(double) * (size_t)deg);
    if (!prob) { free(small); free(large); free(alias_slot); return OR_ERR_NO_MEMORY; }
    for (int64_t s = 0; s < deg; ++s) prob[s] = 1.0;
    while (ns > 0 && nl > 0) {
        int64_t l = small[--ns];
        int64_t g = large[--nl];
        prob[l] = q[l];
        alias_slot[l] = (int32_t)g;
        q[g] = (q[g] + q[l]) - 1.0;
        if (q[g] < 1.0) small[ns++] = g; else large[nl++] = g;
    }
    /* whatever is left (large, or small through rounding) keeps itself */
    for (int64_t s = 0; s < deg; ++s) {
        if (prob[s] >= 1.0 || alias_slot[s] == (int32_t)s) {
            thr[s] = 0xFFFFFFFFu;
            alias[s] = col[s];
            alias_slot_out[s] = (int32_t)s;
        } else {
            thr[s] = (uint32_t)(prob[s] * 4294967296.0);   /* floor, prob in [0,1) */
            alias[s] = col[alias_slot[s]];
            alias_slot_out[s] = alias_slot[s];
        }
    }
    free(small); free(large); free(alias_slot); free(prob);
    return OR_OK;
}

/* Split every row into diagonal, jump rate and jump law (paper Sec. 2 and
 * Eq. (paths)); build the alias tables.  If bias is non-NULL the jump rates
 * are tilted: a~_ij = a_ij * exp(b_ij), r~_i = sum a~_ij, d~_i = d_i + (r~_i - r_i)
 * and every jump over edge ij carries the log-weight correction -b_ij. */
static int build_tables(const oracle_t *o, const int64_t *rowptr, const int32_t *colv,
                        const double *valv, const float *bias, const table_set *base,
                        table_set *ts)
{
    int64_t n = o->n, ns = o->nslots;
    ts->a_diag = (double *)calloc((size_t)n, sizeof(double));
    ts->r = (double *)calloc((size_t)n, sizeof(double));
    ts->d = (double *)calloc((size_t)n, sizeof(double));
    ts->inv_r = (double *)calloc((size_t)n, sizeof(double));
    ts->deg = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    ts->begin = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    ts->uniform = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    ts->col = (int32_t *)calloc((size_t)(ns > 0 ? ns : 1), sizeof(int32_t));
    ts->val = (double *)calloc((size_t)(ns > 0 ? ns : 1), sizeof(double));
    ts->thr = (uint32_t *)calloc((size_t)(ns > 0 ? ns : 1), sizeof(uint32_t));
    ts->alias = (int32_t *)calloc((size_t)(ns > 0 ? ns : 1), sizeof(int32_t));
    ts->alias_slot = (int32_t *)calloc((size_t)(ns > 0 ? ns : 1), sizeof(int32_t));
    ts->logcorr = (double *)calloc((size_t)(ns > 0 ? ns : 1), sizeof(double));
    if (!ts->a_diag || !ts->r || !ts->d || !ts->inv_r || !ts->deg || !ts->begin ||
        !ts->uniform || !ts->col || !ts->val || !ts->thr || !ts->alias || !ts->alias_slot ||
        !ts->logcorr)
        return OR_ERR_NO_MEMORY;

    int64_t slot = 0;
    for (int64_t i = 0; i < n; ++i) {
        double diag = 0.0, rate = 0.0;
        int64_t deg = 0;
        ts->begin[i] = slot;
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            int32_t j = colv[p];
            double a = valv[p];
            if (j == i) {
                diag = diag + a;
            } else if (a > 0.0) {
                double at = a;
                if (bias) {
                    at = a * exp((double)bias[p]);
                    if (!isfinite(at) || !(at > 0.0)) return OR_ERR_NONFINITE;
                    ts->logcorr[slot] = -(double)bias[p];
                }
                ts->col[slot] = j;
                ts->val[slot] = at;
                rate = rate + at;
                ++slot; ++deg;
            }
        }
        ts->a_diag[i] = diag;
        ts->r[i] = rate;
        ts->deg[i] = deg;
        if (base) {
            /* tilted weight exponent d~ = d + (r~ - r); exactly d when r~ == r */
            ts->d[i] = base->d[i] + (rate - base->r[i]);
        } else {
            ts->d[i] = diag + rate;
        }
        if (deg > 0) {
            ts->inv_r[i] = 1.0 / rate;
            if (!isfinite(ts->inv_r[i])) return OR_ERR_INVALID_ARG;
        } else {
            ts->inv_r[i] = 0.0;
        }
        if (!isfinite(ts->d[i])) return OR_ERR_NONFINITE;
        /* alias table */
        if (deg > 0) {
            int64_t b = ts->begin[i];
            int uni = 1;
            for (int64_t s = 1; s < deg; ++s)
                if (ts->val[b + s] != ts->val[b]) { uni = 0; break; }
            ts->uniform[i] = uni;
            if (uni) {
                for (int64_t s = 0; s < deg; ++s) {
                    ts->thr[b + s] = 0xFFFFFFFFu;
                    ts->alias[b + s] = ts->col[b + s];
                    ts->alias_slot[b + s] = (int32_t)s;
                }
            } else {
                double *q = (double *)malloc(sizeof(double) * (size_t)deg);
                if (!q) return OR_ERR_NO_MEMORY;
                for (int64_t s = 0; s < deg; ++s)
                    q[s] = (ts->val[b + s] * (double)deg) / rate;
                int st = vose_row(deg, q, ts->col + b, ts->thr + b, ts->alias + b,
                                  ts->alias_slot + b);
                free(q);
                if (st != OR_OK) return st;
            }
        }
    }
    return OR_OK;
}

/* Validate the CSR matrix: shape, column range, finiteness and the sign of the
 * off-diagonal entries (they are jump rates, so they must be >= 0). */
static int validate(int64_t n, int64_t nnz, const int64_t *rowptr, const int32_t *col,
                    const double *val, double t)
{
    if (n < 0 || nnz < 0) return OR_ERR_INVALID_ARG;
    if (!(t >= 0.0) || !isfinite(t)) return OR_ERR_INVALID_ARG;
    if (n == 0) return OR_OK;
    if (!rowptr || rowptr[0] != 0 || rowptr[n] != nnz) return OR_ERR_INVALID_ARG;
    if (nnz > 0 && (!col || !val)) return OR_ERR_INVALID_ARG;
    if (nnz >= ((int64_t)1 << 32)) return OR_ERR_INVALID_ARG;
    for (int64_t i = 0; i < n; ++i)
        if (rowptr[i + 1] < rowptr[i]) return OR_ERR_INVALID_ARG;
    /* precedence: column index > non-finite value > negative off-diagonal */
    int bad_col = 0, bad_val = 0, bad_sign = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            if (col[p] < 0 || col[p] >= n) bad_col = 1;
            else if (!isfinite(val[p])) bad_val = 1;
            else if (col[p] != i && val[p] < 0.0) bad_sign = 1;
        }
    }
    if (bad_col) return OR_ERR_INVALID_ARG;
    if (bad_val) return OR_ERR_NONFINITE;
    if (bad_sign) return OR_ERR_NOT_METZLER;
    return OR_OK;
}

/* Create the oracle for matrix A (CSR, host arrays), horizon t and seed. */
int oracle_create(oracle_t **out, int64_t n, int64_t nnz, const int64_t *rowptr,
                  const int32_t *col, const double *val, double t, uint64_t seed, int mode,
                  double dt_req, uint32_t instance, uint32_t max_events)
{
    *out = NULL;
    int st = validate(n, nnz, rowptr, col, val, t);
    if (st != OR_OK) return st;
    if (mode != OR_EXACT && mode != OR_STRANG && mode != OR_LIE) return OR_ERR_INVALID_ARG;
    oracle_t *o = (oracle_t *)calloc(1, sizeof(oracle_t));
    if (o) o->qmc_bits = 9;
    if (!o) return OR_ERR_NO_MEMORY;
    o->n = n; o->nnz = nnz; o->t = t; o->seed = seed; o->mode = mode;
    o->instance = instance;
    o->max_events = max_events ? max_events : (1u << 24);
    o->ngrid = 1;
    if (mode != OR_EXACT) {
        if (!(dt_req > 0.0) || !isfinite(dt_req)) { free(o); return OR_ERR_INVALID_ARG; }
        double steps = ceil(t / dt_req);
        if (steps > 2147483647.0) { free(o); return OR_ERR_INVALID_ARG; }
        o->ngrid = steps < 1.0 ? 1 : (int64_t)steps;
    }
    o->dt = t / (double)o->ngrid;
    o->inv_dt = (double)o->ngrid / t;
    int64_t ns = 0;
    o->slot_of_csr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nnz > 0 ? nnz : 1));
    if (!o->slot_of_csr) { free(o); return OR_ERR_NO_MEMORY; }
    for (int64_t i = 0; i < n; ++i)
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            if (col[p] != i && val[p] > 0.0) o->slot_of_csr[p] = ns++;
            else o->slot_of_csr[p] = -1;
        }
    o->nslots = ns;
    st = build_tables(o, rowptr, col, val, NULL, NULL, &o->plain);
    if (st != OR_OK) { oracle_destroy(o); return st; }
    *out = o;
    return OR_OK;
}

/* Install (bias != NULL) or remove (bias == NULL) the tilted proposal.  The
 * bias array has one entry per CSR position; only positive off-diagonal
 * positions are read. */
int oracle_set_proposal(oracle_t *o, const int64_t *rowptr, const int32_t *col,
                        const double *val, const float *bias)
{
    free_tables(&o->prop);
    o->has_proposal = 0;
    if (!bias) return OR_OK;
    for (int64_t p = 0; p < o->nnz; ++p)
        if (o->slot_of_csr[p] >= 0 && !isfinite(bias[p])) return OR_ERR_NONFINITE;
    int st = build_tables(o, rowptr, col, val, bias, &o->plain, &o->prop);
    if (st != OR_OK) { free_tables(&o->prop); return st; }
    o->has_proposal = 1;
    return OR_OK;
}

/* ------------------------------------------------------------------- walk */
typedef struct {
    double f;          /* weight * v[X_t] */
    double logw;       /* log of the weight */
    int32_t x_end;     /* X_t */
    uint32_t events;   /* holding intervals = jumps + 1 */
    uint32_t jumps;
    int status;
} walk_out;

/* Grid index of time s: K(s) = min(N, ceil(s * N / t)). */
static int64_t grid_index(const oracle_t *o, double s)
{
    double g = ceil(s * o->inv_dt);
    if (g >= (double)o->ngrid) return o->ngrid;
    return (int64_t)g;
}

/* Trapezoid (STRANG) or right-Riemann (LIE) coefficient of grid point k. */
static double grid_coef(const oracle_t *o, int64_t k)
{
    if (o->mode == OR_STRANG) return (k == 0 || k == o->ngrid) ? 0.5 : 1.0;
    return k == 0 ? 0.0 : 1.0;
}

/* Philox counter word that marks a forward walk in place of the start node. */
#define FORWARD_MARK 0xFFFFFFFFu

/* Randomised quasi-Monte Carlo for the first event (a variance reduction of the
 * kind Sec. 5 names).  The walkers w of one start node form replicates of
 * B = 2^b consecutive ordinals: replicate c = w >> b, and within it the walker
 * w mod B takes point j = the b bits of w mod B reversed (radical-inverse order,
 * so that the first 2^k walkers of a replicate are the 2^k-point sub-lattice and
 * a replicate cut short stays stratified).  The first event of walker w takes its
 * three random words from the point j of the
 * rank-1 lattice with generating vector (1, g1, g2) (Korobov: g1 = a,
 * g2 = a^2 mod B, a = 119 for B = 512 and a = 149 for B = 1024, the values
 * minimising the lattice criterion P_2 over odd a), shifted modulo 1 by a
 * replicate's own random shift: with (r0, r1, r2, r3) = Philox4x32-10 of the
 * counter (0xFFFFFFFE, c, start, instance),
 *     64-bit word of U:   j * 2^(64-b) + (r0 * 2^32 + r1)   mod 2^64
 *     slot word:          j * g1 * 2^(32-b) + r2           mod 2^32
 *     alias word:         j * g2 * 2^(32-b) + r3           mod 2^32.
 * Each coordinate is uniform on its range (a uniform shift modulo 1), so every
 * walker has the law of the plain walk and the mean is unbiased; within a
 * replicate the B points are evenly spread (stratified jump/no-jump choice,
 * holding time and first jump), which reduces the variance of the mean.  Later
 * events draw Philox as in the plain walk.  The standard error comes from the R
 * replicate means m_c (counts n_c of M walkers): se^2 = R/(R-1) sum_c (n_c/M)^2
 * (m_c - mean)^2 when R >= 2, the i.i.d. formula otherwise. */
#define QMC_SHIFT_MARK 0xFFFFFFFEu

/* The b low bits of j in reverse order. */
static uint64_t radical_index(uint32_t j, uint32_t b)
{
    uint64_t r = 0;
    for (uint32_t i = 0; i < b; ++i)
        r |= (uint64_t)((j >> i) & 1u) << (b - 1 - i);
    return r;
}

static void qmc_first_words(const oracle_t *o, int64_t start, uint32_t w, const uint32_t key[2],
                            uint32_t rnd[4])
{
    const uint32_t b = (uint32_t)o->qmc_bits;
    const uint64_t g1 = b == 9 ? 119u : 149u;
    const uint64_t g2 = (g1 * g1) % (1u << b);
    const uint64_t j = radical_index(w & ((1u << b) - 1u), b);
    uint32_t ctr[4] = { QMC_SHIFT_MARK, w >> b, (uint32_t)start, o->instance };
    uint32_t sh[4];
    oracle_philox4x32_10(ctr, key, sh);
    const uint64_t u0 = (j << (64 - b)) + (((uint64_t)sh[0] << 32) | sh[1]);
    rnd[0] = (uint32_t)(u0 >> 32);
    rnd[1] = (uint32_t)u0;
    rnd[2] = (uint32_t)(((j * g1) << (32 - b)) + sh[2]);
    rnd[3] = (uint32_t)(((j * g2) << (32 - b)) + sh[3]);
}

/* One walker started at node `start`, ordinal w.  The path is recorded as
 * the sequence of visited states and entry times, then the weight is formed
 * from the recorded path.  Backward walks (Algorithm 1) use the counters
 * (k, w, start, instance), k = 0, 1, ...; forward walks (Algorithm 2) use
 * (k, w, FORWARD_MARK, instance), k = 1, 2, ... (k = 0 drew the start) and
 * read the grid coefficients in reverse time order, c_{N-k}. */
/* With cond set (backward walks only), the first holding time is drawn
 * conditioned on a jump before t: with q = 1 - e^{-r t}, S = -log(1 - U q) / r
 * for U in [0,1) (the inverse of the exponential law truncated to [0, t)), and
 * the walker jumps whatever S.  The value returned is then
 *     e^{-r t} K + q W v[X_t],
 * K the value of a walker that never leaves the start node: the no-jump event,
 * of probability e^{-r t}, is integrated exactly and only the jump event is
 * sampled, so the mean is unchanged and the variance of the start node's
 * jump/no-jump choice is removed.  It applies to start nodes with exits and
 * r t <= cond_max_rt (decided as t <= cond_max_rt * (1/r), the stored 1/r). */
static void walk_path(const oracle_t *o, int64_t start, uint32_t w, const double *v,
                      int use_prop, int forward, int64_t *path_x, double *path_s,
                      double *path_c, walk_out *res)
{
    const table_set *ts = use_prop ? &o->prop : &o->plain;
    const int cond = o->cond && !forward && ts->deg[start] > 0 &&
                     o->t <= o->cond_max_rt * ts->inv_r[start];
    uint32_t key[2] = { (uint32_t)o->seed, (uint32_t)(o->seed >> 32) };
    int64_t x = start;
    double s = 0.0;
    uint32_t events = 0, jumps = 0;
    int64_t len = 0;
    path_x[0] = x; path_s[0] = 0.0; path_c[0] = 0.0;
    res->status = OR_OK;
    for (;;) {
        if (ts->deg[x] == 0) { ++events; break; }         /* rate 0: stays until t */
        if (events >= o->max_events) { res->status = OR_ERR_WALK_LIMIT; break; }
        uint32_t ctr[4] = { forward ? events + 1u : events, w,
                            forward ? FORWARD_MARK : (uint32_t)start, o->instance };
        uint32_t rnd[4];
        if (o->qmc && !forward && events == 0)
            qmc_first_words(o, start, w, key, rnd);
        else
            oracle_philox4x32_10(ctr, key, rnd);
        ++events;
        double S;
        int jump;
        if (cond && events == 1) {
            double q = -expm1(-ts->r[x] * o->t);
            S = -log(1.0 - uniform_open1(rnd[0], rnd[1]) * q) * ts->inv_r[x];
            jump = 1;
        } else {
            S = -log(uniform_open0(rnd[0], rnd[1])) * ts->inv_r[x];
            jump = s + S < o->t;
        }
        if (jump && o->cdf_jump) {
            /* inverse CDF of the jump law over the row's rates in CSR order: the first
             * slot whose running sum exceeds u r, u = o2 2^-32 in [0, 1) (the last slot
             * when rounding leaves u r at or above the sum) */
            s = s + S;
            const double target = ((double)rnd[2] * 0x1p-32) * ts->r[x];
            const int64_t b = ts->begin[x];
            int64_t sl = ts->deg[x] - 1;
            double cum = 0.0;
            for (int64_t k = 0; k < ts->deg[x]; ++k) {
                cum = cum + ts->val[b + k];
                if (target < cum) { sl = k; break; }
            }
            x = ts->col[b + sl];
            ++jumps;
            ++len;
            path_x[len] = x; path_s[len] = s; path_c[len] = use_prop ? ts->logcorr[b + sl] : 0.0;
        } else if (jump) {
            s = s + S;
            int64_t slot = (int64_t)(((uint64_t)rnd[2] * (uint64_t)ts->deg[x]) >> 32);
            int64_t q = ts->begin[x] + slot;
            int64_t y;
            double corr;
            if (rnd[3] < ts->thr[q]) {
                y = ts->col[q];
                corr = ts->logcorr[q];
            } else {
                y = ts->alias[q];
                corr = ts->logcorr[ts->begin[x] + ts->alias_slot[q]];
            }
            x = y;
            ++jumps;
            ++len;
            path_x[len] = x; path_s[len] = s; path_c[len] = use_prop ? corr : 0.0;
        } else {
            break;
        }
    }
    /* weight from the recorded path */
    double logw = 0.0;
    if (o->mode == OR_EXACT) {
        for (int64_t m = 0; m <= len; ++m) {
            double sb = (m < len) ? path_s[m + 1] : o->t;
            double held = (m < len) ? (sb - path_s[m]) : (o->t - path_s[m]);
            logw += ts->d[path_x[m]] * held;
            logw += path_c[m];
        }
    } else if (o->t > 0.0) {
        /* state at grid point k: the last recorded state entered with K(s) <= k */
        double acc = 0.0;
        int64_t m = 0;
        for (int64_t k = 0; k <= o->ngrid; ++k) {
            while (m < len && grid_index(o, path_s[m + 1]) <= k) ++m;
            acc += grid_coef(o, forward ? o->ngrid - k : k) * ts->d[path_x[m]];
        }
        logw = acc * o->dt;
    }
    res->logw = logw;
    res->f = exp(logw) * v[x];
    if (cond) {
        /* no-jump value K of the start node (its weight over the whole horizon) */
        double logk = 0.0;
        if (o->mode == OR_EXACT) {
            logk = ts->d[start] * o->t;
        } else if (o->t > 0.0) {
            double acc = 0.0;
            for (int64_t k = 0; k <= o->ngrid; ++k) acc += grid_coef(o, k) * ts->d[start];
            logk = acc * o->dt;
        }
        double rt = ts->r[start] * o->t;
        res->f = exp(-rt) * (exp(logk) * v[start]) + (-expm1(-rt)) * res->f;
    }
    if (!isfinite(res->f) && res->status == OR_OK) res->status = OR_ERR_OVERFLOW;
    res->x_end = (int32_t)x;
    res->events = events;
    res->jumps = jumps;
}

static void walk_one(const oracle_t *o, int64_t start, uint32_t w, const double *v,
                     int use_prop, int64_t *path_x, double *path_s, double *path_c,
                     walk_out *res)
{
    walk_path(o, start, w, v, use_prop, 0, path_x, path_s, path_c, res);
}

/* Per-walker trace for parity checks: walkers w0 .. w0+count-1 from `start`. */
int oracle_trace(const oracle_t *o, const double *v, int64_t start, uint32_t w0, int64_t count,
                 int use_prop, int32_t *x_end, uint32_t *events, uint32_t *jumps, double *f,
                 double *logw)
{
    if (start < 0 || start >= o->n) return OR_ERR_OUT_OF_RANGE;
    if (use_prop && !o->has_proposal) return OR_ERR_INVALID_ARG;
    size_t cap = (size_t)o->max_events + 2;
    int64_t *px = (int64_t *)malloc(sizeof(int64_t) * cap);
    double *ps = (double *)malloc(sizeof(double) * cap);
    double *pc = (double *)malloc(sizeof(double) * cap);
    if (!px || !ps || !pc) { free(px); free(ps); free(pc); return OR_ERR_NO_MEMORY; }
    int st = OR_OK;
    for (int64_t c = 0; c < count; ++c) {
        walk_out r;
        walk_one(o, start, w0 + (uint32_t)c, v, use_prop, px, ps, pc, &r);
        x_end[c] = r.x_end; events[c] = r.events; jumps[c] = r.jumps; f[c] = r.f; logw[c] = r.logw;
        if (r.status != OR_OK && st == OR_OK) st = r.status;
    }
    free(px); free(ps); free(pc);
    return st;
}

/* ------------------------------------------------------------- estimator */
/* Neumaier's compensated sum. */
static double neumaier_sum(const double *x, int64_t m)
{
    double s = 0.0, c = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        double t = s + x[i];
        if (fabs(s) >= fabs(x[i])) c += (s - t) + x[i];
        else c += (x[i] - t) + s;
        s = t;
    }
    return s + c;
}

typedef struct {
    const oracle_t *o;
    const double *v;
    const int64_t *idx;       /* NULL: entry e is node e */
    int64_t k, nwalk;
    int use_prop;
    double *est, *se;
    uint64_t *events, *jumps; /* per entry */
    int nthreads, tid;
    int status;
} job_t;

static void *run_job(void *arg)
{
    job_t *jb = (job_t *)arg;
    const oracle_t *o = jb->o;
    size_t cap = (size_t)o->max_events + 2;
    int64_t *px = (int64_t *)malloc(sizeof(int64_t) * cap);
    double *ps = (double *)malloc(sizeof(double) * cap);
    double *pc = (double *)malloc(sizeof(double) * cap);
    double *fs = (double *)malloc(sizeof(double) * (size_t)jb->nwalk);
    double *dev = (double *)malloc(sizeof(double) * (size_t)jb->nwalk);
    if (!px || !ps || !pc || !fs || !dev) { jb->status = OR_ERR_NO_MEMORY; goto done; }
    for (int64_t e = jb->tid; e < jb->k; e += jb->nthreads) {
        int64_t i = jb->idx ? jb->idx[e] : e;
        if (i < 0 || i >= o->n) {
            jb->est[e] = NAN; if (jb->se) jb->se[e] = NAN;
            if (jb->status == OR_OK) jb->status = OR_ERR_OUT_OF_RANGE;
            continue;
        }
        uint64_t ev = 0, ju = 0;
        for (int64_t w = 0; w < jb->nwalk; ++w) {
            walk_out r;
            walk_one(o, i, (uint32_t)w, jb->v, jb->use_prop, px, ps, pc, &r);
            if (r.status != OR_OK && jb->status == OR_OK) jb->status = r.status;
            fs[w] = r.f;
            ev += r.events; ju += r.jumps;
        }
        double mean = neumaier_sum(fs, jb->nwalk) / (double)jb->nwalk;
        jb->est[e] = mean;
        const int64_t B = (int64_t)1 << o->qmc_bits;
        if (jb->se && o->qmc && jb->nwalk > B) {
            /* replicate means */
            const int64_t R = (jb->nwalk + B - 1) / B;
            double acc = 0.0;
            for (int64_t c = 0; c < R; ++c) {
                const int64_t w0 = c * B;
                const int64_t nc = jb->nwalk - w0 < B ? jb->nwalk - w0 : B;
                const double mc = neumaier_sum(fs + w0, nc) / (double)nc;
                const double wc = (double)nc / (double)jb->nwalk;
                acc += wc * wc * (mc - mean) * (mc - mean);
            }
            jb->se[e] = sqrt(acc * (double)R / (double)(R - 1));
        } else if (jb->se) {
            if (jb->nwalk > 1) {
                for (int64_t w = 0; w < jb->nwalk; ++w) dev[w] = (fs[w] - mean) * (fs[w] - mean);
                double var = neumaier_sum(dev, jb->nwalk) / (double)(jb->nwalk - 1);
                jb->se[e] = sqrt(var / (double)jb->nwalk);
            } else {
                jb->se[e] = 0.0;
            }
        }
        if (jb->events) jb->events[e] = ev;
        if (jb->jumps) jb->jumps[e] = ju;
    }
done:
    free(px); free(ps); free(pc); free(fs); free(dev);
    return NULL;
}

/* Estimate entries idx[0..k-1] (or every node when idx == NULL) of exp(tA)v
 * with nwalk walkers each.  The result does not depend on nthreads: every
 * entry is summed by one thread in walker-ordinal order. */
int oracle_estimate(const oracle_t *o, const double *v, const int64_t *idx, int64_t k,
                    int64_t nwalk, int use_prop, int nthreads, double *est, double *se,
                    uint64_t *events, uint64_t *jumps)
{
    if (nwalk <= 0 || nwalk > 0xFFFFFFFFll) return OR_ERR_INVALID_ARG;
    if (use_prop && !o->has_proposal) return OR_ERR_INVALID_ARG;
    if (nthreads < 1) nthreads = 1;
    job_t *jobs = (job_t *)calloc((size_t)nthreads, sizeof(job_t));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!jobs || !th) { free(jobs); free(th); return OR_ERR_NO_MEMORY; }
    for (int tI = 0; tI < nthreads; ++tI) {
        jobs[tI] = (job_t){ o, v, idx, k, nwalk, use_prop, est, se, events, jumps,
                            nthreads, tI, OR_OK };
    }
    if (nthreads == 1) {
        run_job(&jobs[0]);
    } else {
        for (int tI = 0; tI < nthreads; ++tI) pthread_create(&th[tI], NULL, run_job, &jobs[tI]);
        for (int tI = 0; tI < nthreads; ++tI) pthread_join(th[tI], NULL);
    }
    int st = OR_OK;
    for (int tI = 0; tI < nthreads; ++tI)
        if (jobs[tI].status != OR_OK && st == OR_OK) st = jobs[tI].status;
    free(jobs); free(th);
    return st;
}

/* Jump rule: 0 = Vose alias table (default), 1 = inverse CDF over the row's rates
 * in CSR order (the rule of the matrix-free stencil walk). */
int oracle_set_jump_rule(oracle_t *o, int rule)
{
    if (rule != 0 && rule != 1) return OR_ERR_INVALID_ARG;
    o->cdf_jump = rule;
    return OR_OK;
}

/* Switch the randomised lattice of the first event on or off (bits = 9 or 10:
 * replicates of 512 or 1024 walkers). */
int oracle_set_qmc(oracle_t *o, int on, int bits)
{
    if (on && bits != 9 && bits != 10) return OR_ERR_INVALID_ARG;
    if (on && o->max_events >= QMC_SHIFT_MARK) return OR_ERR_INVALID_ARG;
    o->qmc = on ? 1 : 0;
    o->qmc_bits = on ? bits : 9;
    return OR_OK;
}

/* Switch the first-jump conditioning of backward walks on or off; it applies
 * to start nodes with exits and r t <= max_rt, decided as t <= max_rt (1/r). */
int oracle_set_conditioning(oracle_t *o, int on, double max_rt)
{
    o->cond = on ? 1 : 0;
    o->cond_max_rt = max_rt;
    return OR_OK;
}

/* ---------------------------------------------------- forward estimator */
/* Full vector by forward walks (Lemma 2 and Theorem 2; Algorithm 2 with its
 * update applied to the state where the walk ends).  Walker w (w = 0..M-1)
 * draws its start j with probability |v_j| / V, V = sum_l |v_l|: with U from
 * the counter (0, w, FORWARD_MARK, instance), j is the first node whose
 * cumulative sum |v_0| + ... + |v_j| (taken in node order) reaches U V.  It
 * then walks forward for time t and contributes Y = V sign(v_j) W to the entry
 * of its end state X_t (the indicator of the terminal state in Theorem 2).
 * E[Y 1{X_t = i}] = sum_j v_j (e^{tA})_{ji} = (e^{tA^T} v)_i, which is
 * (e^{tA} v)_i for the symmetric A of the paper.  For v >= 0 this is Lemma 2's
 * sampling; a sign carries negative entries.
 * Outputs: est_i = (1/M) sum_w Y_w 1{end_w = i}; se_i = sqrt(s_i^2 / M) with s_i^2
 * the sample variance of Y_w 1{end_w = i} over the M walkers; *sum, *sum_se =
 * mean and standard error of Y (an estimate of sum_i x_i).  Per-walker
 * arrays (nullable): start, end state, events, jumps, Y. */
int oracle_forward(const oracle_t *o, const double *v, int64_t nwalk, int use_prop,
                   double *est, double *se, double *sum, double *sum_se,
                   int32_t *w_start, int32_t *w_end, uint32_t *w_events, uint32_t *w_jumps,
                   double *w_y)
{
    if (nwalk <= 0 || nwalk > 0xFFFFFFFFll) return OR_ERR_INVALID_ARG;
    if (use_prop) return OR_ERR_INVALID_ARG;
    int64_t n = o->n;
    double *cdf = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *s1 = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    double *c1 = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    double *s2 = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    double *c2 = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    double *ys = (double *)malloc(sizeof(double) * (size_t)nwalk);
    size_t cap = (size_t)o->max_events + 2;
    int64_t *px = (int64_t *)malloc(sizeof(int64_t) * cap);
    double *ps = (double *)malloc(sizeof(double) * cap);
    double *pc = (double *)malloc(sizeof(double) * cap);
    int st = OR_OK;
    if (!cdf || !s1 || !c1 || !s2 || !c2 || !ys || !px || !ps || !pc) { st = OR_ERR_NO_MEMORY; goto out; }
    double V = 0.0;
    for (int64_t j = 0; j < n; ++j) { V = V + fabs(v[j]); cdf[j] = V; }
    uint32_t key[2] = { (uint32_t)o->seed, (uint32_t)(o->seed >> 32) };
    for (int64_t w = 0; w < nwalk; ++w) {
        double y = 0.0;
        int32_t j = -1, x_end = -1;
        walk_out r = { 0.0, 0.0, -1, 0, 0, OR_OK };
        if (V > 0.0) {
            uint32_t ctr[4] = { 0u, (uint32_t)w, FORWARD_MARK, o->instance };
            uint32_t rnd[4];
            oracle_philox4x32_10(ctr, key, rnd);
            double target = uniform_open0(rnd[0], rnd[1]) * V;
            int64_t lo = 0, hi = n - 1;             /* first j with cdf[j] >= target */
            while (lo < hi) {
                int64_t mid = lo + (hi - lo) / 2;
                if (cdf[mid] >= target) hi = mid; else lo = mid + 1;
            }
            j = (int32_t)lo;
            walk_path(o, lo, (uint32_t)w, v, 0, 1, px, ps, pc, &r);
            if (r.status != OR_OK && st == OR_OK) st = r.status;
            /* r.f = W v[X_t]; the forward value uses W alone */
            y = V * (v[lo] > 0.0 ? 1.0 : -1.0) * exp(r.logw);
            if (!isfinite(y) && st == OR_OK) st = OR_ERR_OVERFLOW;
            x_end = r.x_end;
            /* per-node compensated sums of Y and Y^2 (Neumaier) */
            double *pairs[2][2] = { { s1, c1 }, { s2, c2 } };
            double add[2] = { y, y * y };
            for (int q = 0; q < 2; ++q) {
                double *sq = pairs[q][0], *cq = pairs[q][1];
                double a = sq[x_end], b = add[q], tt = a + b;
                if (fabs(a) >= fabs(b)) cq[x_end] += (a - tt) + b;
                else cq[x_end] += (b - tt) + a;
                sq[x_end] = tt;
            }
        }
        ys[w] = y;
        if (w_start) w_start[w] = j;
        if (w_end) w_end[w] = x_end;
        if (w_events) w_events[w] = r.events;
        if (w_jumps) w_jumps[w] = r.jumps;
        if (w_y) w_y[w] = y;
    }
    for (int64_t i = 0; i < n; ++i) {
        double sy = s1[i] + c1[i], syy = s2[i] + c2[i];
        double mean = sy / (double)nwalk;
        if (est) est[i] = mean;
        if (se) {
            if (nwalk > 1) {
                double var = (syy - (double)nwalk * mean * mean) / (double)(nwalk - 1);
                se[i] = sqrt((var > 0.0 ? var : 0.0) / (double)nwalk);
            } else {
                se[i] = 0.0;
            }
        }
    }
    {
        double mean = neumaier_sum(ys, nwalk) / (double)nwalk;
        if (sum) *sum = mean;
        if (sum_se) {
            if (nwalk > 1) {
                for (int64_t w = 0; w < nwalk; ++w) ys[w] = (ys[w] - mean) * (ys[w] - mean);
                *sum_se = sqrt(neumaier_sum(ys, nwalk) / (double)(nwalk - 1) / (double)nwalk);
            } else {
                *sum_se = 0.0;
            }
        }
    }
out:
    free(cdf); free(s1); free(c1); free(s2); free(c2); free(ys); free(px); free(ps); free(pc);
    return st;
}

/* ------------------------------------------------------------- accessors */
int64_t oracle_nslots(const oracle_t *o) { return o->nslots; }
int64_t oracle_ngrid(const oracle_t *o) { return o->ngrid; }
double oracle_dt(const oracle_t *o) { return o->dt; }

/* Copy the per-row and per-slot tables (plain, or proposal when use_prop). */
int oracle_get_tables(const oracle_t *o, int use_prop, double *r, double *d, double *inv_r,
                      int64_t *deg, int64_t *begin, int32_t *col, uint32_t *thr,
                      int32_t *alias, double *logcorr)
{
    const table_set *ts = use_prop ? &o->prop : &o->plain;
    if (use_prop && !o->has_proposal) return OR_ERR_INVALID_ARG;
    int64_t n = o->n, ns = o->nslots;
    if (r) memcpy(r, ts->r, sizeof(double) * (size_t)n);
    if (d) memcpy(d, ts->d, sizeof(double) * (size_t)n);
    if (inv_r) memcpy(inv_r, ts->inv_r, sizeof(double) * (size_t)n);
    if (deg) memcpy(deg, ts->deg, sizeof(int64_t) * (size_t)n);
    if (begin) memcpy(begin, ts->begin, sizeof(int64_t) * (size_t)n);
    if (col) memcpy(col, ts->col, sizeof(int32_t) * (size_t)ns);
    if (thr) memcpy(thr, ts->thr, sizeof(uint32_t) * (size_t)ns);
    if (alias) memcpy(alias, ts->alias, sizeof(int32_t) * (size_t)ns);
    if (logcorr) memcpy(logcorr, ts->logcorr, sizeof(double) * (size_t)ns);
    return OR_OK;
}
