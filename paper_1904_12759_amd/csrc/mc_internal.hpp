// Internal declarations of libmcexpmv: device table layout, the Philox
// generator, and the launch entry points shared between translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mc_expmv.h"

namespace mc {

// ---------------------------------------------------------------- tables
// Row record, 16 bytes: everything a walker needs about its current state x
// except the weight exponent d_x, which sits in its own array so that the
// FP32 weight mode reads 4 bytes instead of 8.
struct alignas(16) RowRec {
    double inv_r;      // 1 / r_x (unused when deg == 0)
    uint32_t deg;      // number of jump slots (positive off-diagonal entries)
    uint32_t begin;    // first slot; slots of row x are begin .. begin+deg-1
};

// Alias slot, 16 bytes (one dwordx4 gather per jump): keep `self` iff
// o3 < thr, else jump to `alias`.  aslot is the slot (within the row) that
// `alias` came from, used to locate the tilted-proposal correction.
struct alignas(16) SlotRec {
    uint32_t thr;
    int32_t self;
    int32_t alias;
    uint32_t aslot;
};

// Alias slot with its two destinations' row records and d values, 64 bytes
// (one aligned cache-line half): a jump then needs one gather instead of a slot
// gather followed by the destination's row and d gathers, which halves the
// chain of dependent loads per event where the tables miss in cache.  ds/da
// hold the weight precision's d exactly (a float widened to double in FP32
// mode).  Built from the final (walk-order) tables, so values equal theirs.
struct alignas(64) FatSlot {
    SlotRec s;
    RowRec rs, ra;     // rows of s.self and s.alias
    double ds, da;     // d of s.self and s.alias
};
// State of a node of the matrix-free 7-point stencil: 1/r, which faces carry a
// rate, and the jump thresholds, 32 bytes in two arrays -- a RowRec in `rows`
// (deg = the face word, non-zero iff the node has an exit; begin = the first
// threshold) read with the state as for the table walk, and the other four
// thresholds (a uint4 in the tail array) read at a jump.  Faces of x in column
// order are -z, -y, -x, +x, +y, +z (codes 0..5); with p_1 < ... < p_k the faces of
// positive rate, the inverse-CDF jump with u = o2 2^-32 goes to p_{1+m},
// m = #{j < k : o2 > e_j}: e_j is the largest o2 whose u r stays below the running
// sum of the faces up to p_j (found exactly at setup, so the walk compares
// integers), and e_j = 2^32 - 1 for j >= k (never counted).  The face word is
// k (bits 0..2) | p_j (3 bits at bit 3j, j = 1..k).

// Automatic choice (opts.slot_rows == 0): 64-byte slots when the row, d and slot
// tables together exceed kFatAutoBytes, about the size past which they stop
// being cache resident, and the 64-byte slots take at most kFatAutoMaxBytes
// (larger tables, such as those of 3-D grids, come with gathers that stay
// near each other, where the 4x slot memory buys nothing).
constexpr int64_t kFatAutoBytes = 64ll << 20;
constexpr int64_t kFatAutoMaxBytes = 4ll << 30;

// One set of walk tables (plain, or the tilted proposal).
struct Tables {
    RowRec *rows = nullptr;    // [n]
    double *d64 = nullptr;     // [n] weight exponent d_x
    float *d32 = nullptr;      // [n] (float)d_x for the FP32 weight mode
    double *r = nullptr;       // [n] exit rate r_x (setup and export only)
    SlotRec *slots = nullptr;  // [nnz]: row x uses slots rowptr[x] .. rowptr[x]+deg-1
    float2 *corr = nullptr;    // [nnz] proposal only: (-b_self, -b_alias) per slot
    // relabelled walk order (only with relabel): row/d of new id k = those of row
    // inv[k]; slot columns then hold new ids
    RowRec *wrows = nullptr;
    double *wd64 = nullptr;
    float *wd32 = nullptr;
    FatSlot *fat = nullptr;    // [nnz] 64-byte slots of the walk-order tables, or null
};

// Error flags latched on the device (bit i = status code i).
enum : uint32_t {
    F_INVALID_ARG = 1u << MC_ERR_INVALID_ARG,
    F_NOT_METZLER = 1u << MC_ERR_NOT_METZLER,
    F_NONFINITE = 1u << MC_ERR_NONFINITE,
    F_OUT_OF_RANGE = 1u << MC_ERR_OUT_OF_RANGE,
    F_WALK_LIMIT = 1u << MC_ERR_WALK_LIMIT,
    F_OVERFLOW = 1u << MC_ERR_OVERFLOW,
};

// Philox4x32-10 output block.
struct U4 {
    uint32_t x, y, z, w;
};

// ---------------------------------------------------------- launch params
// What a task needs to know about its instance (matrix, horizon, weights).
struct InstArgs {
    const RowRec *rows;
    const double *d64;
    const float *d32;
    const SlotRec *slots;
    const float2 *corr;        // non-null only for the tilted walk
    const FatSlot *fat;        // non-null: jumps read these instead of slots + rows + d
    const void *v;             // double* (FP64 weights) or float* (FP32 weights)
    const uint32_t *perm;      // relabel: original node -> walk id (null: identity)
    const uint32_t *inv;       // relabel: walk id -> original node (null: identity)
    uint32_t hot;              // walk ids < hot have their row and d staged in LDS
    const RowRec *lrows;       // LDS copy of rows[0 .. hot) (set inside the kernel)
    const void *ld;            // LDS copy of d[0 .. hot)
    double t;
    double dt;                 // t / N
    double inv_dt;             // N / t
    int32_t ngrid;             // N
    uint32_t key0, key1, inst, max_events;
    double cond_max_rt;        // first-jump conditioning for start nodes with t <= this / r
    uint32_t resort;           // relabelled walks: re-sort a wave's walkers every this many events (0: never)
    uint32_t qmc;              // 1: first event from the randomised rank-1 lattice (backward walks)
    // 7-point stencil without slots (stail null: the alias slots above): node
    // x = i + nx (j + ny k) has its state in rows[x], stail[x] and d64 / d32 [x]
    const uint4 *stail;
    uint32_t nx, nxy;
};

// Randomised rank-1 lattice of the first event: replicates of B = 2^b walker
// ordinals (b = 10 with FP32 weights, 9 with FP64: one replicate per chunk),
// Korobov generator a (119 for B = 512, 149 for B = 1024), shift drawn from
// the Philox counter (kQmcShiftMark, replicate, start node, instance).
constexpr uint32_t kQmcShiftMark = 0xFFFFFFFEu;
__host__ __device__ constexpr uint32_t qmc_bits(bool fp32) { return fp32 ? 10u : 9u; }

// Per-walker record (parity checks only).
struct TraceOut {
    int32_t *x = nullptr;
    uint32_t *ev = nullptr;
    uint32_t *ju = nullptr;
    double *f = nullptr;
    int64_t base = 0;
};

struct WalkArgs {
    InstArgs P;
    const int64_t *idx;        // null: entry e is node e
    int64_t k;                 // entries
    int64_t n;
    int64_t nwalk;             // walkers per entry
    int64_t w0;                // first walker ordinal (trace, and entries sized on the device)
    uint32_t chunk;            // walkers per task
    int64_t chunks;            // chunks per entry
    uint32_t group;            // entries per task (1 when chunks > 1)
    int64_t ntasks;            // ceil(k / group) * chunks
    double *est;               // [k]   (chunks == 1) final results
    double *se;                // [k] or null
    double *part;              // [k * chunks * 3] (count, mean, M2) per chunk
    unsigned long long *counters;  // [2 * grid]: events, jumps of every block
    uint32_t *flags;
    TraceOut trace;
    bool cond;                 // first-jump conditioning
    bool qmc;                  // standard errors from the replicate (chunk) means
    // entries with their own walker counts (null otherwise): entry e owns the
    // chunk slots var_task[e] .. var_task[e+1]-1 and var_nwalk[e] walkers; a task
    // takes `group` consecutive slots of the var_slots
    const int64_t *var_task;
    const int64_t *var_nwalk;
    int64_t var_slots;
    int64_t var_chunks_max;    // most chunks of one entry
    // walker counts written on the device (null otherwise): *slots_dev chunk slots,
    // one per task; ntasks and var_slots are then only an upper bound for the grid
    const int64_t *slots_dev;
};

// Forward (Algorithm 2) walks: one wave per chunk of kFwdChunk walker ordinals.
constexpr uint32_t kFwdChunk = 128;
// Guide-table cells for n nodes: about eight nodes per cell.
inline int64_t guide_cells(int64_t n) { return n > 8 ? (n + 7) / 8 : 1; }
// A visited state's record for the forward walks: the row record and d side by
// side (one 32-byte gather instead of two), built once per handle from P.rows
// and P.d64 / P.d32 in the same (walk) order.
struct alignas(16) FwdRow {
    double inv_r;
    uint32_t deg, begin;
    double d64;
    float d32;
    uint32_t pad;
};
static_assert(sizeof(FwdRow) == 32, "one 32-byte record per state");

struct FwdArgs {
    InstArgs P;                // plain tables; P.hot must be 0
    const FwdRow *frows;       // [n] row record + d of every state (walk order)
    int64_t n;
    int64_t nwalk;             // M
    int64_t w0;                // first walker ordinal (trace, and entries sized on the device)
    int64_t chunks;            // ceil(M / kFwdChunk)
    const double *cdf;         // [n] cumulative sums of |v| in node order
    const double *absv;        // [n] |v|
    const int8_t *vsign;       // [n] sign of v: 1, -1, or 0 for v = 0 (a small, cache-resident array)
    const int32_t *guide;      // [gcells + 1] guide table over cdf
    int64_t gcells;            // G = guide_cells(n)
    double *acc1, *acc2;       // [n] sums of Y and Y^2 per end node (acc2 may be null)
    double *part;              // [chunks * 3] (count, mean, M2) of Y per chunk
    unsigned long long *counters;  // [2 * grid]
    uint32_t *flags;
    int32_t *t_start, *t_end;  // per-walker trace (parity checks only)
    uint32_t *t_ev, *t_ju;
    double *t_y;
};

// One instance of a batched launch.
struct BatchInst {
    InstArgs P;
    const int64_t *idx;        // null: full vector
    int64_t k, n, nwalk, chunks;
    uint32_t group;            // entries per task
    int64_t task_begin;        // first task of this instance in the batch
    int64_t part_off;          // offset (doubles) of its chunk partials
    double *est, *se;
    int32_t mode, fp32;
};

// Largest number of instances in one batch (their task offsets sit in LDS).
constexpr int kMaxBatch = 1024;

struct BatchArgs {
    const BatchInst *inst;     // the instances of one class (weight mode, precision)
    int32_t ninst;
    int64_t ntasks;            // tasks of those instances
    int64_t task0;             // their first task in the batch's task numbering
    double *part;
    unsigned long long *counters;  // [2 * grid]
    uint32_t *flags;
    unsigned long long *queue;     // dynamic schedule counter
    uint32_t group;                // tasks per grab; 0 = static stride
    const int64_t *fin_begin;      // [ninst + 1] first finalize thread of each instance
    int64_t nfin;                  // finalize threads (a multiple of 64)
};

// Walkers per task (an entry with more walkers is split into chunks merged in a
// fixed order), and the most entries one task may pack when they have fewer.
// A task keeps one value per walker that may jump in LDS, so FP64 tasks are
// half as long as FP32 ones: both then fit five waves per SIMD.
constexpr uint32_t kChunkMax = 1024;
constexpr uint32_t kGroupMax = 64;
constexpr uint32_t chunk_walkers(bool fp32) { return fp32 ? kChunkMax : kChunkMax / 2; }
// Lanes that merge one entry's chunk partials: one for up to 8 chunks, then
// doubling up to sixteen waves of one block, so that a lane merges at most
// about eight partials, fetched together.
constexpr uint32_t kFinLanesMax = 1024;
__host__ __device__ constexpr uint32_t fin_lanes(int64_t chunks) {
    uint32_t l = 1;
    while (l < kFinLanesMax && (int64_t)l * 8 < chunks) l <<= 1;
    return l;
}
// Largest LDS budget for hot rows (bytes per block).
constexpr uint32_t kMaxHotBytes = 65536;
constexpr uint32_t kLdsPerCu = 160 * 1024;   // LDS bytes of one gfx950 compute unit

// Entries packed into one task when each of k entries has nwalk walkers.  A task
// runs its entries in LDS sessions of up to chunk_walkers() listed walkers, so
// packing keeps the lanes of the full-walk phase busy.  task_walkers > 0 asks
// for about that many walkers per task.  0 aims at kMinTasks tasks (four waves
// per SIMD slot at five waves per SIMD on 256 CUs, so that the last waves do
// not run alone) with between kTaskWalkersMin and kTaskWalkersMax walkers each,
// but leaves at least kFullTasks tasks (five waves on every SIMD) where there
// are that many entries: a small launch gains more from waves than from full
// lanes.
constexpr int64_t kTaskWalkersMin = 1024;
constexpr int64_t kTaskWalkersMax = 16384;
constexpr int64_t kMinTasks = 20480;
constexpr int64_t kFullTasks = 5120;
// Chunk slots of entries with their own walker counts each fill an LDS session
// already, so packing them only saves per-task work and lengthens the tail: the
// automatic group stops at this many walkers per task.
constexpr int64_t kSlotTaskWalkersMax = 2048;
inline uint32_t group_size(int64_t nwalk, int64_t k, uint32_t task_walkers) {
    int64_t g;
    if (task_walkers) {
        g = (int64_t)task_walkers / nwalk;
    } else {
        g = k / kMinTasks;
        if (g < kTaskWalkersMin / nwalk) g = kTaskWalkersMin / nwalk;
        if (g > kTaskWalkersMax / nwalk) g = kTaskWalkersMax / nwalk;
        if (g > k / kFullTasks) g = k / kFullTasks;
    }
    if (g > (int64_t)kGroupMax) g = kGroupMax;
    return (uint32_t)(g < 1 ? 1 : g);
}

// Tasks the grid of a run sized on the device covers at most (five waves on each
// of 1024 SIMDs, twice): the kernel then strides over the device's slot count.
constexpr int64_t kTargetGridTasks = 10240;

// Largest walk grid (blocks); the per-block counter buffer has this many pairs.
constexpr int kMaxWalkGrid = 1 << 16;

// host-side launchers (forward.hip)
hipError_t launch_check_symmetric(int64_t nnz, const int64_t *rowptr, const int32_t *rowof,
                                  const int32_t *col, const double *val, uint32_t *flag,
                                  hipStream_t s);
hipError_t launch_fwd_rows(int64_t n, const InstArgs &P, FwdRow *frows, hipStream_t s);
hipError_t launch_fwd_cdf(int64_t n, const void *v, bool fp32, double *absv, int8_t *vsign, double *cdf,
                          int32_t *guide, void *temp, size_t &temp_bytes, hipStream_t s);
int forward_grid(int64_t chunks);
hipError_t launch_forward(const FwdArgs &a, int mode, bool fp32, bool trace, double *sum_out,
                          hipStream_t s);

// host-side launchers (walk.hip)
int launch_walk_grid(int64_t ntasks, int block);
hipError_t launch_walk(const WalkArgs &a, int mode, bool fp32, bool prop, bool trace,
                       int block, hipStream_t s);
hipError_t launch_finalize(const WalkArgs &a, hipStream_t s);
// Walker counts of a run to a relative standard error target from a pilot run's
// estimates (walk.hip): var_task[0 .. k], var_nwalk[0 .. k), and at out2 the total
// chunk slots and the total walkers.
hipError_t launch_size_to_target(int64_t k, int64_t pilot, double target, double margin,
                                 int64_t min_walkers, int64_t max_walkers, int64_t chunk,
                                 const double *est, const double *se, int64_t *var_task,
                                 int64_t *var_nwalk, int64_t *out2, hipStream_t s);
hipError_t launch_math_eval(int fn, const double *x, double *y, int64_t n, hipStream_t s);

// batched launch (batch.hip): queue reset, persistent walk, finalize
// Instances of one weight mode and precision, contiguous in the batch.
struct BatchClass {
    int32_t mode;
    bool fp32;
    int32_t inst0, ninst;      // instances inst0 .. inst0+ninst-1
    int64_t task0, ntasks;     // their tasks task0 .. task0+ntasks-1
};
// One persistent walk launch per class (counters for class c at counters +
// 2 * grid * c), then one finalize launch for every instance.
hipError_t launch_batch(const BatchArgs &a, const BatchClass *classes, int nclass, int block,
                        int grid, hipStream_t s);

// learned proposal network (mlp.hip); parameter vector of kMlpParams floats:
// W1[64][8], b1[64], W2[64][64], b2[64], w3[64], b3
constexpr int kMlpParams = 64 * 8 + 64 + 64 * 64 + 64 + 64 + 1;
int mlp_grad_stride();
int mlp_blocks(int64_t ntile, int max_blocks);
// Blocks (of four waves) of a training step: each wave then accumulates several
// 16-edge tiles, and the per-wave partials to reduce stay few.
constexpr int kMlpTrainBlocks = 256;
hipError_t launch_rowof(int64_t n, const int64_t *rowptr, int32_t *rowof, hipStream_t s);
hipError_t launch_features(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                           const RowRec *rows, const double *r, const void *v, int v_fp32,
                           double *raw, double *stats, float *feats, hipStream_t s);
hipError_t launch_log_h(int64_t n, const double *est, const double *se, double nwalk, float *lh,
                        hipStream_t s);
hipError_t launch_net_forward(const uint16_t *wbf, const float *feats, const int32_t *rowof,
                              const int32_t *col, const double *val, const double *r, int64_t nnz,
                              float *out_b, hipStream_t s);
hipError_t launch_net_gradient(const uint16_t *wbf, const float *feats, const int32_t *rowof,
                               const int32_t *col, const double *val, const double *r,
                               const float *lh, int64_t p0, int64_t p1, int64_t tile0,
                               int64_t ntile, int64_t stride, int64_t tmod, int blocks,
                               float *gpart, double *gsum, float *grad, float *loss,
                               hipStream_t s);
hipError_t launch_adam(const float *grad, float *w, float *m, float *v, uint16_t *wbf, float lr,
                       int step, hipStream_t s);
hipError_t launch_mlp_init(float *w, float *m, float *v, uint16_t *wbf, uint64_t seed,
                           hipStream_t s);
hipError_t launch_params_bf16(const float *w, uint16_t *wbf, hipStream_t s);

// relabelling (setup.hip): hot rows (largest exit rate) first
hipError_t launch_relabel_keys(int64_t n, const double *r, unsigned long long *keys, uint32_t *vals,
                               hipStream_t s);
hipError_t launch_relabel_apply(int64_t n, const int64_t *rowptr, const uint32_t *inv,
                                uint32_t *perm, Tables &tb, bool build_perm, hipStream_t s);
hipError_t sort_pairs_u64(void *temp, size_t &temp_bytes, const unsigned long long *kin,
                          unsigned long long *kout, const uint32_t *vin, uint32_t *vout, int64_t n,
                          hipStream_t s);

// 64-byte slots of a finished table set (walk_order: the relabelled copies)
hipError_t launch_fat_slots(int64_t n, int64_t nnz, const Tables &tb, bool walk_order, bool fp32,
                            hipStream_t s);

// setup kernels (setup.hip)
hipError_t launch_stencil_rows(int64_t n, int64_t nx, int64_t ny, const double *fx, const double *fy,
                               const double *fz, const double *diag, RowRec *rows, uint4 *stail,
                               double *d64, float *d32, uint32_t *flags, unsigned long long *nslots,
                               hipStream_t s);
hipError_t launch_check_rowptr(int64_t n, int64_t nnz, const int64_t *rowptr, uint32_t *flags,
                               hipStream_t s);
hipError_t launch_setup_rows(int64_t n, const int64_t *rowptr, const int32_t *col,
                             const double *val, const float *bias, const Tables &base,
                             Tables &out, double *q_scratch, int32_t *stack_small,
                             int32_t *stack_large, uint32_t *flags, hipStream_t s);

}  // namespace mc
