// Host side of the C ABI declared in include/mc_expmv.h: argument checks,
// device allocations, kernel launches on the caller's stream, latched device
// errors and run statistics.  No C++ exception leaves this file.
#include <math.h>

#include <algorithm>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <new>
#include <vector>

#include "alloc.hpp"
#include "mlp.hpp"
#include "mc_internal.hpp"

using namespace mc;

// Scratch of mc_expmv_entries_noalloc: the (count, mean, M2) partials of entries
// that span several walker chunks, in a static device array so that the call
// allocates nothing.  Every GPU the library runs on holds its own copy, at its
// own address, until the process ends; host code uses the address obtained from
// hipGetSymbolAddress for the current device, never the array's name.
static __device__ __align__(256) double scratch[MC_NOALLOC_SCRATCH_DOUBLES];

struct mc_expmv_s {
    int dev = 0;
    int64_t n = 0, nnz = 0, nslots = 0;
    double t = 0.0;
    uint64_t seed = 0;
    mc_expmv_opts opts{};
    int64_t ngrid = 1;
    double dt = 0.0, inv_dt = 0.0;
    hipStream_t stream = nullptr;
    // copy of A, needed to rebuild tilted tables
    int64_t *rowptr = nullptr;
    int32_t *col = nullptr;
    double *val = nullptr;
    Tables plain, prop;
    bool has_prop = false;
    bool use_fat = false;                // 64-byte slots for every table set
    uint32_t *flags = nullptr;           // latched device errors
    uint32_t *flag_host = nullptr;       // pinned copy of *flags, read by mc_expmv_sync
    unsigned long long *counters = nullptr;
    double *part = nullptr;              // chunk partials
    int64_t part_cap = 0;                // doubles
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // last run
    bool ran = false;
    uint64_t last_walkers = 0;
    const int64_t *last_walkers_dev = nullptr;   // walker total written on the device
    int last_grid = 0;
    int32_t *rowof = nullptr;            // row of each CSR position (learned proposal)
    uint32_t *perm = nullptr;            // relabel: original node -> walk id
    uint32_t *inv = nullptr;             // relabel: walk id -> original node
    uint32_t hot = 0;                    // walk ids staged in LDS (lds_budget)
    float *bias = nullptr;               // copy of the installed proposal's edge biases
    bool last_fp32 = false, last_prop = false;
    // forward estimator
    int sym_state = -1;                  // A == A^T: -1 not checked yet, 0 no, 1 yes
    double *fwd_abs = nullptr, *fwd_cdf = nullptr;   // [n] |v| and its cumulative sums
    int8_t *fwd_sign = nullptr;          // [n] sign of v
    int32_t *fwd_guide = nullptr;        // guide table over fwd_cdf
    FwdRow *fwd_rows = nullptr;          // merged state records of the forward walks
    void *fwd_temp = nullptr;            // scan scratch
    size_t fwd_temp_bytes = 0;
    double *fwd_part = nullptr;          // chunk partials of Y
    int64_t fwd_part_cap = 0;
    double *fwd_acc = nullptr;           // [n] sums for trace runs
    bool last_fwd = false;
    // entries with their own walker counts
    int64_t *var_dev = nullptr;          // [2k + 1]: task offsets (k + 1), then counts (k)
    int64_t *var_host = nullptr;         // pinned staging of the same
    int64_t var_cap = 0;                 // int64 slots in both
    hipEvent_t var_ev = nullptr;         // staging copy done
    double *tgt_se = nullptr;            // pilot standard errors of entries_to_target
    int64_t tgt_se_cap = 0;
    double *scratch = nullptr;           // this device's copy of `scratch` (noalloc entries)
    // matrix-free 7-point stencil (mc_expmv_create_stencil7): the other half of the
    // state (rows and d in plain)
    bool stencil = false;
    uint4 *stail = nullptr;
    uint32_t snx = 0, snxy = 0;
};

namespace mc {

namespace {
thread_local int g_fault_at = 0;     // MC_EXPMV_FAULT=alloc:K -> K (0: off)
thread_local int g_fault_count = 0;  // allocations made since the scope began

bool fault_fires() { return g_fault_at > 0 && ++g_fault_count == g_fault_at; }
}  // namespace

void fault_scope_begin() {
    g_fault_at = 0;
    g_fault_count = 0;
    const char *f = getenv("MC_EXPMV_FAULT");
    if (f && strncmp(f, "alloc:", 6) == 0) {
        const long k = strtol(f + 6, nullptr, 10);
        if (k > 0 && k < 1000000) g_fault_at = (int)k;
    }
}

hipError_t dev_malloc(void **p, size_t bytes) {
    *p = nullptr;
    if (fault_fires()) return hipErrorOutOfMemory;
    return hipMalloc(p, bytes);
}

hipError_t host_malloc(void **p, size_t bytes) {
    *p = nullptr;
    if (fault_fires()) return hipErrorOutOfMemory;
    return hipHostMalloc(p, bytes, 0);
}

}  // namespace mc

namespace {

constexpr int kMaxDevices = 64;
// Largest batch grid per compute unit (the per-block counters are sized for it).
constexpr int kBatchBlocksPerCuMax = 128;
std::mutex g_scratch_mu;
double *g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
hipError_t scratch_address(int dev, double **out) {
    *out = nullptr;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_dev[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

mc_status from_hip(hipError_t e) {
    if (e == hipSuccess) return MC_OK;
    if (e == hipErrorOutOfMemory) return MC_ERR_NO_MEMORY;
    (void)hipGetLastError();
    return MC_ERR_DEVICE;
}

#define HIP_TRY(expr)                               \
    do {                                            \
        hipError_t e_ = (expr);                     \
        if (e_ != hipSuccess) return from_hip(e_);  \
    } while (0)

mc_status flags_to_status(uint32_t f) {
    static const mc_status order[] = {MC_ERR_INVALID_ARG, MC_ERR_NONFINITE, MC_ERR_NOT_METZLER,
                                      MC_ERR_OUT_OF_RANGE, MC_ERR_WALK_LIMIT, MC_ERR_OVERFLOW};
    for (mc_status s : order)
        if (f & (1u << s)) return s;
    return MC_OK;
}

template <class T>
hipError_t dalloc(T **p, int64_t count) {
    *p = nullptr;
    if (count <= 0) count = 1;
    return dev_malloc((void **)p, sizeof(T) * (size_t)count);
}

void free_tables(Tables &tb) {
    (void)hipFree(tb.rows);
    (void)hipFree(tb.d64);
    (void)hipFree(tb.d32);
    (void)hipFree(tb.r);
    (void)hipFree(tb.slots);
    (void)hipFree(tb.corr);
    (void)hipFree(tb.wrows);
    (void)hipFree(tb.wd64);
    (void)hipFree(tb.wd32);
    (void)hipFree(tb.fat);
    tb = Tables{};
}

hipError_t alloc_tables(Tables &tb, int64_t n, int64_t nnz, bool with_corr) {
    hipError_t e;
    if ((e = dalloc(&tb.rows, n)) != hipSuccess) return e;
    if ((e = dalloc(&tb.d64, n)) != hipSuccess) return e;
    if ((e = dalloc(&tb.d32, n)) != hipSuccess) return e;
    if ((e = dalloc(&tb.r, n)) != hipSuccess) return e;
    if ((e = dalloc(&tb.slots, nnz)) != hipSuccess) return e;
    if (with_corr && (e = dalloc(&tb.corr, nnz)) != hipSuccess) return e;
    return hipSuccess;
}

// Walk-order copies of a table set under the handle's permutation; with
// build == true the permutation itself is computed first (descending r).
mc_status relabel_tables(mc_expmv_s *h, Tables &tb, bool build) {
    const int64_t n = h->n;
    hipError_t e = dalloc(&tb.wrows, n);
    if (e == hipSuccess) e = dalloc(&tb.wd64, n);
    if (e == hipSuccess) e = dalloc(&tb.wd32, n);
    if (e != hipSuccess) return from_hip(e);
    if (build) {
        unsigned long long *kin = nullptr, *kout = nullptr;
        uint32_t *vin = nullptr;
        void *tmp = nullptr;
        size_t tmp_bytes = 0;
        e = dalloc(&h->perm, n);
        if (e == hipSuccess) e = dalloc(&h->inv, n);
        if (e == hipSuccess) e = dalloc(&kin, n);
        if (e == hipSuccess) e = dalloc(&kout, n);
        if (e == hipSuccess) e = dalloc(&vin, n);
        if (e == hipSuccess) e = launch_relabel_keys(n, tb.r, kin, vin, h->stream);
        if (e == hipSuccess) e = sort_pairs_u64(nullptr, tmp_bytes, kin, kout, vin, h->inv, n, h->stream);
        if (e == hipSuccess) e = dev_malloc(&tmp, tmp_bytes > 0 ? tmp_bytes : 1);
        if (e == hipSuccess) e = sort_pairs_u64(tmp, tmp_bytes, kin, kout, vin, h->inv, n, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        (void)hipFree(kin);
        (void)hipFree(kout);
        (void)hipFree(vin);
        (void)hipFree(tmp);
        if (e != hipSuccess) return from_hip(e);
    }
    e = launch_relabel_apply(n, h->rowptr, h->inv, h->perm, tb, build, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    return from_hip(e);
}

// Build one table set from the handle's copy of A (bias == null: plain).
mc_status build_tables(mc_expmv_s *h, const float *bias, Tables &out) {
    double *q = nullptr;
    int32_t *st_small = nullptr, *st_large = nullptr;
    mc_status st = MC_OK;
    hipError_t e = dalloc(&q, h->nnz);
    if (e == hipSuccess) e = dalloc(&st_small, h->nnz);
    if (e == hipSuccess) e = dalloc(&st_large, h->nnz);
    if (e == hipSuccess) e = hipMemsetAsync(h->flags, 0, sizeof(uint32_t), h->stream);
    if (e == hipSuccess)
        e = launch_setup_rows(h->n, h->rowptr, h->col, h->val, bias, h->plain, out, q, st_small,
                              st_large, h->flags, h->stream);
    uint32_t f = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&f, h->flags, sizeof(f), hipMemcpyDeviceToHost,
                                            h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) st = from_hip(e);
    else st = flags_to_status(f);
    (void)hipFree(q);
    (void)hipFree(st_small);
    (void)hipFree(st_large);
    return st;
}

mc_status check_opts(const mc_expmv_opts &o) {
    if (o.mode != MC_EXACT && o.mode != MC_STRANG && o.mode != MC_LIE) return MC_ERR_INVALID_ARG;
    if (o.weight_prec != MC_FP64 && o.weight_prec != MC_FP32) return MC_ERR_INVALID_ARG;
    if (o.mode != MC_EXACT && (!isfinite(o.dt) || !(o.dt > 0.0))) return MC_ERR_INVALID_ARG;
    const uint32_t b = o.walkers_per_block;
    if (b != 64 && b != 128 && b != 256) return MC_ERR_INVALID_ARG;
    if (o.resort_period != 0 && !o.relabel) return MC_ERR_INVALID_ARG;
    if (o.relabel != 0 && o.relabel != 1) return MC_ERR_INVALID_ARG;
    if (o.lds_budget != 0 && (!o.relabel || o.lds_budget > kMaxHotBytes)) return MC_ERR_INVALID_ARG;
    if (o.cond_first_jump != 0 && o.cond_first_jump != 1) return MC_ERR_INVALID_ARG;
    if (!(o.cond_max_rt >= 0.0)) return MC_ERR_INVALID_ARG;
    if (o.slot_rows < -1 || o.slot_rows > 1) return MC_ERR_INVALID_ARG;
    if (o.qmc_first != 0 && o.qmc_first != 1) return MC_ERR_INVALID_ARG;
    // the lattice's shift counters (kQmcShiftMark, ...) must never be an event index
    if (o.qmc_first && (o.cond_first_jump || o.relabel || o.max_events >= kQmcShiftMark))
        return MC_ERR_INVALID_ARG;
    return MC_OK;
}

// 64-byte slots for a finished table set, when the handle uses them
mc_status fat_tables(mc_expmv_s *h, Tables &tb) {
    if (!h->use_fat) return MC_OK;
    hipError_t e = dalloc(&tb.fat, h->nnz);
    if (e == hipSuccess)
        e = launch_fat_slots(h->n, h->nnz, tb, h->perm != nullptr, h->opts.weight_prec == MC_FP32,
                             h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    return from_hip(e);
}

void fill_inst(const mc_expmv_s *h, const void *v, bool prop, InstArgs &P) {
    const Tables &tb = prop ? h->prop : h->plain;
    const bool rl = h->perm != nullptr;
    P.rows = rl ? tb.wrows : tb.rows;
    P.d64 = rl ? tb.wd64 : tb.d64;
    P.d32 = rl ? tb.wd32 : tb.d32;
    P.slots = tb.slots;
    P.corr = prop ? tb.corr : nullptr;
    P.fat = tb.fat;
    P.v = v;
    P.perm = h->perm;
    P.inv = h->inv;
    P.hot = h->hot;
    P.lrows = nullptr;
    P.ld = nullptr;
    P.t = h->t;
    P.dt = h->dt;
    P.inv_dt = h->inv_dt;
    P.ngrid = (int32_t)h->ngrid;
    P.key0 = (uint32_t)h->seed;
    P.key1 = (uint32_t)(h->seed >> 32);
    P.inst = h->opts.instance_id;
    P.max_events = h->opts.max_events ? h->opts.max_events : (1u << 24);
    P.cond_max_rt = h->opts.cond_max_rt;
    P.resort = rl ? h->opts.resort_period : 0u;
    P.qmc = h->opts.qmc_first ? 1u : 0u;
    P.stail = h->stencil ? h->stail : nullptr;
    P.nx = h->snx;
    P.nxy = h->snxy;
}

// Run the walk kernel for k entries (idx == null: every node).
// With ext_part set, chunk partials go there (ext_cap doubles) and nothing is
// allocated; a run that needs more returns MC_ERR_TOO_LARGE before any launch.
mc_status run_walk(mc_expmv_s *h, const void *v, const int64_t *idx, int64_t k, int64_t nwalk,
                   double *est, double *se, bool trace, int64_t w0, int32_t use_prop,
                   int32_t *tx, uint32_t *tev, uint32_t *tju, double *tf,
                   double *ext_part = nullptr, int64_t ext_cap = 0) {
    if (!v || nwalk < 1 || nwalk > 0xFFFFFFFFll) return MC_ERR_INVALID_ARG;
    if (use_prop && !h->has_prop) return MC_ERR_INVALID_ARG;
    if (k < 0) return MC_ERR_INVALID_ARG;
    const bool prop = use_prop != 0;
    const bool fp32 = h->opts.weight_prec == MC_FP32;
    const int64_t chunk = chunk_walkers(fp32);   // fixes the summation order
    const int64_t chunks = (nwalk + chunk - 1) / chunk;
    WalkArgs a{};
    fill_inst(h, v, prop, a.P);
    a.idx = idx;
    a.k = k;
    a.n = h->n;
    a.nwalk = nwalk;
    a.w0 = w0;
    a.chunk = (uint32_t)chunk;
    a.chunks = chunks;
    a.group = trace ? 1u : group_size(nwalk, k, h->opts.task_walkers);
    a.cond = h->opts.cond_first_jump != 0;
    a.qmc = h->opts.qmc_first != 0;
    a.ntasks = (k + a.group - 1) / a.group * chunks;
    a.est = est;
    a.se = se;
    a.counters = h->counters;
    a.flags = h->flags;
    if (trace) {
        a.trace.x = tx;
        a.trace.ev = tev;
        a.trace.ju = tju;
        a.trace.f = tf;
    }
    if (chunks > 1 && ext_part) {
        if (k > ext_cap / (3 * chunks)) return MC_ERR_TOO_LARGE;
        a.part = ext_part;
    } else if (chunks > 1) {
        const int64_t need = k * chunks * 3;
        if (need > h->part_cap) {
            HIP_TRY(hipStreamSynchronize(h->stream));
            (void)hipFree(h->part);
            h->part = nullptr;
            h->part_cap = 0;
            HIP_TRY(dalloc(&h->part, need));
            h->part_cap = need;
        }
        a.part = h->part;
    }
    HIP_TRY(hipEventRecord(h->ev0, h->stream));
    HIP_TRY(launch_walk(a, h->opts.mode, fp32, prop, trace, (int)h->opts.walkers_per_block,
                        h->stream));
    HIP_TRY(launch_finalize(a, h->stream));
    HIP_TRY(hipEventRecord(h->ev1, h->stream));
    h->ran = true;
    h->last_walkers = (uint64_t)k * (uint64_t)nwalk;
    h->last_walkers_dev = nullptr;
    h->last_grid = a.ntasks > 0 ? launch_walk_grid(a.ntasks, (int)h->opts.walkers_per_block) : 0;
    h->last_fp32 = fp32;
    h->last_prop = prop;
    h->last_fwd = false;
    return MC_OK;
}

}  // namespace

extern "C" {

void mc_expmv_default_opts(mc_expmv_opts *o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->struct_size = sizeof(mc_expmv_opts);
    o->mode = MC_EXACT;
    o->dt = 0.03125;
    o->weight_prec = MC_FP64;
    o->relabel = 0;
    o->lds_budget = 0;
    o->resort_period = 0;
    o->walkers_per_block = 64;
    o->instance_id = 0;
    o->max_events = 0;
    o->stream = nullptr;
    o->cond_first_jump = 0;
    o->cond_max_rt = INFINITY;
    o->task_walkers = 0;
    o->slot_rows = 0;
}

const char *mc_expmv_status_string(mc_status s) {
    switch (s) {
        case MC_OK: return "ok";
        case MC_ERR_INVALID_ARG: return "invalid argument";
        case MC_ERR_NOT_METZLER: return "negative off-diagonal entry";
        case MC_ERR_NONFINITE: return "non-finite value";
        case MC_ERR_OUT_OF_RANGE: return "entry index out of range";
        case MC_ERR_NOT_SYMMETRIC: return "matrix is not symmetric";
        case MC_ERR_NO_MEMORY: return "out of memory";
        case MC_ERR_DEVICE: return "HIP runtime error";
        case MC_ERR_WALK_LIMIT: return "walk-length cap reached";
        case MC_ERR_OVERFLOW: return "weight overflow";
        case MC_ERR_TOO_LARGE:
            return "request exceeds the fixed scratch of mc_expmv_entries_noalloc";
    }
    return "unknown status";
}

void mc_expmv_destroy(mc_expmv_t h) {
    if (!h) return;
    (void)hipSetDevice(h->dev);
    (void)hipStreamSynchronize(h->stream);
    free_tables(h->plain);
    free_tables(h->prop);
    (void)hipFree(h->rowptr);
    (void)hipFree(h->col);
    (void)hipFree(h->val);
    (void)hipFree(h->flags);
    if (h->flag_host) (void)hipHostFree(h->flag_host);
    (void)hipFree(h->counters);
    (void)hipFree(h->part);
    (void)hipFree(h->rowof);
    (void)hipFree(h->bias);
    (void)hipFree(h->perm);
    (void)hipFree(h->inv);
    (void)hipFree(h->fwd_abs);
    (void)hipFree(h->fwd_sign);
    (void)hipFree(h->fwd_cdf);
    (void)hipFree(h->fwd_guide);
    (void)hipFree(h->fwd_rows);
    (void)hipFree(h->fwd_temp);
    (void)hipFree(h->fwd_part);
    (void)hipFree(h->fwd_acc);
    (void)hipFree(h->var_dev);
    (void)hipFree(h->stail);
    if (h->var_host) (void)hipHostFree(h->var_host);
    if (h->var_ev) (void)hipEventDestroy(h->var_ev);
    (void)hipFree(h->tgt_se);
    if (h->ev0) (void)hipEventDestroy(h->ev0);
    if (h->ev1) (void)hipEventDestroy(h->ev1);
    delete h;
}

mc_status mc_expmv_create(mc_expmv_t *out, int64_t n, int64_t nnz, const int64_t *rowptr,
                          const int32_t *col, const double *val, double t, uint64_t seed,
                          const mc_expmv_opts *opts) {
    fault_scope_begin();
    if (!out) return MC_ERR_INVALID_ARG;
    *out = nullptr;
    mc_expmv_opts o;
    mc_expmv_default_opts(&o);
    if (opts) {
        if (opts->struct_size != sizeof(mc_expmv_opts)) return MC_ERR_INVALID_ARG;
        o = *opts;
    }
    mc_status st = check_opts(o);
    if (st != MC_OK) return st;
    if (n < 0 || n >= ((int64_t)1 << 31) || nnz < 0 || nnz >= ((int64_t)1 << 32))
        return MC_ERR_INVALID_ARG;
    if (!rowptr || (nnz > 0 && (!col || !val))) return MC_ERR_INVALID_ARG;
    if (!isfinite(t) || !(t >= 0.0)) return MC_ERR_INVALID_ARG;
    mc_expmv_s *h = new (std::nothrow) mc_expmv_s();
    if (!h) return MC_ERR_NO_MEMORY;
    h->n = n;
    h->nnz = nnz;
    h->t = t;
    h->seed = seed;
    h->opts = o;
    h->stream = (hipStream_t)o.stream;
    if (o.mode != MC_EXACT) {
        const double steps = ceil(t / o.dt);
        if (!(steps <= 2147483647.0)) {
            delete h;
            return MC_ERR_INVALID_ARG;
        }
        h->ngrid = steps < 1.0 ? 1 : (int64_t)steps;
    }
    h->dt = t / (double)h->ngrid;
    h->inv_dt = (double)h->ngrid / t;
#define CREATE_TRY(expr)                         \
    do {                                         \
        hipError_t e_ = (expr);                  \
        if (e_ != hipSuccess) {                  \
            mc_status s_ = from_hip(e_);         \
            mc_expmv_destroy(h);                 \
            return s_;                           \
        }                                        \
    } while (0)
    CREATE_TRY(hipGetDevice(&h->dev));
    CREATE_TRY(scratch_address(h->dev, &h->scratch));
    CREATE_TRY(hipEventCreate(&h->ev0));
    CREATE_TRY(hipEventCreate(&h->ev1));
    CREATE_TRY(dalloc(&h->flags, 1));
    CREATE_TRY(host_malloc((void **)&h->flag_host, sizeof(uint32_t)));
    CREATE_TRY(dalloc(&h->counters, 2 * (int64_t)kMaxWalkGrid));
    CREATE_TRY(hipMemsetAsync(h->flags, 0, sizeof(uint32_t), h->stream));
    CREATE_TRY(dalloc(&h->rowptr, n + 1));
    CREATE_TRY(dalloc(&h->col, nnz));
    CREATE_TRY(dalloc(&h->val, nnz));
    CREATE_TRY(hipMemcpyAsync(h->rowptr, rowptr, sizeof(int64_t) * (size_t)(n + 1),
                              hipMemcpyDefault, h->stream));
    if (nnz > 0) {
        CREATE_TRY(hipMemcpyAsync(h->col, col, sizeof(int32_t) * (size_t)nnz, hipMemcpyDefault,
                                  h->stream));
        CREATE_TRY(hipMemcpyAsync(h->val, val, sizeof(double) * (size_t)nnz, hipMemcpyDefault,
                                  h->stream));
    }
    // the row offsets must be valid before any row is read
    CREATE_TRY(launch_check_rowptr(n, nnz, h->rowptr, h->flags, h->stream));
    uint32_t f = 0;
    CREATE_TRY(hipMemcpyAsync(&f, h->flags, sizeof(f), hipMemcpyDeviceToHost, h->stream));
    CREATE_TRY(hipStreamSynchronize(h->stream));
    if (f) {
        mc_expmv_destroy(h);
        return MC_ERR_INVALID_ARG;
    }
    CREATE_TRY(alloc_tables(h->plain, n, nnz, false));
    {
        const int64_t table_bytes = n * (int64_t)(sizeof(RowRec) + sizeof(double)) +
                                    nnz * (int64_t)sizeof(SlotRec);
        const int64_t fat_bytes = nnz * (int64_t)sizeof(FatSlot);
        h->use_fat = o.slot_rows == 1 || (o.slot_rows == 0 && table_bytes > kFatAutoBytes &&
                                          fat_bytes <= kFatAutoMaxBytes);
    }
    st = build_tables(h, nullptr, h->plain);
    if (st == MC_OK && o.relabel) st = relabel_tables(h, h->plain, true);
    if (st == MC_OK) st = fat_tables(h, h->plain);
    if (st != MC_OK) {
        mc_expmv_destroy(h);
        return st;
    }
    if (o.lds_budget) {
        const uint32_t per_row = (uint32_t)sizeof(RowRec) +
                                 (o.weight_prec == MC_FP32 ? (uint32_t)sizeof(float) : (uint32_t)sizeof(double));
        const int64_t hot = o.lds_budget / per_row;
        h->hot = (uint32_t)(hot < n ? hot : n);
    }
    // number of jump slots
    {
        std::vector<RowRec> rows((size_t)n);
        if (n > 0)
            CREATE_TRY(hipMemcpy(rows.data(), h->plain.rows, sizeof(RowRec) * (size_t)n,
                                 hipMemcpyDeviceToHost));
        int64_t ns = 0;
        for (const RowRec &r : rows) ns += r.deg;
        h->nslots = ns;
    }
#undef CREATE_TRY
    *out = h;
    return MC_OK;
}

mc_status mc_expmv_create_stencil7(mc_expmv_t *out, int64_t nx, int64_t ny, int64_t nz,
                                   const double *fx, const double *fy, const double *fz,
                                   const double *diag, double t, uint64_t seed,
                                   const mc_expmv_opts *opts) {
    fault_scope_begin();
    if (!out) return MC_ERR_INVALID_ARG;
    *out = nullptr;
    mc_expmv_opts o;
    mc_expmv_default_opts(&o);
    if (opts) {
        if (opts->struct_size != sizeof(mc_expmv_opts)) return MC_ERR_INVALID_ARG;
        o = *opts;
    }
    mc_status st = check_opts(o);
    if (st != MC_OK) return st;
    if (o.relabel || o.cond_first_jump || o.qmc_first || o.slot_rows == 1) return MC_ERR_INVALID_ARG;
    if (nx < 1 || ny < 1 || nz < 1 || nx * ny >= ((int64_t)1 << 31) ||
        nx * ny * nz >= ((int64_t)1 << 31))
        return MC_ERR_INVALID_ARG;
    if (!fx || !fy || !fz || !diag) return MC_ERR_INVALID_ARG;
    if (!isfinite(t) || !(t >= 0.0)) return MC_ERR_INVALID_ARG;
    const int64_t n = nx * ny * nz;
    mc_expmv_s *h = new (std::nothrow) mc_expmv_s();
    if (!h) return MC_ERR_NO_MEMORY;
    h->n = n;
    h->nnz = 0;
    h->t = t;
    h->seed = seed;
    h->opts = o;
    h->stream = (hipStream_t)o.stream;
    h->stencil = true;
    h->snx = (uint32_t)nx;
    h->snxy = (uint32_t)(nx * ny);
    if (o.mode != MC_EXACT) {
        const double steps = ceil(t / o.dt);
        if (!(steps <= 2147483647.0)) {
            delete h;
            return MC_ERR_INVALID_ARG;
        }
        h->ngrid = steps < 1.0 ? 1 : (int64_t)steps;
    }
    h->dt = t / (double)h->ngrid;
    h->inv_dt = (double)h->ngrid / t;
#define CREATE_TRY(expr)                         \
    do {                                         \
        hipError_t e_ = (expr);                  \
        if (e_ != hipSuccess) {                  \
            mc_status s_ = from_hip(e_);         \
            mc_expmv_destroy(h);                 \
            return s_;                           \
        }                                        \
    } while (0)
    CREATE_TRY(hipGetDevice(&h->dev));
    CREATE_TRY(scratch_address(h->dev, &h->scratch));
    CREATE_TRY(hipEventCreate(&h->ev0));
    CREATE_TRY(hipEventCreate(&h->ev1));
    CREATE_TRY(dalloc(&h->flags, 1));
    CREATE_TRY(host_malloc((void **)&h->flag_host, sizeof(uint32_t)));
    CREATE_TRY(dalloc(&h->counters, 2 * (int64_t)kMaxWalkGrid));
    CREATE_TRY(dalloc(&h->plain.rows, n));
    CREATE_TRY(dalloc(&h->stail, n));
    CREATE_TRY(dalloc(&h->plain.d64, n));
    CREATE_TRY(dalloc(&h->plain.d32, n));
    // the faces and a_xx are needed only to build the state records and d
    double *faces = nullptr;
    CREATE_TRY(dalloc(&faces, 4 * n));
    const size_t bytes = sizeof(double) * (size_t)n;
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMemcpyAsync(faces, fx, bytes, hipMemcpyDefault, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(faces + n, fy, bytes, hipMemcpyDefault, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(faces + 2 * n, fz, bytes, hipMemcpyDefault, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(faces + 3 * n, diag, bytes, hipMemcpyDefault, h->stream);
    // counters[0] doubles as the slot count of the check (cleared by a fill kernel later)
    if (e == hipSuccess) e = hipMemsetAsync(h->flags, 0, sizeof(uint32_t), h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(h->counters, 0, sizeof(unsigned long long), h->stream);
    if (e == hipSuccess)
        e = launch_stencil_rows(n, nx, ny, faces, faces + n, faces + 2 * n, faces + 3 * n,
                                h->plain.rows, h->stail, h->plain.d64, h->plain.d32, h->flags,
                                h->counters, h->stream);
    uint32_t f = 0;
    unsigned long long slots = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&f, h->flags, sizeof(f), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&slots, h->counters, sizeof(slots), hipMemcpyDeviceToHost, h->stream);
    const hipError_t es = hipStreamSynchronize(h->stream);   // also before freeing on failure
    if (e == hipSuccess) e = es;
    (void)hipFree(faces);
    CREATE_TRY(e);
#undef CREATE_TRY
    if (f) {
        mc_expmv_destroy(h);
        return flags_to_status(f);
    }
    h->nslots = (int64_t)slots;
    *out = h;
    return MC_OK;
}

mc_status mc_expmv_entries(mc_expmv_t h, const void *v, const int64_t *idx, int64_t k,
                           int64_t n_walkers, double *est, double *stderr_) {
    fault_scope_begin();
    if (!h) return MC_ERR_INVALID_ARG;
    if (k > 0 && (!idx || !est)) return MC_ERR_INVALID_ARG;
    HIP_TRY(hipSetDevice(h->dev));
    return run_walk(h, v, idx, k, n_walkers, est, stderr_, false, 0, h->has_prop ? 1 : 0,
                    nullptr, nullptr, nullptr, nullptr);
}

mc_status mc_expmv_entries_noalloc(mc_expmv_t h, const void *v, const int64_t *idx, int64_t k,
                                   int64_t n_walkers, double *est, double *stderr_) {
    fault_scope_begin();
    if (!h || !h->scratch) return MC_ERR_INVALID_ARG;
    if (k > 0 && (!idx || !est)) return MC_ERR_INVALID_ARG;
    HIP_TRY(hipSetDevice(h->dev));
    return run_walk(h, v, idx, k, n_walkers, est, stderr_, false, 0, h->has_prop ? 1 : 0,
                    nullptr, nullptr, nullptr, nullptr, h->scratch, MC_NOALLOC_SCRATCH_DOUBLES);
}

mc_status mc_math_eval(int32_t fn, const double *x, double *y, int64_t n, void *stream) {
    if (fn < MC_FN_LOG || fn > MC_FN_EXP_F32 || n < 0) return MC_ERR_INVALID_ARG;
    if (n > 0 && (!x || !y)) return MC_ERR_INVALID_ARG;
    HIP_TRY(launch_math_eval(fn, x, y, n, (hipStream_t)stream));
    return MC_OK;
}

mc_status mc_expmv_entries_multi(mc_expmv_t h, const void *v, const int64_t *idx, int64_t k,
                                 const int64_t *n_walkers, double *est, double *stderr_) {
    fault_scope_begin();
    if (!h || !v || k < 0) return MC_ERR_INVALID_ARG;
    if (k > 0 && (!idx || !est || !n_walkers)) return MC_ERR_INVALID_ARG;
    HIP_TRY(hipSetDevice(h->dev));
    if (k == 0) return MC_OK;
    const bool fp32 = h->opts.weight_prec == MC_FP32;
    const int64_t chunk = chunk_walkers(fp32);
    const int64_t need = 2 * k + 1;
    if (need > h->var_cap) {
        HIP_TRY(hipStreamSynchronize(h->stream));
        (void)hipFree(h->var_dev);
        if (h->var_host) (void)hipHostFree(h->var_host);
        h->var_dev = nullptr;
        h->var_host = nullptr;
        h->var_cap = 0;
        HIP_TRY(dalloc(&h->var_dev, need));
        HIP_TRY(host_malloc((void **)&h->var_host, sizeof(int64_t) * (size_t)need));
        h->var_cap = need;
    }
    if (!h->var_ev) HIP_TRY(hipEventCreateWithFlags(&h->var_ev, hipEventDisableTiming));
    HIP_TRY(hipEventSynchronize(h->var_ev));   // the previous call's copy has left the staging
    int64_t *offs = h->var_host, *cnts = h->var_host + k + 1;
    uint64_t walkers = 0;
    int64_t chunks_max = 0;
    offs[0] = 0;
    for (int64_t e = 0; e < k; ++e) {
        const int64_t m = n_walkers[e];
        if (m < 1 || m > 0xFFFFFFFFll) return MC_ERR_INVALID_ARG;
        cnts[e] = m;
        const int64_t c = (m + chunk - 1) / chunk;
        offs[e + 1] = offs[e] + c;
        if (c > chunks_max) chunks_max = c;
        walkers += (uint64_t)m;
    }
    const int64_t ntasks = offs[k];
    if (ntasks * 3 > h->part_cap) {
        HIP_TRY(hipStreamSynchronize(h->stream));
        (void)hipFree(h->part);
        h->part = nullptr;
        h->part_cap = 0;
        HIP_TRY(dalloc(&h->part, ntasks * 3));
        h->part_cap = ntasks * 3;
    }
    HIP_TRY(hipMemcpyAsync(h->var_dev, h->var_host, sizeof(int64_t) * (size_t)need,
                           hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipEventRecord(h->var_ev, h->stream));
    const bool prop = h->has_prop;
    WalkArgs a{};
    fill_inst(h, v, prop, a.P);
    a.idx = idx;
    a.k = k;
    a.n = h->n;
    a.nwalk = 0;
    a.w0 = 0;
    a.chunk = (uint32_t)chunk;
    a.chunks = 1;
    // chunk slots packed per task like entries are (group_size with one chunk's
    // walkers per slot), automatically at most kSlotTaskWalkersMax walkers a task
    a.group = group_size(chunk, ntasks, h->opts.task_walkers);
    if (!h->opts.task_walkers && a.group > kSlotTaskWalkersMax / chunk)
        a.group = (uint32_t)(kSlotTaskWalkersMax / chunk);
    a.var_slots = ntasks;
    a.ntasks = (ntasks + a.group - 1) / a.group;
    a.est = est;
    a.se = stderr_;
    a.part = h->part;
    a.counters = h->counters;
    a.flags = h->flags;
    a.cond = h->opts.cond_first_jump != 0;
    a.qmc = h->opts.qmc_first != 0;
    a.var_task = h->var_dev;
    a.var_nwalk = h->var_dev + k + 1;
    a.var_chunks_max = chunks_max;
    HIP_TRY(hipEventRecord(h->ev0, h->stream));
    HIP_TRY(launch_walk(a, h->opts.mode, fp32, prop, false, (int)h->opts.walkers_per_block,
                        h->stream));
    HIP_TRY(launch_finalize(a, h->stream));
    HIP_TRY(hipEventRecord(h->ev1, h->stream));
    h->ran = true;
    h->last_walkers = walkers;
    h->last_walkers_dev = nullptr;
    h->last_grid = launch_walk_grid(a.ntasks, (int)h->opts.walkers_per_block);
    h->last_fp32 = fp32;
    h->last_prop = prop;
    h->last_fwd = false;
    return MC_OK;
}

mc_status mc_expmv_entries_to_target(mc_expmv_t h, const void *v, const int64_t *idx, int64_t k,
                                     int64_t pilot_walkers, double target, double margin,
                                     int64_t min_walkers, int64_t max_walkers, double *est,
                                     double *stderr_, int64_t *walkers_out) {
    fault_scope_begin();
    if (!h || !v || k < 0) return MC_ERR_INVALID_ARG;
    if (k > 0 && (!idx || !est)) return MC_ERR_INVALID_ARG;
    if (pilot_walkers < 2 || pilot_walkers > ((int64_t)1 << 31)) return MC_ERR_INVALID_ARG;
    if (!isfinite(target) || !(target > 0.0) || !isfinite(margin) || !(margin >= 1.0))
        return MC_ERR_INVALID_ARG;
    if (min_walkers < 2 || max_walkers < min_walkers || pilot_walkers + max_walkers > 0x100000000ll)
        return MC_ERR_INVALID_ARG;
    HIP_TRY(hipSetDevice(h->dev));
    if (k == 0) return MC_OK;
    if (k > 0x7FFFFFFF) return MC_ERR_INVALID_ARG;
    const bool fp32 = h->opts.weight_prec == MC_FP32;
    const int64_t chunk = chunk_walkers(fp32);
    // lattice replicates are chunks of ordinals: the production run starts on one
    if (h->opts.qmc_first && pilot_walkers % chunk != 0) return MC_ERR_INVALID_ARG;
    const int64_t per_entry = (max_walkers + chunk - 1) / chunk;
    if (per_entry > ((int64_t)1 << 40) / k) return MC_ERR_INVALID_ARG;
    const int64_t ub = k * per_entry;            // most chunk slots the sizing can ask for
    // pilot: ordinals 0 .. pilot-1, its estimates in est / stderr_ (a stderr buffer
    // of the handle's when the caller passes none: the sizing needs it)
    double *pse = stderr_;
    if (!pse) {
        if (k > h->tgt_se_cap) {
            HIP_TRY(hipStreamSynchronize(h->stream));
            (void)hipFree(h->tgt_se);
            h->tgt_se = nullptr;
            h->tgt_se_cap = 0;
            HIP_TRY(dalloc(&h->tgt_se, k));
            h->tgt_se_cap = k;
        }
        pse = h->tgt_se;
    }
    mc_status st = run_walk(h, v, idx, k, pilot_walkers, est, pse, false, 0, h->has_prop ? 1 : 0,
                            nullptr, nullptr, nullptr, nullptr);
    if (st != MC_OK) return st;
    const int64_t need = 2 * k + 3;
    if (need > h->var_cap) {
        HIP_TRY(hipStreamSynchronize(h->stream));
        (void)hipFree(h->var_dev);
        if (h->var_host) (void)hipHostFree(h->var_host);
        h->var_dev = nullptr;
        h->var_host = nullptr;
        h->var_cap = 0;
        HIP_TRY(dalloc(&h->var_dev, need));
        HIP_TRY(host_malloc((void **)&h->var_host, sizeof(int64_t) * (size_t)need));
        h->var_cap = need;
    }
    if (ub * 3 > h->part_cap) {
        HIP_TRY(hipStreamSynchronize(h->stream));
        (void)hipFree(h->part);
        h->part = nullptr;
        h->part_cap = 0;
        HIP_TRY(dalloc(&h->part, ub * 3));
        h->part_cap = ub * 3;
    }
    // the previous entries_multi's staging copy into var_dev is ordered before this
    // stream's work, so the sizing kernel may overwrite var_dev
    int64_t *var_task = h->var_dev, *var_nwalk = h->var_dev + k + 1, *out2 = h->var_dev + 2 * k + 1;
    HIP_TRY(launch_size_to_target(k, pilot_walkers, target, margin, min_walkers, max_walkers, chunk,
                                  est, pse, var_task, var_nwalk, out2, h->stream));
    const bool prop = h->has_prop;
    WalkArgs a{};
    fill_inst(h, v, prop, a.P);
    a.idx = idx;
    a.k = k;
    a.n = h->n;
    a.nwalk = 0;
    a.w0 = pilot_walkers;
    a.chunk = (uint32_t)chunk;
    a.chunks = 1;
    a.group = 1;
    // the grid covers at most the waves that stay resident several times over; the
    // kernel walks the device's slot count with a grid stride
    const int64_t grid_tasks = ub < kTargetGridTasks ? ub : kTargetGridTasks;
    a.var_slots = grid_tasks;
    a.ntasks = grid_tasks;
    a.slots_dev = out2;
    a.est = est;
    a.se = stderr_;
    a.part = h->part;
    a.counters = h->counters;
    a.flags = h->flags;
    a.cond = h->opts.cond_first_jump != 0;
    a.qmc = h->opts.qmc_first != 0;
    a.var_task = var_task;
    a.var_nwalk = var_nwalk;
    a.var_chunks_max = per_entry;
    HIP_TRY(hipEventRecord(h->ev0, h->stream));
    HIP_TRY(launch_walk(a, h->opts.mode, fp32, prop, false, (int)h->opts.walkers_per_block,
                        h->stream));
    HIP_TRY(launch_finalize(a, h->stream));
    HIP_TRY(hipEventRecord(h->ev1, h->stream));
    if (walkers_out)
        HIP_TRY(hipMemcpyAsync(walkers_out, var_nwalk, sizeof(int64_t) * (size_t)k,
                               hipMemcpyDeviceToDevice, h->stream));
    h->ran = true;
    h->last_walkers = 0;
    h->last_walkers_dev = out2 + 1;
    h->last_grid = launch_walk_grid(a.ntasks, (int)h->opts.walkers_per_block);
    h->last_fp32 = fp32;
    h->last_prop = prop;
    h->last_fwd = false;
    return MC_OK;
}

mc_status mc_expmv_full(mc_expmv_t h, const void *v, int64_t n_per_node, double *est,
                        double *stderr_) {
    fault_scope_begin();
    if (!h) return MC_ERR_INVALID_ARG;
    if (h->n > 0 && !est) return MC_ERR_INVALID_ARG;
    HIP_TRY(hipSetDevice(h->dev));
    return run_walk(h, v, nullptr, h->n, n_per_node, est, stderr_, false, 0,
                    h->has_prop ? 1 : 0, nullptr, nullptr, nullptr, nullptr);
}

mc_status mc_expmv_trace(mc_expmv_t h, const void *v, int64_t start, int64_t w0, int64_t count,
                         int32_t use_proposal, int32_t *x_end, uint32_t *events,
                         uint32_t *jumps, double *f) {
    fault_scope_begin();
    if (!h || !x_end || !events || !jumps || !f) return MC_ERR_INVALID_ARG;
    if (count < 1 || count > (1 << 20) || w0 < 0 || w0 + count > 0xFFFFFFFFll)
        return MC_ERR_INVALID_ARG;
    if (start < 0 || start >= h->n) return MC_ERR_OUT_OF_RANGE;
    HIP_TRY(hipSetDevice(h->dev));
    int64_t *didx = nullptr;
    double *dest = nullptr;
    HIP_TRY(dalloc(&didx, 1));
    hipError_t e = dalloc(&dest, 1);
    if (e == hipSuccess)
        e = hipMemcpyAsync(didx, &start, sizeof(int64_t), hipMemcpyHostToDevice, h->stream);
    mc_status st = from_hip(e);
    if (st == MC_OK)
        st = run_walk(h, v, didx, 1, count, dest, nullptr, true, w0, use_proposal, x_end, events,
                      jumps, f);
    if (st == MC_OK) st = from_hip(hipStreamSynchronize(h->stream));
    (void)hipFree(didx);
    (void)hipFree(dest);
    return st;
}

mc_status mc_expmv_set_proposal(mc_expmv_t h, const float *edge_bias) {
    fault_scope_begin();
    if (!h || h->stencil) return MC_ERR_INVALID_ARG;
    HIP_TRY(hipSetDevice(h->dev));
    HIP_TRY(hipStreamSynchronize(h->stream));
    free_tables(h->prop);
    h->has_prop = false;
    if (!edge_bias) return MC_OK;
    if (h->opts.mode != MC_EXACT) return MC_ERR_INVALID_ARG;
    HIP_TRY(alloc_tables(h->prop, h->n, h->nnz, true));
    mc_status st = build_tables(h, edge_bias, h->prop);
    if (st == MC_OK && h->perm) st = relabel_tables(h, h->prop, false);
    if (st == MC_OK) st = fat_tables(h, h->prop);
    if (st != MC_OK) {
        free_tables(h->prop);
        return st;
    }
    if (!h->bias) HIP_TRY(dalloc(&h->bias, h->nnz));
    HIP_TRY(hipMemcpyAsync(h->bias, edge_bias, sizeof(float) * (size_t)h->nnz,
                           hipMemcpyDeviceToDevice, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    h->has_prop = true;
    return MC_OK;
}

mc_status mc_expmv_get_proposal(mc_expmv_t h, float *edge_bias) {
    if (!h || h->stencil || !edge_bias || !h->has_prop) return MC_ERR_INVALID_ARG;
    HIP_TRY(hipSetDevice(h->dev));
    HIP_TRY(hipMemcpyAsync(edge_bias, h->bias, sizeof(float) * (size_t)h->nnz,
                           hipMemcpyDeviceToDevice, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return MC_OK;
}

mc_status mc_expmv_set_stream(mc_expmv_t h, void *stream) {
    if (!h) return MC_ERR_INVALID_ARG;
    hipStream_t next = (hipStream_t)stream;
    if (next != h->stream) {
        // the handle's scratch (partials, counters, staging) may still be in use by
        // work queued on the old stream: the new stream waits for it (no host wait)
        HIP_TRY(hipSetDevice(h->dev));
        hipEvent_t ev = nullptr;
        HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        hipError_t e = hipEventRecord(ev, h->stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(next, ev, 0);
        (void)hipEventDestroy(ev);
        HIP_TRY(e);
    }
    h->stream = next;
    h->opts.stream = stream;
    return MC_OK;
}

mc_status mc_expmv_sync(mc_expmv_t h) {
    if (!h) return MC_ERR_INVALID_ARG;
    HIP_TRY(hipSetDevice(h->dev));
    // the flag word comes back behind the stream's own work and is cleared there,
    // so the wait below is the only synchronisation
    HIP_TRY(hipMemcpyAsync(h->flag_host, h->flags, sizeof(uint32_t), hipMemcpyDeviceToHost,
                           h->stream));
    HIP_TRY(hipMemsetAsync(h->flags, 0, sizeof(uint32_t), h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return flags_to_status(*h->flag_host);
}

mc_status mc_expmv_stats(mc_expmv_t h, mc_expmv_run_stats *out) {
    if (!h || !out) return MC_ERR_INVALID_ARG;
    memset(out, 0, sizeof(*out));
    if (!h->ran) return MC_OK;
    HIP_TRY(hipSetDevice(h->dev));
    HIP_TRY(hipEventSynchronize(h->ev1));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, h->ev0, h->ev1));
    unsigned long long c[2] = {0, 0};
    if (h->last_grid > 0) {
        std::vector<unsigned long long> pc((size_t)h->last_grid * 2);
        HIP_TRY(hipMemcpy(pc.data(), h->counters, sizeof(unsigned long long) * pc.size(),
                          hipMemcpyDeviceToHost));
        for (int b = 0; b < h->last_grid; ++b) {
            c[0] += pc[2 * (size_t)b];
            c[1] += pc[2 * (size_t)b + 1];
        }
    }
    if (h->last_walkers_dev) {
        int64_t w = 0;
        HIP_TRY(hipMemcpy(&w, h->last_walkers_dev, sizeof(w), hipMemcpyDeviceToHost));
        h->last_walkers = (uint64_t)w;
        h->last_walkers_dev = nullptr;
    }
    out->walkers = h->last_walkers;
    out->events = c[0];
    out->jumps = c[1];
    out->ms = ms;
    // Algorithmic bytes with no reuse: a row record (16 B) and d (8/4 B) per
    // visited state, a 12 B alias slot (+8 B correction when tilted) per jump,
    // v[X_t] (8/4 B) per walker.
    const double dbytes = h->last_fp32 ? 4.0 : 8.0;
    const double row = 16.0 + dbytes;
    const double slot = 12.0 + (h->last_prop ? 8.0 : 0.0);
    out->alg_bytes = row * (double)(c[0]) + slot * (double)c[1] + dbytes * (double)h->last_walkers;
    if (h->stencil)   // a row record and d per visited state, 16 B of thresholds per jump
        out->alg_bytes = row * (double)(c[0]) + 16.0 * (double)c[1] + dbytes * (double)h->last_walkers;
    if (h->last_fwd) {
        // forward walks: per walker also the binary search over the cumulative
        // sums (8 B per step) and two FP64 read-modify-writes at the end node
        const double steps = h->n > 1 ? ceil(log2((double)h->n)) : 0.0;
        out->alg_bytes += (8.0 * steps + 32.0) * (double)h->last_walkers;
    }
    return MC_OK;
}

mc_status mc_expmv_get_stencil(mc_expmv_t h, double *d, double *inv_r, uint32_t *faces,
                               uint32_t *thr) {
    if (!h || !h->stencil) return MC_ERR_INVALID_ARG;
    HIP_TRY(hipSetDevice(h->dev));
    HIP_TRY(hipStreamSynchronize(h->stream));
    const size_t n = (size_t)h->n;
    std::vector<RowRec> head(n);
    std::vector<uint4> tail(n);
    std::vector<double> dd(n);
    if (n > 0) {
        HIP_TRY(hipMemcpy(head.data(), h->plain.rows, sizeof(RowRec) * n, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(tail.data(), h->stail, sizeof(uint4) * n, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(dd.data(), h->plain.d64, sizeof(double) * n, hipMemcpyDeviceToHost));
    }
    for (size_t i = 0; i < n; ++i) {
        if (d) d[i] = dd[i];
        if (inv_r) inv_r[i] = head[i].inv_r;
        if (faces) faces[i] = head[i].deg;
        if (thr) {
            uint32_t *q = thr + 5 * i;
            q[0] = head[i].begin;
            q[1] = tail[i].x;
            q[2] = tail[i].y;
            q[3] = tail[i].z;
            q[4] = tail[i].w;
        }
    }
    return MC_OK;
}

mc_status mc_expmv_get_tables(mc_expmv_t h, int32_t use_proposal, double *r, double *d,
                              double *inv_r, int64_t *deg, int64_t *begin, int32_t *col,
                              uint32_t *thr, int32_t *alias) {
    if (!h || h->stencil) return MC_ERR_INVALID_ARG;
    if (use_proposal && !h->has_prop) return MC_ERR_INVALID_ARG;
    HIP_TRY(hipSetDevice(h->dev));
    HIP_TRY(hipStreamSynchronize(h->stream));
    const Tables &tb = use_proposal ? h->prop : h->plain;
    const size_t n = (size_t)h->n;
    std::vector<RowRec> rows(n);
    std::vector<double> dd(n), rr(n);
    std::vector<SlotRec> sl((size_t)(h->nnz > 0 ? h->nnz : 1));
    if (n > 0) {
        HIP_TRY(hipMemcpy(rows.data(), tb.rows, sizeof(RowRec) * n, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(dd.data(), tb.d64, sizeof(double) * n, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(rr.data(), tb.r, sizeof(double) * n, hipMemcpyDeviceToHost));
    }
    if (h->nnz > 0)
        HIP_TRY(hipMemcpy(sl.data(), tb.slots, sizeof(SlotRec) * (size_t)h->nnz,
                          hipMemcpyDeviceToHost));
    std::vector<uint32_t> inv;
    if (h->inv) {
        inv.resize(n);
        HIP_TRY(hipMemcpy(inv.data(), h->inv, sizeof(uint32_t) * n, hipMemcpyDeviceToHost));
    }
    auto orig = [&](int32_t c) { return h->inv ? (int32_t)inv[(size_t)c] : c; };
    int64_t pos = 0;
    for (size_t i = 0; i < n; ++i) {
        if (r) r[i] = rr[i];
        if (d) d[i] = dd[i];
        if (inv_r) inv_r[i] = rows[i].inv_r;
        if (deg) deg[i] = rows[i].deg;
        if (begin) begin[i] = pos;
        for (uint32_t s = 0; s < rows[i].deg; ++s) {
            const SlotRec &q = sl[rows[i].begin + s];
            if (col) col[pos] = orig(q.self);
            if (thr) thr[pos] = q.thr;
            if (alias) alias[pos] = orig(q.alias);
            ++pos;
        }
    }
    return MC_OK;
}

mc_status mc_expmv_info(mc_expmv_t h, int64_t *n, int64_t *nslots, int64_t *ngrid, double *dt) {
    if (!h) return MC_ERR_INVALID_ARG;
    if (n) *n = h->n;
    if (nslots) *nslots = h->nslots;
    if (ngrid) *ngrid = h->ngrid;
    if (dt) *dt = h->dt;
    return MC_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batches
#include <stdio.h>
#include <stdlib.h>

#include <string>

struct mc_batch_s {
    int dev = 0;
    int ncu = 0;
    std::string devname;
    hipStream_t user = nullptr;      // caller's stream
    hipStream_t stream = nullptr;    // private stream (graph capture needs a non-null one)
    uint64_t seed = 0;
    std::vector<mc_expmv_t> handles; // table owners, one per instance
    std::vector<BatchInst> inst;         // grouped by class (weight mode, precision)
    std::vector<BatchClass> classes;
    std::vector<int64_t> fin_begin;
    BatchInst *d_inst = nullptr;
    int64_t *d_fin = nullptr;
    double *part = nullptr;
    unsigned long long *counters = nullptr;
    unsigned long long *queue = nullptr;
    uint32_t *flags = nullptr;
    uint32_t *flag_host = nullptr;       // pinned copy of *flags, read by mc_expmv_batch_sync
    BatchArgs args{};
    int block = 256, grid = 0;
    uint32_t group = 0;
    bool use_graph = true;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr, ev_user = nullptr, ev_done = nullptr;
    uint64_t walkers = 0;
    bool ran = false;
};

namespace {

void batch_free(mc_batch_s *b) {
    if (!b) return;
    (void)hipSetDevice(b->dev);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (mc_expmv_t h : b->handles) mc_expmv_destroy(h);
    (void)hipFree(b->d_inst);
    (void)hipFree(b->d_fin);
    (void)hipFree(b->part);
    (void)hipFree(b->counters);
    (void)hipFree(b->queue);
    (void)hipFree(b->flags);
    if (b->flag_host) (void)hipHostFree(b->flag_host);
    if (b->ev0) (void)hipEventDestroy(b->ev0);
    if (b->ev1) (void)hipEventDestroy(b->ev1);
    if (b->ev_user) (void)hipEventDestroy(b->ev_user);
    if (b->ev_done) (void)hipEventDestroy(b->ev_done);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

hipError_t batch_launch(mc_batch_s *b) {
    b->args.group = b->group;
    return launch_batch(b->args, b->classes.data(), (int)b->classes.size(), b->block, b->grid,
                        b->stream);
}

// (Re)build the graph for the current block / grid / group.
hipError_t batch_capture(mc_batch_s *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    if (!b->use_graph) return hipSuccess;
    hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = batch_launch(b);
    e = hipStreamEndCapture(b->stream, &b->graph);
    if (le != hipSuccess) return le;
    if (e != hipSuccess) return e;
    return hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
}

// Candidate schedules for the autotuner; none of them changes any result.
struct Sched {
    int block, per_cu;
    uint32_t group;
};

std::string tune_key(const mc_batch_s *b) {
    char buf[256];
    uint64_t tasks = (uint64_t)b->args.ntasks;
    snprintf(buf, sizeof(buf), "%s|cu%d|inst%zu|tasks%llu|walkers%llu", b->devname.c_str(),
             b->ncu, b->inst.size(), (unsigned long long)tasks,
             (unsigned long long)b->walkers);
    std::string k(buf);
    for (char &c : k)
        if (c == ' ') c = '_';
    return k;
}

bool tune_cache_lookup(const mc_batch_s *b, Sched &out) {
    const char *path = getenv("MC_EXPMV_TUNE_CACHE");
    if (!path || !*path) return false;
    FILE *f = fopen(path, "r");
    if (!f) return false;
    const std::string key = tune_key(b);
    char k[512];
    int blk, pcu;
    unsigned grp;
    bool found = false;
    while (fscanf(f, "%511s %d %d %u", k, &blk, &pcu, &grp) == 4) {
        if (key == k && (blk == 64 || blk == 128 || blk == 256) && pcu > 0 && pcu <= 64) {
            out = Sched{blk, pcu, grp};
            found = true;
        }
    }
    fclose(f);
    return found;
}

void tune_cache_store(const mc_batch_s *b, const Sched &s) {
    const char *path = getenv("MC_EXPMV_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s %d %d %u\n", tune_key(b).c_str(), s.block, s.per_cu, s.group);
    fclose(f);
}

// Time each candidate schedule (one warm-up and two timed launches) and keep
// the fastest.
mc_status autotune(mc_batch_s *b, float *best_ms_out) {
    static const Sched cands[] = {
        {256, 4, 0},  {256, 8, 0},   {256, 16, 0},  {256, 32, 0}, {256, 64, 0}, {256, 128, 0},
        {128, 8, 0},
        {128, 16, 0}, {128, 32, 0},  {64, 16, 0},   {64, 32, 0},  {256, 8, 16}, {256, 8, 128},
        {128, 16, 16}, {64, 32, 16}, {64, 32, 64},  {256, 16, 64},
    };
    float best = 1e30f;
    Sched bs = cands[0];
    for (const Sched &c : cands) {
        b->block = c.block;
        b->grid = b->ncu * c.per_cu;
        b->group = c.group;
        float tmin = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            HIP_TRY(hipEventRecord(b->ev0, b->stream));
            HIP_TRY(batch_launch(b));
            HIP_TRY(hipEventRecord(b->ev1, b->stream));
            HIP_TRY(hipEventSynchronize(b->ev1));
            float ms = 0.0f;
            HIP_TRY(hipEventElapsedTime(&ms, b->ev0, b->ev1));
            if (rep > 0 && ms < tmin) tmin = ms;
        }
        if (tmin < best) {
            best = tmin;
            bs = c;
        }
    }
    b->block = bs.block;
    b->grid = b->ncu * bs.per_cu;
    b->group = bs.group;
    if (best_ms_out) *best_ms_out = best;
    tune_cache_store(b, bs);
    return MC_OK;
}

}  // namespace

extern "C" {

void mc_batch_default_opts(mc_batch_opts *o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->struct_size = sizeof(mc_batch_opts);
    o->walkers_per_block = 0;
    o->blocks_per_cu = 0;
    o->group = 0;
    o->use_graph = 1;
    o->max_events = 0;
    o->stream = nullptr;
    o->slot_rows = 0;
}

void mc_expmv_batch_destroy(mc_batch_t b) { batch_free(b); }

mc_status mc_expmv_batch_create(mc_batch_t *out, int32_t n_inst, const mc_instance_desc *desc,
                                uint64_t seed, const mc_batch_opts *opts) {
    fault_scope_begin();
    if (!out) return MC_ERR_INVALID_ARG;
    *out = nullptr;
    if (n_inst < 1 || n_inst > kMaxBatch || !desc) return MC_ERR_INVALID_ARG;
    mc_batch_opts o;
    mc_batch_default_opts(&o);
    if (opts) {
        if (opts->struct_size != sizeof(mc_batch_opts)) return MC_ERR_INVALID_ARG;
        o = *opts;
    }
    const uint32_t wpb = o.walkers_per_block;
    if (wpb != 0 && wpb != 64 && wpb != 128 && wpb != 256) return MC_ERR_INVALID_ARG;
    if (o.blocks_per_cu > kBatchBlocksPerCuMax) return MC_ERR_INVALID_ARG;
    if (o.slot_rows < -1 || o.slot_rows > 1) return MC_ERR_INVALID_ARG;
    for (int i = 0; i < n_inst; ++i) {
        const mc_instance_desc &d = desc[i];
        if (!d.v || d.n_walkers < 1 || d.n_walkers > 0xFFFFFFFFll) return MC_ERR_INVALID_ARG;
        if (d.idx && (d.k < 0 || (d.k > 0 && !d.est))) return MC_ERR_INVALID_ARG;
        if (!d.idx && d.n > 0 && !d.est) return MC_ERR_INVALID_ARG;
    }
    mc_batch_s *b = new (std::nothrow) mc_batch_s();
    if (!b) return MC_ERR_NO_MEMORY;
    b->seed = seed;
    b->user = (hipStream_t)o.stream;
    b->use_graph = o.use_graph != 0;
#define B_TRY(expr)                              \
    do {                                         \
        hipError_t e_ = (expr);                  \
        if (e_ != hipSuccess) {                  \
            mc_status s_ = from_hip(e_);         \
            batch_free(b);                       \
            return s_;                           \
        }                                        \
    } while (0)
    B_TRY(hipGetDevice(&b->dev));
    hipDeviceProp_t prop;
    B_TRY(hipGetDeviceProperties(&prop, b->dev));
    b->ncu = prop.multiProcessorCount;
    b->devname = prop.gcnArchName;
    B_TRY(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
    B_TRY(hipEventCreate(&b->ev0));
    B_TRY(hipEventCreate(&b->ev1));
    B_TRY(hipEventCreateWithFlags(&b->ev_user, hipEventDisableTiming));
    B_TRY(hipEventCreateWithFlags(&b->ev_done, hipEventDisableTiming));
    // the caller's stream may still be producing A, v or idx
    B_TRY(hipEventRecord(b->ev_user, b->user));
    B_TRY(hipStreamWaitEvent(b->stream, b->ev_user, 0));

    int64_t ntasks = 0, part_doubles = 0, nfin = 0;
    b->fin_begin.assign((size_t)n_inst + 1, 0);
    // instances grouped by class (weight mode, precision), each class one
    // specialised persistent launch; order within a class as given
    std::vector<int> order((size_t)n_inst);
    for (int i = 0; i < n_inst; ++i) order[(size_t)i] = i;
    auto cls = [&](int i) { return desc[i].mode * 2 + (desc[i].weight_prec == MC_FP32 ? 1 : 0); };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cls(x) < cls(y); });
    // entries of the whole batch: the instances share one persistent grid, so task
    // packing is sized by the batch's task count, not by each instance's
    int64_t k_all = 0;
    for (int i = 0; i < n_inst; ++i) k_all += desc[i].idx ? desc[i].k : desc[i].n;
    for (int oi = 0; oi < n_inst; ++oi) {
        const int i = order[(size_t)oi];
        const mc_instance_desc &d = desc[i];
        if (b->classes.empty() || b->classes.back().mode * 2 + (b->classes.back().fp32 ? 1 : 0) != cls(i))
            b->classes.push_back(BatchClass{d.mode, d.weight_prec == MC_FP32, oi, 0, ntasks, 0});
        mc_expmv_opts io;
        mc_expmv_default_opts(&io);
        io.mode = d.mode;
        io.dt = d.dt;
        io.weight_prec = d.weight_prec;
        io.instance_id = d.instance_id;
        io.max_events = o.max_events;
        io.stream = b->stream;
        io.slot_rows = o.slot_rows;
        mc_expmv_t h = nullptr;
        mc_status st = mc_expmv_create(&h, d.n, d.nnz, d.rowptr, d.col, d.val, d.t, seed, &io);
        if (st != MC_OK) {
            batch_free(b);
            return st;
        }
        b->handles.push_back(h);
        BatchInst I{};
        fill_inst(h, d.v, false, I.P);
        I.idx = d.idx;
        I.k = d.idx ? d.k : d.n;
        I.n = d.n;
        I.nwalk = d.n_walkers;
        const bool fp32 = d.weight_prec == MC_FP32;
        const int64_t chunk = chunk_walkers(fp32);
        I.chunks = (d.n_walkers + chunk - 1) / chunk;
        I.group = group_size(d.n_walkers, k_all, 0);
        I.task_begin = ntasks;
        I.part_off = part_doubles;
        I.est = d.est;
        I.se = d.stderr_;
        I.mode = d.mode;
        I.fp32 = fp32;
        const int64_t itasks = (I.k + I.group - 1) / I.group * I.chunks;
        ntasks += itasks;
        b->classes.back().ninst += 1;
        b->classes.back().ntasks += itasks;
        if (I.chunks > 1) {
            // a multiple of 64 and of the lane count: a group never spans two blocks
            const int64_t L = fin_lanes(I.chunks), al = L > 64 ? L : 64;
            nfin = (nfin + al - 1) / al * al;
            b->fin_begin[(size_t)oi] = nfin;
            part_doubles += I.k * I.chunks * 3;
            nfin += (I.k * L + 63) / 64 * 64;
        } else {
            b->fin_begin[(size_t)oi] = nfin;
        }
        b->walkers += (uint64_t)I.k * (uint64_t)I.nwalk;
        b->inst.push_back(I);
    }
    b->fin_begin[n_inst] = nfin;
    B_TRY(dalloc(&b->d_inst, n_inst));
    B_TRY(dalloc(&b->d_fin, n_inst + 1));
    B_TRY(dalloc(&b->part, part_doubles));
    B_TRY(dalloc(&b->counters, 2 * (int64_t)b->ncu * kBatchBlocksPerCuMax * (int64_t)b->classes.size()));
    B_TRY(dalloc(&b->queue, 1));
    B_TRY(dalloc(&b->flags, 1));
    B_TRY(host_malloc((void **)&b->flag_host, sizeof(uint32_t)));
    B_TRY(hipMemcpyAsync(b->d_inst, b->inst.data(), sizeof(BatchInst) * (size_t)n_inst,
                         hipMemcpyHostToDevice, b->stream));
    B_TRY(hipMemcpyAsync(b->d_fin, b->fin_begin.data(), sizeof(int64_t) * (size_t)(n_inst + 1),
                         hipMemcpyHostToDevice, b->stream));
    B_TRY(hipMemsetAsync(b->flags, 0, sizeof(uint32_t), b->stream));
    B_TRY(hipStreamSynchronize(b->stream));
    BatchArgs &a = b->args;
    a.inst = b->d_inst;
    a.ninst = n_inst;
    a.ntasks = ntasks;
    a.part = b->part;
    a.counters = b->counters;
    a.flags = b->flags;
    a.queue = b->queue;
    a.fin_begin = b->d_fin;
    a.nfin = nfin;

    // schedule: given, cached, or tuned
    Sched sc{256, 8, 0};
    if (wpb != 0 && o.blocks_per_cu != 0) {
        sc = Sched{(int)wpb, (int)o.blocks_per_cu, o.group};
        b->block = sc.block;
        b->grid = b->ncu * sc.per_cu;
        b->group = sc.group;
    } else if (tune_cache_lookup(b, sc)) {
        b->block = sc.block;
        b->grid = b->ncu * sc.per_cu;
        b->group = sc.group;
    } else {
        mc_status st = autotune(b, nullptr);
        if (st != MC_OK) {
            batch_free(b);
            return st;
        }
    }
    B_TRY(hipStreamSynchronize(b->stream));
    B_TRY(hipMemsetAsync(b->flags, 0, sizeof(uint32_t), b->stream));
    B_TRY(batch_capture(b));
    B_TRY(hipStreamSynchronize(b->stream));
#undef B_TRY
    *out = b;
    return MC_OK;
}

mc_status mc_expmv_batch_run(mc_batch_t b) {
    if (!b) return MC_ERR_INVALID_ARG;
    HIP_TRY(hipSetDevice(b->dev));
    HIP_TRY(hipEventRecord(b->ev_user, b->user));
    HIP_TRY(hipStreamWaitEvent(b->stream, b->ev_user, 0));
    HIP_TRY(hipEventRecord(b->ev0, b->stream));
    if (b->exec)
        HIP_TRY(hipGraphLaunch(b->exec, b->stream));
    else
        HIP_TRY(batch_launch(b));
    HIP_TRY(hipEventRecord(b->ev1, b->stream));
    HIP_TRY(hipEventRecord(b->ev_done, b->stream));
    HIP_TRY(hipStreamWaitEvent(b->user, b->ev_done, 0));
    b->ran = true;
    return MC_OK;
}

mc_status mc_expmv_batch_sync(mc_batch_t b) {
    if (!b) return MC_ERR_INVALID_ARG;
    HIP_TRY(hipSetDevice(b->dev));
    HIP_TRY(hipMemcpyAsync(b->flag_host, b->flags, sizeof(uint32_t), hipMemcpyDeviceToHost,
                           b->stream));
    HIP_TRY(hipMemsetAsync(b->flags, 0, sizeof(uint32_t), b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    return flags_to_status(*b->flag_host);
}

mc_status mc_expmv_batch_stats(mc_batch_t b, mc_expmv_run_stats *out, mc_batch_schedule *sched) {
    if (!b) return MC_ERR_INVALID_ARG;
    HIP_TRY(hipSetDevice(b->dev));
    if (sched) {
        sched->walkers_per_block = (uint32_t)b->block;
        sched->blocks_per_cu = (uint32_t)(b->grid / (b->ncu > 0 ? b->ncu : 1));
        sched->group = b->group;
        sched->tasks = b->args.ntasks;
    }
    if (!out) return MC_OK;
    memset(out, 0, sizeof(*out));
    if (!b->ran) return MC_OK;
    HIP_TRY(hipEventSynchronize(b->ev1));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, b->ev0, b->ev1));
    // one counter block per class launch (classes without tasks leave theirs unused)
    std::vector<unsigned long long> pc((size_t)b->grid * 2 * b->classes.size());
    HIP_TRY(hipMemcpy(pc.data(), b->counters, sizeof(unsigned long long) * pc.size(),
                      hipMemcpyDeviceToHost));
    unsigned long long ev = 0, ju = 0;
    for (size_t c = 0; c < b->classes.size(); ++c) {
        if (b->classes[c].ntasks == 0) continue;
        for (int i = 0; i < b->grid; ++i) {
            ev += pc[2 * ((size_t)b->grid * c + (size_t)i)];
            ju += pc[2 * ((size_t)b->grid * c + (size_t)i) + 1];
        }
    }
    out->walkers = b->walkers;
    out->events = ev;
    out->jumps = ju;
    out->ms = ms;
    // algorithmic bytes as for a single instance, per instance precision
    double bytes = 0.0;
    double wsum64 = 0.0, wsum32 = 0.0;
    for (const BatchInst &I : b->inst) {
        const double w = (double)I.k * (double)I.nwalk;
        if (I.fp32) wsum32 += w;
        else wsum64 += w;
    }
    // events and jumps are not split by precision; attribute them in proportion
    const double wt = wsum32 + wsum64 > 0 ? wsum32 / (wsum32 + wsum64) : 0.0;
    const double row = 16.0 + 4.0 * wt + 8.0 * (1.0 - wt);
    bytes = row * (double)ev + 12.0 * (double)ju + 4.0 * wsum32 + 8.0 * wsum64;
    out->alg_bytes = bytes;
    return MC_OK;
}

mc_status mc_expmv_batch_set_schedule(mc_batch_t b, const mc_batch_schedule *sched) {
    if (!b || !sched) return MC_ERR_INVALID_ARG;
    const uint32_t wpb = sched->walkers_per_block;
    if (wpb != 64 && wpb != 128 && wpb != 256) return MC_ERR_INVALID_ARG;
    if (sched->blocks_per_cu < 1 || sched->blocks_per_cu > kBatchBlocksPerCuMax) return MC_ERR_INVALID_ARG;
    HIP_TRY(hipSetDevice(b->dev));
    HIP_TRY(hipStreamSynchronize(b->stream));
    b->block = (int)wpb;
    b->grid = b->ncu * (int)sched->blocks_per_cu;
    b->group = sched->group;
    HIP_TRY(batch_capture(b));
    return MC_OK;
}

}  // extern "C"

// ------------------------------------------------------- learned proposal
struct mc_mlp_s {
    int dev = 0;
    hipStream_t stream = nullptr;
    float *w = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr, *loss = nullptr;
    uint16_t *wbf = nullptr;
    float *gpart = nullptr;
    double *gsum = nullptr;              // [kMlpParams + 2] FP64 column sums of gpart
    int gpart_blocks = 0;
    int step = 0;
};

namespace {

hipError_t ensure_rowof(mc_expmv_s *h) {
    if (h->rowof) return hipSuccess;
    hipError_t e = dalloc(&h->rowof, h->nnz);
    if (e != hipSuccess) return e;
    return launch_rowof(h->n, h->rowptr, h->rowof, h->stream);
}

hipError_t ensure_gpart(mc_mlp_s *m, int blocks) {
    if (blocks <= m->gpart_blocks) return hipSuccess;
    hipError_t e = hipStreamSynchronize(m->stream);
    if (e != hipSuccess) return e;
    (void)hipFree(m->gpart);
    m->gpart = nullptr;
    m->gpart_blocks = 0;
    e = dalloc(&m->gpart, (int64_t)blocks * 4 * mlp_grad_stride());
    if (e == hipSuccess) m->gpart_blocks = blocks;
    return e;
}

int64_t gcd64(int64_t a, int64_t b) {
    while (b) {
        const int64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

}  // namespace

extern "C" {

void mc_mlp_destroy(mc_mlp_t m) {
    if (!m) return;
    (void)hipSetDevice(m->dev);
    (void)hipStreamSynchronize(m->stream);
    (void)hipFree(m->w);
    (void)hipFree(m->m);
    (void)hipFree(m->v);
    (void)hipFree(m->grad);
    (void)hipFree(m->loss);
    (void)hipFree(m->wbf);
    (void)hipFree(m->gpart);
    (void)hipFree(m->gsum);
    delete m;
}

mc_status mc_mlp_create(mc_mlp_t *out, uint64_t seed, void *stream) {
    fault_scope_begin();
    if (!out) return MC_ERR_INVALID_ARG;
    *out = nullptr;
    mc_mlp_s *m = new (std::nothrow) mc_mlp_s();
    if (!m) return MC_ERR_NO_MEMORY;
    m->stream = (hipStream_t)stream;
#define M_TRY(expr)                              \
    do {                                         \
        hipError_t e_ = (expr);                  \
        if (e_ != hipSuccess) {                  \
            mc_status s_ = from_hip(e_);         \
            mc_mlp_destroy(m);                   \
            return s_;                           \
        }                                        \
    } while (0)
    M_TRY(hipGetDevice(&m->dev));
    M_TRY(dalloc(&m->w, kMlpParams));
    M_TRY(dalloc(&m->m, kMlpParams));
    M_TRY(dalloc(&m->v, kMlpParams));
    M_TRY(dalloc(&m->grad, kMlpParams));
    M_TRY(dalloc(&m->gsum, kMlpParams + 2));
    M_TRY(dalloc(&m->loss, 1));
    M_TRY(dalloc(&m->wbf, kMlpParams));
    M_TRY(launch_mlp_init(m->w, m->m, m->v, m->wbf, seed, m->stream));
    M_TRY(hipStreamSynchronize(m->stream));
#undef M_TRY
    *out = m;
    return MC_OK;
}

mc_status mc_mlp_get_params(mc_mlp_t m, float *host) {
    if (!m || !host) return MC_ERR_INVALID_ARG;
    HIP_TRY(hipSetDevice(m->dev));
    HIP_TRY(hipStreamSynchronize(m->stream));
    HIP_TRY(hipMemcpy(host, m->w, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost));
    return MC_OK;
}

mc_status mc_mlp_set_params(mc_mlp_t m, const float *host) {
    if (!m || !host) return MC_ERR_INVALID_ARG;
    HIP_TRY(hipSetDevice(m->dev));
    HIP_TRY(hipStreamSynchronize(m->stream));
    HIP_TRY(hipMemcpy(m->w, host, sizeof(float) * kMlpParams, hipMemcpyHostToDevice));
    HIP_TRY(hipMemset(m->m, 0, sizeof(float) * kMlpParams));
    HIP_TRY(hipMemset(m->v, 0, sizeof(float) * kMlpParams));
    HIP_TRY(launch_params_bf16(m->w, m->wbf, m->stream));
    HIP_TRY(hipStreamSynchronize(m->stream));
    m->step = 0;
    return MC_OK;
}

mc_status mc_mlp_features(mc_expmv_t h, const void *v, float *feats) {
    fault_scope_begin();
    if (!h || h->stencil || !v || (h->n > 0 && !feats)) return MC_ERR_INVALID_ARG;
    HIP_TRY(hipSetDevice(h->dev));
    double *raw = nullptr, *stats = nullptr;
    HIP_TRY(dalloc(&raw, 4 * h->n));
    hipError_t e = dalloc(&stats, kFeatStatsDoubles);
    if (e == hipSuccess)
        e = launch_features(h->n, h->rowptr, h->col, h->val, h->plain.rows, h->plain.r, v,
                            h->opts.weight_prec == MC_FP32, raw, stats, feats, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    (void)hipFree(raw);
    (void)hipFree(stats);
    return from_hip(e);
}

mc_status mc_mlp_log_h(mc_expmv_t h, const double *est, const double *se, int64_t n_walkers,
                       float *lh) {
    if (!h || h->stencil || !est || !se || !lh || n_walkers < 2) return MC_ERR_INVALID_ARG;
    HIP_TRY(hipSetDevice(h->dev));
    HIP_TRY(launch_log_h(h->n, est, se, (double)n_walkers, lh, h->stream));
    return MC_OK;
}

mc_status mc_mlp_forward(mc_mlp_t m, mc_expmv_t h, const float *feats, float *bias) {
    fault_scope_begin();
    if (!m || !h || h->stencil || !feats || (h->nnz > 0 && !bias)) return MC_ERR_INVALID_ARG;
    HIP_TRY(hipSetDevice(h->dev));
    HIP_TRY(hipStreamSynchronize(m->stream));
    HIP_TRY(ensure_rowof(h));
    HIP_TRY(launch_net_forward(m->wbf, feats, h->rowof, h->col, h->val, h->plain.r, h->nnz, bias,
                               h->stream));
    return MC_OK;
}

mc_status mc_mlp_gradient(mc_mlp_t m, mc_expmv_t h, const float *feats, const float *lh,
                          int64_t p0, int64_t p1, float *grad, float *loss) {
    fault_scope_begin();
    if (!m || !h || h->stencil || !feats || !lh || !grad) return MC_ERR_INVALID_ARG;
    if (p0 < 0 || p1 > h->nnz || p1 <= p0) return MC_ERR_INVALID_ARG;
    HIP_TRY(hipSetDevice(h->dev));
    HIP_TRY(hipStreamSynchronize(m->stream));
    HIP_TRY(ensure_rowof(h));
    const int64_t tile0 = p0 / 16;
    const int64_t ntile = (p1 - tile0 * 16 + 15) / 16;
    const int blocks = mlp_blocks(ntile, kMlpTrainBlocks);
    HIP_TRY(ensure_gpart(m, blocks));
    HIP_TRY(launch_net_gradient(m->wbf, feats, h->rowof, h->col, h->val, h->plain.r, lh, p0, p1,
                                tile0, ntile, 1, (int64_t)1 << 62, blocks, m->gpart, m->gsum, grad,
                                loss,
                                h->stream));
    return MC_OK;
}

mc_status mc_mlp_adam_step(mc_mlp_t m, const float *grad, float lr) {
    if (!m || !grad || !(lr > 0.0f)) return MC_ERR_INVALID_ARG;
    HIP_TRY(hipSetDevice(m->dev));
    m->step += 1;
    HIP_TRY(launch_adam(grad, m->w, m->m, m->v, m->wbf, lr, m->step, m->stream));
    return MC_OK;
}

mc_status mc_mlp_train(mc_mlp_t m, mc_expmv_t h, const float *feats, const float *lh,
                       int32_t steps, int64_t batch, float lr, float *loss_host) {
    fault_scope_begin();
    if (!m || !h || h->stencil || !feats || !lh || steps < 1 || batch < 16 || !(lr > 0.0f))
        return MC_ERR_INVALID_ARG;
    if (h->nnz == 0) return MC_OK;
    HIP_TRY(hipSetDevice(h->dev));
    HIP_TRY(hipStreamSynchronize(m->stream));
    HIP_TRY(ensure_rowof(h));
    const int64_t tmod = (h->nnz + 15) / 16;
    int64_t ntile = (batch + 15) / 16;
    if (ntile > tmod) ntile = tmod;
    // visit tiles in the order T_k = (k * stride) mod tmod with stride coprime
    // to tmod, so every batch spreads over the whole matrix
    int64_t stride = (int64_t)(0.6180339887498949 * (double)tmod) | 1;
    while (stride > 1 && gcd64(stride, tmod) != 1) stride += 2;
    if (stride < 1 || stride >= tmod) stride = 1;
    const int blocks = mlp_blocks(ntile, kMlpTrainBlocks);
    HIP_TRY(ensure_gpart(m, blocks));
    float *dloss = nullptr;
    HIP_TRY(dalloc(&dloss, steps));
    mc_status st = MC_OK;
    for (int32_t s = 0; s < steps && st == MC_OK; ++s) {
        const int64_t tile0 = ((int64_t)s * ntile % tmod) * stride % tmod;
        hipError_t e = launch_net_gradient(m->wbf, feats, h->rowof, h->col, h->val, h->plain.r,
                                           lh, 0, h->nnz, tile0, ntile, stride, tmod, blocks,
                                           m->gpart, m->gsum, m->grad, dloss + s, h->stream);
        if (e == hipSuccess) {
            m->step += 1;
            e = launch_adam(m->grad, m->w, m->m, m->v, m->wbf, lr, m->step, h->stream);
        }
        st = from_hip(e);
    }
    if (st == MC_OK && loss_host)
        st = from_hip(hipMemcpy(loss_host, dloss, sizeof(float) * (size_t)steps,
                                hipMemcpyDeviceToHost));
    (void)hipStreamSynchronize(h->stream);
    (void)hipFree(dloss);
    return st;
}

void mc_learn_default_opts(mc_learn_opts *o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->struct_size = sizeof(mc_learn_opts);
    o->pilot_walkers = 256;
    o->steps = 400;
    o->batch = 1 << 16;
    o->lr = 3e-3f;
    o->seed = 1;
}

mc_status mc_expmv_learn_proposal(mc_expmv_t h, const void *v, const mc_learn_opts *opts,
                                  mc_learn_report *rep) {
    fault_scope_begin();
    if (!h || h->stencil || !v) return MC_ERR_INVALID_ARG;
    mc_learn_opts o;
    mc_learn_default_opts(&o);
    if (opts) {
        if (opts->struct_size != sizeof(mc_learn_opts)) return MC_ERR_INVALID_ARG;
        o = *opts;
    }
    if (o.pilot_walkers < 2 || o.steps < 1 || o.batch < 16 || !(o.lr > 0.0f))
        return MC_ERR_INVALID_ARG;
    if (h->opts.mode != MC_EXACT) return MC_ERR_INVALID_ARG;
    HIP_TRY(hipSetDevice(h->dev));
    if (rep) memset(rep, 0, sizeof(*rep));
    const int64_t n = h->n;
    double *est = nullptr, *se = nullptr;
    float *lh = nullptr, *feats = nullptr, *bias = nullptr;
    mc_mlp_t net = nullptr;
    hipEvent_t t0 = nullptr, t1 = nullptr, t2 = nullptr;
    std::vector<float> losses((size_t)o.steps);
    mc_status st = from_hip(dalloc(&est, n));
    if (st == MC_OK) st = from_hip(dalloc(&se, n));
    if (st == MC_OK) st = from_hip(dalloc(&lh, n));
    if (st == MC_OK) st = from_hip(dalloc(&feats, 4 * n));
    if (st == MC_OK) st = from_hip(dalloc(&bias, h->nnz));
    if (st == MC_OK) st = from_hip(hipEventCreate(&t0));
    if (st == MC_OK) st = from_hip(hipEventCreate(&t1));
    if (st == MC_OK) st = from_hip(hipEventCreate(&t2));
    // 1. plain pilot over every node: per-node second moments of the plain walk
    //    (without first-jump conditioning, whose second moments differ)
    const int32_t cond = h->opts.cond_first_jump;
    h->opts.cond_first_jump = 0;
    if (st == MC_OK) st = from_hip(hipEventRecord(t0, h->stream));
    if (st == MC_OK)
        st = run_walk(h, v, nullptr, n, o.pilot_walkers, est, se, false, 0, 0, nullptr, nullptr,
                      nullptr, nullptr);
    h->opts.cond_first_jump = cond;
    if (st == MC_OK) st = mc_expmv_sync(h);
    if (st == MC_OK) st = mc_mlp_log_h(h, est, se, o.pilot_walkers, lh);
    if (st == MC_OK) st = mc_mlp_features(h, v, feats);
    if (st == MC_OK) st = from_hip(hipEventRecord(t1, h->stream));
    // 2. train the network on the GPU
    if (st == MC_OK) st = mc_mlp_create(&net, o.seed, h->stream);
    if (st == MC_OK) st = mc_mlp_train(net, h, feats, lh, o.steps, o.batch, o.lr, losses.data());
    // 3. inference over every edge, install the tilted tables
    if (st == MC_OK) st = mc_mlp_forward(net, h, feats, bias);
    if (st == MC_OK) st = from_hip(hipEventRecord(t2, h->stream));
    if (st == MC_OK) st = from_hip(hipStreamSynchronize(h->stream));
    if (st == MC_OK) st = mc_expmv_set_proposal(h, bias);
    if (st == MC_OK && o.params_out) st = mc_mlp_get_params(net, o.params_out);
    if (st == MC_OK && rep) {
        float a = 0.0f, b = 0.0f;
        (void)hipEventElapsedTime(&a, t0, t1);
        (void)hipEventElapsedTime(&b, t1, t2);
        rep->pilot_ms = a;
        rep->train_ms = b;
        rep->initial_loss = losses.front();
        rep->final_loss = losses.back();
        rep->steps = o.steps;
    }
    mc_mlp_destroy(net);
    (void)hipFree(est);
    (void)hipFree(se);
    (void)hipFree(lh);
    (void)hipFree(feats);
    (void)hipFree(bias);
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    if (t2) (void)hipEventDestroy(t2);
    return st;
}

}  // extern "C"

// ------------------------------------------------------------ forward estimator
namespace {

// A == A^T (summed duplicates compared exactly), checked once per handle.
mc_status check_symmetric(mc_expmv_s *h) {
    if (h->sym_state >= 0) return h->sym_state ? MC_OK : MC_ERR_NOT_SYMMETRIC;
    HIP_TRY(ensure_rowof(h));
    uint32_t *flag = nullptr;
    HIP_TRY(dalloc(&flag, 1));
    uint32_t f = 0;
    hipError_t e = hipMemcpyAsync(flag, &f, sizeof(f), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess)
        e = launch_check_symmetric(h->nnz, h->rowptr, h->rowof, h->col, h->val, flag, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&f, flag, sizeof(f), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    (void)hipFree(flag);
    HIP_TRY(e);
    h->sym_state = f ? 0 : 1;
    return f ? MC_ERR_NOT_SYMMETRIC : MC_OK;
}

mc_status run_forward(mc_expmv_s *h, const void *v, int64_t w0, int64_t nwalk, double *acc1,
                      double *acc2, double *sum_out, bool trace, int32_t *ts, int32_t *te,
                      uint32_t *tev, uint32_t *tju, double *ty) {
    if (!v || (!acc1 && !sum_out) || (!acc1 && acc2) || nwalk < 1 || nwalk > 0xFFFFFFFFll ||
        w0 < 0 || w0 + nwalk > 0x100000000ll)
        return MC_ERR_INVALID_ARG;
    HIP_TRY(hipSetDevice(h->dev));
    mc_status st = check_symmetric(h);
    if (st != MC_OK) return st;
    const bool fp32 = h->opts.weight_prec == MC_FP32;
    const int64_t n = h->n;
    if (n > 0 && !h->fwd_cdf) {
        HIP_TRY(dalloc(&h->fwd_abs, n));
        HIP_TRY(dalloc(&h->fwd_sign, n));
        HIP_TRY(dalloc(&h->fwd_cdf, n));
        HIP_TRY(dalloc(&h->fwd_guide, guide_cells(n) + 1));
        size_t bytes = 0;
        HIP_TRY(launch_fwd_cdf(n, v, fp32, h->fwd_abs, h->fwd_sign, h->fwd_cdf, h->fwd_guide, nullptr, bytes,
                               h->stream));
        HIP_TRY(dev_malloc(&h->fwd_temp, bytes > 0 ? bytes : 1));
        h->fwd_temp_bytes = bytes;
    }
    const int64_t chunks = (nwalk + kFwdChunk - 1) / kFwdChunk;
    if (chunks * 3 > h->fwd_part_cap) {
        HIP_TRY(hipStreamSynchronize(h->stream));
        (void)hipFree(h->fwd_part);
        h->fwd_part = nullptr;
        h->fwd_part_cap = 0;
        HIP_TRY(dalloc(&h->fwd_part, chunks * 3));
        h->fwd_part_cap = chunks * 3;
    }
    HIP_TRY(hipEventRecord(h->ev0, h->stream));
    if (n > 0) {
        size_t bytes = h->fwd_temp_bytes;
        HIP_TRY(launch_fwd_cdf(n, v, fp32, h->fwd_abs, h->fwd_sign, h->fwd_cdf, h->fwd_guide, h->fwd_temp, bytes,
                               h->stream));
    }
    FwdArgs a{};
    fill_inst(h, v, false, a.P);
    a.P.hot = 0;
    if (n > 0 && !h->fwd_rows) {
        HIP_TRY(dalloc(&h->fwd_rows, n));
        HIP_TRY(launch_fwd_rows(n, a.P, h->fwd_rows, h->stream));
    }
    a.frows = h->fwd_rows;
    a.n = n;
    a.nwalk = nwalk;
    a.w0 = w0;
    a.chunks = chunks;
    a.cdf = h->fwd_cdf;
    a.absv = h->fwd_abs;
    a.vsign = h->fwd_sign;
    a.guide = h->fwd_guide;
    a.gcells = guide_cells(n);
    a.acc1 = acc1;
    a.acc2 = acc2;
    a.part = h->fwd_part;
    a.counters = h->counters;
    a.flags = h->flags;
    a.t_start = ts;
    a.t_end = te;
    a.t_ev = tev;
    a.t_ju = tju;
    a.t_y = ty;
    HIP_TRY(launch_forward(a, h->opts.mode, fp32, trace, sum_out, h->stream));
    HIP_TRY(hipEventRecord(h->ev1, h->stream));
    h->ran = true;
    h->last_walkers = (uint64_t)nwalk;
    h->last_walkers_dev = nullptr;
    h->last_grid = forward_grid(chunks);
    h->last_fp32 = fp32;
    h->last_prop = false;
    h->last_fwd = true;
    return MC_OK;
}

}  // namespace

extern "C" {

mc_status mc_expmv_forward(mc_expmv_t h, const void *v, int64_t n_walkers, double *est,
                           double *stderr_, double *sum_out) {
    fault_scope_begin();
    if (!h || h->stencil) return MC_ERR_INVALID_ARG;
    return run_forward(h, v, 0, n_walkers, est, stderr_, sum_out, false, nullptr, nullptr,
                       nullptr, nullptr, nullptr);
}

mc_status mc_expmv_forward_trace(mc_expmv_t h, const void *v, int64_t w0, int64_t count,
                                 int32_t *start, int32_t *end, uint32_t *events, uint32_t *jumps,
                                 double *y) {
    fault_scope_begin();
    if (!h || h->stencil || !start || !end || !events || !jumps || !y) return MC_ERR_INVALID_ARG;
    if (!h->fwd_acc && h->n > 0) HIP_TRY(dalloc(&h->fwd_acc, h->n));
    return run_forward(h, v, w0, count, h->fwd_acc, nullptr, nullptr, true, start, end, events,
                       jumps, y);
}

}  // extern "C"
