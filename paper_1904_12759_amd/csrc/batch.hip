// Batched walks: many instances (each its own matrix, horizon, weight mode,
// precision, vector and request) in one persistent launch.
//
// The tasks of all instances form one index space (instance i owns tasks
// task_begin[i] .. task_begin[i+1]-1, each an (entry, chunk) exactly as in the
// single-instance kernel).  Waves either stride through it statically or take
// `group` consecutive tasks at a time from a global counter; which one is
// faster depends on the mix and is left to the autotuner.  Each task runs the
// same run_group as the single-instance kernel and writes its own outputs, so
// results do not depend on the schedule and equal separate per-instance runs.
#include "walk_task.hpp"

namespace mc {
namespace {


static_assert(sizeof(BatchInst) % 4 == 0, "the instance record is copied as 32-bit words");

// One task of a class's index space: instance, then (entry group, chunk).
template <int MODE, bool FP32>
__device__ __forceinline__ void do_task(const BatchArgs &a, const int64_t *tb, int64_t task,
                                        unsigned char *lds, unsigned long long &my_events,
                                        unsigned long long &my_jumps, uint32_t &err) {
    // instance owning this task: the last i with tb[i] <= task
    int lo = 0, hi = a.ninst - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tb[mid] <= task) lo = mid;
        else hi = mid - 1;
    }
    // the instance is the same for the whole wave.  Its record arrives through
    // vector loads (the kernel stores to global memory, so the compiler does not
    // use scalar loads for it); every word is moved to a scalar register at once,
    // so the instance holds no vector registers during the walk (111 -> 100)
    lo = __builtin_amdgcn_readfirstlane(lo);
    BatchInst I;
    {
        const uint32_t *src = reinterpret_cast<const uint32_t *>(a.inst + lo);
        uint32_t *dst = reinterpret_cast<uint32_t *>(&I);
#pragma unroll
        for (int i = 0; i < (int)(sizeof(BatchInst) / 4); ++i)
            dst[i] = __builtin_amdgcn_readfirstlane(src[i]);
    }
    const int64_t local = task - tb[lo];
    const int64_t grp = local / I.chunks;
    const int64_t c = local - grp * I.chunks;
    const int64_t e_first = grp * (int64_t)I.group;
    const int64_t left = I.k - e_first;
    const uint32_t G = (uint32_t)(left < (int64_t)I.group ? left : (int64_t)I.group);
    const int64_t chunk = chunk_walkers(FP32);
    const int64_t wbase = c * chunk;
    const int64_t rem = I.nwalk - wbase;
    const uint32_t cnt = (uint32_t)(rem < chunk ? rem : chunk);
    const GroupOut out{I.est, I.se, a.part + I.part_off, e_first, I.chunks, e_first * I.chunks + c};
    TraceOut none;
    // instances of one class may differ in their slot layout: FAT = 2 tests I.P.fat
    run_group<MODE, FP32, false, false, false, false, false, 2>(
        I.P, I.idx, I.n, G, (uint32_t)wbase, cnt, none, out,
        *reinterpret_cast<GroupLds<typename WeightT<FP32>::T> *>(lds), my_events, my_jumps, err);
}

// Persistent kernel over the tasks of one class.  Dynamic LDS: one task
// scratch per wave, then the class's task offsets (ninst of them: sized to the
// class, so that a small batch leaves the LDS to more resident waves).
template <int MODE, bool FP32>
__global__ __launch_bounds__(256) void k_walk_batched(BatchArgs a) {
    extern __shared__ __align__(16) unsigned char dyn_lds[];
    int64_t *sh_tb = reinterpret_cast<int64_t *>(
        dyn_lds + (size_t)(blockDim.x / WAVE) * sizeof(GroupLds<typename WeightT<FP32>::T>));
    __shared__ unsigned long long sh_count[256 / WAVE][2];
    for (int i = threadIdx.x; i < a.ninst; i += blockDim.x) sh_tb[i] = a.inst[i].task_begin - a.task0;
    __syncthreads();
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = threadIdx.x / WAVE;
    unsigned char *lds = dyn_lds + (size_t)wave * sizeof(GroupLds<typename WeightT<FP32>::T>);
    unsigned long long my_events = 0, my_jumps = 0;
    uint32_t err = 0;
    // one call site of do_task for both schedules (two inlined copies cost
    // registers): static stride over the tasks, or grabs of `group` tasks
    const bool dynamic = a.group != 0;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / WAVE;
    int64_t task = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * blockDim.x + threadIdx.x) / WAVE));
    int64_t end = task;               // dynamic: end of the current grab
    for (;;) {
        if (dynamic && task >= end) {
            unsigned long long base = 0;
            if (lane == 0) base = atomicAdd(a.queue, (unsigned long long)a.group);
            task = (int64_t)((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)base) |
                             ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(base >> 32))
                              << 32));
            end = task + a.group < a.ntasks ? task + a.group : a.ntasks;
        }
        if (task >= a.ntasks) break;
        do_task<MODE, FP32>(a, sh_tb, task, lds, my_events, my_jumps, err);
        task += dynamic ? 1 : nwaves;
    }
    for (int off = 1; off < WAVE; off <<= 1) err |= __shfl_xor(err, off, WAVE);
    if (err && lane == 0) atomicOr(a.flags, err);
    if (lane == 0) {
        sh_count[wave][0] = my_events;
        sh_count[wave][1] = my_jumps;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long ev = 0, ju = 0;
        for (int w = 0; w < (int)(blockDim.x / WAVE); ++w) {
            ev += sh_count[w][0];
            ju += sh_count[w][1];
        }
        a.counters[2 * blockIdx.x] = ev;
        a.counters[2 * blockIdx.x + 1] = ju;
    }
}

// Reset the task counter from inside a captured graph (a kernel node, not a
// memset node).
__global__ void k_reset_queue(unsigned long long *queue) { *queue = 0ull; }

// Merge chunk partials of every entry that spans several chunks, for all
// instances: instance i owns the finalize threads fin_begin[i] .. fin_begin[i]
// + k * fin_lanes(chunks) - 1 (fin_begin[i] a multiple of 64 and of its lane
// count, so that a wave never spans two instances and a group never two
// blocks), fin_lanes(chunks) of them per entry, exactly as in k_finalize.
__global__ __launch_bounds__(kFinLanesMax) void k_finalize_batched(BatchArgs a) {
    __shared__ double lds[kFinLanesMax / WAVE][3];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const BatchInst *I = nullptr;
    if (t < a.nfin) {   // whole waves: nfin is a multiple of 64
        int lo = 0, hi = a.ninst - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.fin_begin[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        I = &a.inst[lo];
    }
    // threads past the instances, or in the padding after one, join the block's
    // barrier with empty groups of their wave's lane count
    const int64_t chunks = I && I->chunks > 1 ? I->chunks : 0;
    const uint32_t L = chunks ? fin_lanes(chunks) : 1;
    const int64_t local = I ? t - a.fin_begin[I - a.inst] : 0;
    const int64_t e = local / L;
    const uint32_t sub = (uint32_t)(local - e * L);
    const bool valid = chunks && e < I->k;
    double n, mean, m2;
    fin_merge(valid ? a.part + I->part_off + e * chunks * 3 : nullptr, valid ? chunks : 0, L, sub, lds,
              n, mean, m2);
    if (valid && sub == 0) {
        I->est[e] = mean;
        if (I->se) I->se[e] = n > 1.0 ? sqrt(m2 / (n - 1.0) / n) : 0.0;
    }
}

}  // namespace

hipError_t launch_batch(const BatchArgs &base, const BatchClass *classes, int nclass, int block,
                        int grid, hipStream_t s) {
    for (int c = 0; c < nclass; ++c) {
        const BatchClass &C = classes[c];
        if (C.ntasks == 0) continue;
        BatchArgs a = base;
        a.inst = base.inst + C.inst0;
        a.ninst = C.ninst;
        a.ntasks = C.ntasks;
        a.task0 = C.task0;
        a.counters = base.counters + 2 * (size_t)grid * (size_t)c;
        if (a.group != 0) {
            hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(1), 0, s, a.queue);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        const size_t lds =
            (size_t)(block / WAVE) * (C.fp32 ? sizeof(GroupLds<float>) : sizeof(GroupLds<double>)) +
            sizeof(int64_t) * (size_t)C.ninst;
#define MC_BATCH(M, F) hipLaunchKernelGGL((k_walk_batched<M, F>), dim3((unsigned)grid), dim3(block), lds, s, a)
        switch (C.mode * 2 + (C.fp32 ? 1 : 0)) {
            case MC_EXACT * 2: MC_BATCH(MC_EXACT, false); break;
            case MC_EXACT * 2 + 1: MC_BATCH(MC_EXACT, true); break;
            case MC_STRANG * 2: MC_BATCH(MC_STRANG, false); break;
            case MC_STRANG * 2 + 1: MC_BATCH(MC_STRANG, true); break;
            case MC_LIE * 2: MC_BATCH(MC_LIE, false); break;
            case MC_LIE * 2 + 1: MC_BATCH(MC_LIE, true); break;
            default: return hipErrorInvalidValue;
        }
#undef MC_BATCH
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (base.nfin > 0) {
        const int fb = (int)kFinLanesMax;
        hipLaunchKernelGGL(k_finalize_batched, dim3((unsigned)((base.nfin + fb - 1) / fb)), dim3(fb),
                           0, s, base);
        return hipGetLastError();
    }
    return hipSuccess;
}

}  // namespace mc
