// The walk: continuous-time Markov-chain paths through the indices of A and
// the multiplicative functional of Theorem 1 (paper Sec. 2-3, Algorithm 1).
//
// Work decomposition.  A task is (group of G consecutive entries, chunk c):
// the walkers with ordinals c*C .. min(M, (c+1)*C)-1 of each entry, with
// C = 1024 (FP32 weights) or 512 (FP64) and G = min(64, C/M) so that a task
// holds about C walkers.  One wavefront
// owns a task and runs it in two phases (run_group): the first event of every
// walker, which for most start nodes already decides that the walker never
// leaves, then complete walks with lane refill for the others.  Paths depend
// only on the Philox counter (event, ordinal, start node, instance), never on
// the lane or the task shape.
//
// Statistics.  Every finished walker's value goes to the LDS slot of its
// position in the entry's ordinal-ordered list of jumpers; each entry's mean and sum of squared deviations come from a
// two-pass sum over its slots in a fixed order plus the closed-form
// contribution of its walkers that never jump, and entries spread over several
// chunks are merged in a fixed order (Chan, Golub, LeVeque).
#include <math.h>

#include "walk_task.hpp"

namespace mc {

namespace {

// Entries (or, with idx == null, every node) of one instance.  Event and
// jump totals are reduced per block and written to counters[2*block] without
// atomics (same-address atomics from every wave serialise across the chip).
// Dynamic LDS: one GroupLds per wave.
template <int MODE, bool FP32, bool PROP, bool TRACE, bool LOC, bool COND, bool RESORT, int FAT,
          bool QMC = false, bool STENCIL = false>
__global__ __launch_bounds__(256) void k_walk(WalkArgs a) {
    using WT = typename WeightT<FP32>::T;
    extern __shared__ __align__(16) unsigned char dyn_lds[];
    __shared__ unsigned long long sh_count[256 / WAVE][2];
    const int nw = blockDim.x / WAVE;
    GroupLds<WT, COND> &L = reinterpret_cast<GroupLds<WT, COND> *>(dyn_lds)[threadIdx.x / WAVE];
    // hot rows: LDS copies of rows[0 .. hot) and d[0 .. hot) after the wave scratch
    InstArgs P = a.P;
    if (LOC && P.hot) {
        RowRec *lr = reinterpret_cast<RowRec *>(dyn_lds + nw * sizeof(GroupLds<WT, COND>));
        WT *ld = reinterpret_cast<WT *>(lr + P.hot);
        const WT *gd = FP32 ? (const WT *)(const void *)a.P.d32 : (const WT *)(const void *)a.P.d64;
        for (uint32_t k = threadIdx.x; k < P.hot; k += blockDim.x) {
            lr[k] = a.P.rows[k];
            ld[k] = gd[k];
        }
        __syncthreads();
        P.lrows = lr;
        P.ld = ld;
    }
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t wave_id = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / WAVE;
    unsigned long long my_events = 0, my_jumps = 0;
    uint32_t err = 0;
    const int64_t ntasks = a.slots_dev ? *a.slots_dev : a.ntasks;
    const int64_t var_slots = a.slots_dev ? ntasks : a.var_slots;
    for (int64_t task = wave_id; task < ntasks; task += nwaves) {
        int64_t e_first, c, chunks, nwalk, pbase;
        uint32_t G;
        GroupOut out{a.est, a.se, a.part, 0, 0, 0};
        if (a.var_task) {
            // entries with their own walker counts: the task is `group` consecutive
            // chunk slots, decoded per slot inside run_group
            const int64_t s0 = task * (int64_t)a.group;
            const int64_t left = var_slots - s0;
            G = (uint32_t)(left < (int64_t)a.group ? left : (int64_t)a.group);
            out.var_task = a.var_task;
            out.var_nwalk = a.var_nwalk;
            out.s0 = s0;
            out.k = a.k;
            c = 0;
            chunks = 0;
            nwalk = 0;
            e_first = 0;
            pbase = 0;
        } else {
            const int64_t grp = task / a.chunks;
            c = task - grp * a.chunks;
            e_first = grp * (int64_t)a.group;
            const int64_t left = a.k - e_first;
            G = (uint32_t)(left < (int64_t)a.group ? left : (int64_t)a.group);
            chunks = a.chunks;
            nwalk = a.nwalk;
            pbase = e_first * chunks + c;
            out.e_first = e_first;
            out.chunks = chunks;
            out.pbase = pbase;
        }
        const int64_t wbase = c * (int64_t)a.chunk;
        const int64_t rem = nwalk - wbase;
        const uint32_t cnt = (uint32_t)(rem < (int64_t)a.chunk ? rem : (int64_t)a.chunk);
        TraceOut tr = a.trace;
        tr.base = wbase;
        run_group<MODE, FP32, PROP, TRACE, LOC, COND, RESORT, FAT, QMC, STENCIL>(P, a.idx, a.n, G, (uint32_t)(a.w0 + wbase), cnt, tr,
                                           out, L, my_events, my_jumps, err);
    }
    for (int off = 1; off < WAVE; off <<= 1) err |= __shfl_xor(err, off, WAVE);
    if (err && lane == 0) atomicOr(a.flags, err);
    const int wave = threadIdx.x / WAVE;
    if (lane == 0) {
        sh_count[wave][0] = my_events;
        sh_count[wave][1] = my_jumps;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long e = 0, j = 0;
        for (int w = 0; w < (int)(blockDim.x / WAVE); ++w) {
            e += sh_count[w][0];
            j += sh_count[w][1];
        }
        a.counters[2 * blockIdx.x] = e;
        a.counters[2 * blockIdx.x + 1] = j;
    }
}

}  // namespace

// Merge the chunk partials of every entry in a fixed order: fin_lanes(chunks)
// lanes per entry (the block is a multiple of them; every thread takes part).
__global__ __launch_bounds__(kFinLanesMax) void k_finalize(int64_t k, int64_t chunks,
                                                           const double *__restrict__ part,
                                                           double *__restrict__ est, double *__restrict__ se) {
    __shared__ double lds[kFinLanesMax / WAVE][3];
    const uint32_t L = fin_lanes(chunks);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t e = t / L;
    const uint32_t sub = (uint32_t)(t - e * L);
    const bool valid = e < k;
    double n, mean, m2;
    fin_merge(valid ? part + e * chunks * 3 : nullptr, valid ? chunks : 0, L, sub, lds, n, mean, m2);
    if (valid && sub == 0) {
        est[e] = mean;
        if (se) se[e] = n > 1.0 ? sqrt(m2 / (n - 1.0) / n) : 0.0;
    }
}

// Chunk partials of entries with their own walker counts (every entry, one chunk
// or many, leaves partials): one block per entry, fin_lanes(chunks of the entry)
// of its threads merging exactly as k_finalize does, and a single partial is
// copied as it is, so results equal those of a run with that walker count.
__global__ __launch_bounds__(kFinLanesMax) void k_finalize_var(int64_t k, const int64_t *__restrict__ var_task,
                                                               const double *__restrict__ part,
                                                               double *__restrict__ est, double *__restrict__ se) {
    __shared__ double lds[kFinLanesMax / WAVE][3];
    const int64_t e = blockIdx.x;
    const int64_t chunks = var_task[e + 1] - var_task[e];
    const uint32_t L = fin_lanes(chunks);
    const bool valid = threadIdx.x < L;   // threads past L form empty groups
    double n, mean, m2;
    fin_merge(valid ? part + 3 * var_task[e] : nullptr, valid ? chunks : 0, L, threadIdx.x % L, lds,
              n, mean, m2);
    if (threadIdx.x == 0) {
        est[e] = mean;
        if (se) se[e] = n > 1.0 ? sqrt(m2 / (n - 1.0) / n) : 0.0;
    }
}

// Standard errors of lattice (randomised quasi-Monte Carlo) estimates from the R
// replicate means of an entry, one replicate per chunk partial (count n_c, mean
// m_c): se^2 = R/(R-1) sum_c (n_c/N)^2 (m_c - est)^2, N = sum_c n_c, after the
// finalize kernel has written est.  One wavefront per entry: lane l takes chunks
// l, l + 64, ... in order, then the wave's fixed tree.  Entries with a single
// replicate keep the i.i.d. standard error.  part + 3 * first[e] holds entry e's
// R = first[e+1] - first[e] partials (first null: R = chunks for every entry).
__global__ __launch_bounds__(256) void k_qmc_stderr(int64_t k, int64_t chunks,
                                                    const int64_t *__restrict__ first,
                                                    const double *__restrict__ part,
                                                    const double *__restrict__ est,
                                                    double *__restrict__ se) {
    const int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const int lane = threadIdx.x & (WAVE - 1);
    if (e >= k) return;                       // whole waves leave together
    const int64_t c0 = first ? first[e] : e * chunks;
    const int64_t R = first ? first[e + 1] - first[e] : chunks;
    if (R < 2) return;
    const double *p = part + 3 * c0;
    double nsum = 0.0;
    for (int64_t c = lane; c < R; c += WAVE) nsum += p[3 * c];
    nsum = wave_sum_f64(nsum);
    const double mean = est[e];
    double acc = 0.0;
    for (int64_t c = lane; c < R; c += WAVE) {
        const double wc = p[3 * c] / nsum;
        const double dm = p[3 * c + 1] - mean;
        acc += wc * wc * dm * dm;
    }
    acc = wave_sum_f64(acc);
    if (lane == 0) se[e] = sqrt(acc * (double)R / (double)(R - 1));
}

__global__ void k_math_eval(int fn, const double *__restrict__ x, double *__restrict__ y,
                            int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double a = x[i];
    y[i] = fn == 0   ? log_unit(a)
           : fn == 1 ? exp_f64(a)
           : fn == 2 ? one_minus_exp_neg(a)
                     : (double)exp_f32((float)a);
}

hipError_t launch_math_eval(int fn, const double *x, double *y, int64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int64_t grid = (n + 255) / 256;
    if (grid > 0x7FFFFFFF) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_math_eval, dim3((unsigned)grid), dim3(256), 0, s, fn, x, y, n);
    return hipGetLastError();
}

namespace {

int walk_grid(int64_t ntasks, int block) {
    const int64_t waves_per_block = block / WAVE;
    int64_t grid = (ntasks + waves_per_block - 1) / waves_per_block;
    if (grid > kMaxWalkGrid) grid = kMaxWalkGrid;
    if (grid < 1) grid = 1;
    return (int)grid;
}

template <int MODE, bool FP32, bool PROP, bool TRACE, int FAT>
void launch_shape(const WalkArgs &a, dim3 grid, int block, size_t lds, hipStream_t s) {
    // the randomised-lattice first event has kernels of its own (plain layout, no
    // conditioning: checked at create), so that the others keep their code
    if (a.P.qmc) {
        hipLaunchKernelGGL((k_walk<MODE, FP32, PROP, TRACE, false, false, false, FAT, true>), grid, dim3(block), lds, s, a);
        return;
    }
    // the matrix-free stencil walk (plain proposal, input order: checked at create)
    if constexpr (!PROP && FAT != 1) {
        if (a.P.stail) {
            hipLaunchKernelGGL((k_walk<MODE, FP32, false, TRACE, false, false, false, 0, false, true>), grid, dim3(block), lds, s, a);
            return;
        }
    }
    // the wave re-sort has kernels of its own, so that it costs the others no registers
    if (a.P.perm && a.P.resort) {
        if (a.cond) hipLaunchKernelGGL((k_walk<MODE, FP32, PROP, TRACE, true, true, true, FAT>), grid, dim3(block), lds, s, a);
        else hipLaunchKernelGGL((k_walk<MODE, FP32, PROP, TRACE, true, false, true, FAT>), grid, dim3(block), lds, s, a);
    } else if (a.P.perm) {
        if (a.cond) hipLaunchKernelGGL((k_walk<MODE, FP32, PROP, TRACE, true, true, false, FAT>), grid, dim3(block), lds, s, a);
        else hipLaunchKernelGGL((k_walk<MODE, FP32, PROP, TRACE, true, false, false, FAT>), grid, dim3(block), lds, s, a);
    } else {
        if (a.cond) hipLaunchKernelGGL((k_walk<MODE, FP32, PROP, TRACE, false, true, false, FAT>), grid, dim3(block), lds, s, a);
        else hipLaunchKernelGGL((k_walk<MODE, FP32, PROP, TRACE, false, false, false, FAT>), grid, dim3(block), lds, s, a);
    }
}

template <int MODE, bool FP32, bool PROP, bool TRACE>
hipError_t launch_t(const WalkArgs &a, int block, hipStream_t s) {
    using WT = typename WeightT<FP32>::T;
    // a task's walkers must fit its LDS value slots
    if (a.chunk != GroupLds<WT>::C || a.group == 0 || a.group > kGroupMax)
        return hipErrorInvalidValue;
    const size_t task_lds = a.cond ? sizeof(GroupLds<WT, true>) : sizeof(GroupLds<WT, false>);
    const size_t lds = (size_t)(block / WAVE) * task_lds +
                       (size_t)a.P.hot * (sizeof(RowRec) + sizeof(WT));
    dim3 grid((unsigned)walk_grid(a.ntasks, block));
    if (a.P.hot) {
        // hot rows are staged once per block: launch only the blocks that stay
        // resident (LDS per CU), each looping over many tasks
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            cus > 0) {
            const int64_t per_cu = (int64_t)kLdsPerCu / (int64_t)(lds + 1024);
            const int64_t resident = (int64_t)cus * (per_cu > 1 ? per_cu : 1);
            if ((int64_t)grid.x > resident) grid.x = (unsigned)resident;
        }
    }
    // 64-byte slots get kernels of their own, so that the others keep their code;
    // the per-walker trace (parity checks only) tests the pointer instead
    if constexpr (TRACE) launch_shape<MODE, FP32, PROP, TRACE, 2>(a, grid, block, lds, s);
    else if (a.P.fat) launch_shape<MODE, FP32, PROP, TRACE, 1>(a, grid, block, lds, s);
    else launch_shape<MODE, FP32, PROP, TRACE, 0>(a, grid, block, lds, s);
    return hipGetLastError();
}

template <int MODE>
hipError_t launch_m(const WalkArgs &a, bool fp32, bool prop, bool trace, int block,
                    hipStream_t s) {
    if (fp32) {
        if (prop) return trace ? launch_t<MODE, true, true, true>(a, block, s)
                               : launch_t<MODE, true, true, false>(a, block, s);
        return trace ? launch_t<MODE, true, false, true>(a, block, s)
                     : launch_t<MODE, true, false, false>(a, block, s);
    }
    if (prop) return trace ? launch_t<MODE, false, true, true>(a, block, s)
                           : launch_t<MODE, false, true, false>(a, block, s);
    return trace ? launch_t<MODE, false, false, true>(a, block, s)
                 : launch_t<MODE, false, false, false>(a, block, s);
}

}  // namespace

namespace {

// Walker counts to a relative standard error target (the two-pass rule of the
// error model of Sec. 5, eps ~ sigma / sqrt(M)): entry e gets
// N_e = ceil(margin (sigma_e / (target |x_e|))^2) walkers, sigma_e = se_e sqrt(pilot)
// from the pilot's estimate x_e and standard error se_e, clamped to
// [min_walkers, max_walkers] (min_walkers when the pilot saw no spread, max_walkers
// when |x_e| = 0 or a value is not finite), then the chunk slots of every entry and
// their prefix sums.  One block: thread j takes a contiguous run of entries, one lane
// scans the run totals (integers, exact).
__global__ __launch_bounds__(1024) void k_size_to_target(int64_t k, int64_t pilot, double target,
                                                         double margin, int64_t min_w, int64_t max_w,
                                                         int64_t chunk, const double *__restrict__ est,
                                                         const double *__restrict__ se,
                                                         int64_t *__restrict__ var_task,
                                                         int64_t *__restrict__ var_nwalk,
                                                         int64_t *__restrict__ out2) {
    __shared__ long long run_s[1024], run_w[1024];
    const int j = threadIdx.x;
    const int64_t per = (k + 1023) / 1024;
    const int64_t lo = (int64_t)j * per;
    const int64_t hi = lo + per < k ? lo + per : k;
    const double sp = sqrt((double)pilot);
    long long cs = 0, ws = 0;
    for (int64_t e = lo; e < hi; ++e) {
        const double x = fabs(est[e]);
        const double sig = (se ? se[e] : 0.0) * sp;
        double nd;
        if (!isfinite(x) || !isfinite(sig)) nd = (double)max_w;
        else if (sig == 0.0) nd = (double)min_w;
        else if (x == 0.0) nd = (double)max_w;
        else {
            const double r = sig / (target * x);
            nd = ceil(margin * r * r);
        }
        if (!(nd >= (double)min_w)) nd = (double)min_w;
        if (nd > (double)max_w) nd = (double)max_w;
        const int64_t m = (int64_t)nd;
        var_nwalk[e] = m;
        cs += (m + chunk - 1) / chunk;
        ws += m;
    }
    run_s[j] = cs;
    run_w[j] = ws;
    __syncthreads();
    if (j == 0) {
        long long e_s = 0, e_w = 0;
        for (int u = 0; u < 1024; ++u) {
            const long long a = run_s[u];
            run_s[u] = e_s;
            e_s += a;
            e_w += run_w[u];
        }
        var_task[k] = e_s;
        out2[0] = e_s;
        out2[1] = e_w;
    }
    __syncthreads();
    long long o = run_s[j];
    for (int64_t e = lo; e < hi; ++e) {
        var_task[e] = o;
        o += (var_nwalk[e] + chunk - 1) / chunk;
    }
}

}  // namespace

hipError_t launch_size_to_target(int64_t k, int64_t pilot, double target, double margin,
                                 int64_t min_walkers, int64_t max_walkers, int64_t chunk,
                                 const double *est, const double *se, int64_t *var_task,
                                 int64_t *var_nwalk, int64_t *out2, hipStream_t s) {
    hipLaunchKernelGGL(k_size_to_target, dim3(1), dim3(1024), 0, s, k, pilot, target, margin,
                       min_walkers, max_walkers, chunk, est, se, var_task, var_nwalk, out2);
    return hipGetLastError();
}

int launch_walk_grid(int64_t ntasks, int block) { return walk_grid(ntasks, block); }

hipError_t launch_walk(const WalkArgs &a, int mode, bool fp32, bool prop, bool trace, int block,
                       hipStream_t s) {
    if (a.ntasks == 0) return hipSuccess;
    switch (mode) {
        case MC_EXACT:
            return launch_m<MC_EXACT>(a, fp32, prop, trace, block, s);
        case MC_STRANG:
            return launch_m<MC_STRANG>(a, fp32, false, trace, block, s);
        case MC_LIE:
            return launch_m<MC_LIE>(a, fp32, false, trace, block, s);
        default:
            return hipErrorInvalidValue;
    }
}

hipError_t launch_finalize(const WalkArgs &a, hipStream_t s) {
    if (a.var_task) {
        if (a.k == 0) return hipSuccess;
        if (a.k > 0x7FFFFFFF) return hipErrorInvalidValue;
        const uint32_t L = fin_lanes(a.var_chunks_max);
        hipLaunchKernelGGL(k_finalize_var, dim3((unsigned)a.k), dim3(L > WAVE ? L : WAVE), 0, s, a.k,
                           a.var_task, a.part, a.est, a.se);
        if (a.qmc && a.se)
            hipLaunchKernelGGL(k_qmc_stderr, dim3((unsigned)((a.k + 3) / 4)), dim3(256), 0, s,
                               a.k, (int64_t)0, a.var_task, a.part, a.est, a.se);
        return hipGetLastError();
    }
    if (a.chunks <= 1 || a.k == 0) return hipSuccess;
    const uint32_t L = fin_lanes(a.chunks);
    const int block = L > 256 ? (int)L : 256;
    const int64_t threads = a.k * (int64_t)L;
    const int64_t grid = (threads + block - 1) / block;
    hipLaunchKernelGGL(k_finalize, dim3((unsigned)grid), dim3(block), 0, s, a.k, a.chunks, a.part,
                       a.est, a.se);
    if (a.qmc && a.se) {
        const int64_t g2 = (a.k + 3) / 4;
        if (g2 > 0x7FFFFFFF) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_qmc_stderr, dim3((unsigned)g2), dim3(256), 0, s, a.k, a.chunks,
                           (const int64_t *)nullptr, a.part, a.est, a.se);
    }
    return hipGetLastError();
}

}  // namespace mc
