// The walk: continuous-time Markov-chain paths through the indices of A and
// the multiplicative functional of Theorem 1 (paper Sec. 2-3, Algorithm 1).
//
// Work decomposition.  A task is (entry e, chunk c): the walkers with
// ordinals c*chunk .. min(N, (c+1)*chunk)-1 started at node idx[e].  One
// wavefront owns a task; its 64 lanes each run one walker and, when a walker
// stops, take the next unstarted ordinal of the chunk (lane refill), so a long
// path holds up one lane instead of the whole wave.  Each lane accumulates
// sum(f - K) and sum((f - K)^2) in FP64, where K is the value of a walker that
// never jumps (most walkers at the benchmark sizes), and the wave combines the
// lane sums with cross-lane shuffles.  Paths depend only on the Philox counter
// (event, ordinal, start node, instance), never on which lane ran them.
#include <math.h>

#include "mc_internal.hpp"

namespace mc {
namespace {

constexpr int WAVE = 64;

template <bool FP32>
struct WeightT {
    using T = double;
};
template <>
struct WeightT<true> {
    using T = float;
};

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, WAVE);
    return x;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, WAVE);
    return x;
}

// Grid index K(s) = min(N, ceil(s * N / t)): the grid points k*dt with
// K(s_a) <= k < K(s_b) lie in the holding interval [s_a, s_b).
__device__ __forceinline__ int64_t grid_index(double s, double inv_dt, int64_t ngrid) {
    const double g = ceil(s * inv_dt);
    return g >= (double)ngrid ? ngrid : (int64_t)g;
}

// Sum of quadrature coefficients c_k over the grid points k in [ka, kb]
// (kb >= ka - 1).  STRANG (trapezoid): c_0 = c_N = 1/2, else 1.  LIE (right
// Riemann sum of Eq. (deff)): c_0 = 0, else 1.
template <int MODE>
__device__ __forceinline__ double grid_coef_sum(int64_t ka, int64_t kb, int64_t ngrid) {
    const int64_t count = kb - ka + 1;
    if (count <= 0) return 0.0;
    double c = (double)count;
    if (ka == 0) c -= (MODE == MC_STRANG) ? 0.5 : 1.0;
    if (MODE == MC_STRANG && kb == ngrid) c -= 0.5;
    return c;
}

template <bool FP32>
__device__ __forceinline__ typename WeightT<FP32>::T load_v(const void *v, int64_t i) {
    if constexpr (FP32)
        return static_cast<const float *>(v)[i];
    else
        return static_cast<const double *>(v)[i];
}

template <bool FP32>
__device__ __forceinline__ typename WeightT<FP32>::T load_d(const WalkArgs &a, int64_t i) {
    if constexpr (FP32)
        return a.d32[i];
    else
        return a.d64[i];
}

template <bool FP32>
__device__ __forceinline__ typename WeightT<FP32>::T wexp(typename WeightT<FP32>::T x) {
    if constexpr (FP32)
        return expf(x);
    else
        return exp(x);
}

// Log-weight of the last holding interval [s, t] in state x (weight exponent dx).
template <int MODE, bool FP32>
__device__ __forceinline__ typename WeightT<FP32>::T final_term(
    typename WeightT<FP32>::T dx, double s, int64_t ka, const WalkArgs &a) {
    using WT = typename WeightT<FP32>::T;
    if constexpr (MODE == MC_EXACT) {
        return dx * (WT)(a.t - s);
    } else {
        const double c = grid_coef_sum<MODE>(ka, a.ngrid, a.ngrid);
        return dx * (WT)(c * a.dt);
    }
}

template <int MODE, bool FP32, bool PROP, bool TRACE>
__global__ __launch_bounds__(256) void k_walk(WalkArgs a) {
    using WT = typename WeightT<FP32>::T;
    const int lane = threadIdx.x & (WAVE - 1);
    const unsigned long long lanemask_lt = (1ull << lane) - 1ull;
    const int64_t wave_id = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / WAVE;
    const double t = a.t;

    for (int64_t task = wave_id; task < a.ntasks; task += nwaves) {
        const int64_t e = task / a.chunks;
        const int64_t c = task - e * a.chunks;
        const int64_t node = a.idx ? a.idx[e] : e;
        if (node < 0 || node >= a.n) {
            if (lane == 0) {
                atomicOr(a.flags, F_OUT_OF_RANGE);
                if (a.chunks == 1) {
                    a.est[e] = NAN;
                    if (a.se) a.se[e] = NAN;
                } else {
                    a.part[(e * a.chunks + c) * 2] = NAN;
                    a.part[(e * a.chunks + c) * 2 + 1] = NAN;
                    if (c == 0) a.shift[e] = NAN;
                }
            }
            continue;
        }
        const int64_t wbase = c * (int64_t)a.chunk;
        const int64_t rem = a.nwalk - wbase;
        const uint32_t cnt = (uint32_t)(rem < (int64_t)a.chunk ? rem : (int64_t)a.chunk);

        // start row: the same for every walker of the task
        const RowRec r0 = a.rows[node];
        const WT d0 = load_d<FP32>(a, node);
        const WT v0 = load_v<FP32>(a.v, node);
        // K: the value returned by a walker that never leaves the start node
        const WT lw0 = final_term<MODE, FP32>(d0, 0.0, 0, a);
        const double K = (double)(wexp<FP32>(lw0) * v0);

        // walker state
        uint32_t wl = (uint32_t)lane;
        bool active = wl < cnt;
        uint32_t x = (uint32_t)node;
        double s = 0.0;
        WT logw = (WT)0;
        uint32_t ev = 0, ju = 0;
        int64_t ka = 0;
        double inv_r = r0.inv_r;
        uint32_t deg = r0.deg, begin = r0.begin;
        WT dx = d0;

        double acc1 = 0.0, acc2 = 0.0;
        unsigned long long evs = 0, jus = 0;
        uint32_t next = WAVE;
        uint32_t err = 0;

        while (__ballot(active) != 0ull) {
            bool fin = false;
            if (active) {
                if (deg == 0) {
                    ++ev;            // a state with no exit rate holds until t
                    fin = true;
                } else if (ev >= a.max_events) {
                    err |= F_WALK_LIMIT;
                    fin = true;
                } else {
                    const U4 o = philox10(ev, (uint32_t)(a.w0 + wbase + wl), (uint32_t)node,
                                          a.inst, a.key0, a.key1);
                    ++ev;
                    const uint64_t m = ((uint64_t)o.x << 21) | ((uint64_t)o.y >> 11);
                    const double U = (double)(m + 1ull) * 0x1p-53;
                    const double S = -log(U) * inv_r;
                    const double sn = s + S;
                    if (sn < t) {
                        if constexpr (MODE == MC_EXACT) {
                            logw = logw + dx * (WT)S;
                        } else {
                            const int64_t kb = grid_index(sn, a.inv_dt, a.ngrid);
                            const double cs = grid_coef_sum<MODE>(ka, kb - 1, a.ngrid);
                            logw = logw + dx * (WT)(cs * a.dt);
                            ka = kb;
                        }
                        s = sn;
                        const uint32_t sl =
                            (uint32_t)(((uint64_t)o.z * (uint64_t)deg) >> 32);
                        const SlotRec q = a.slots[begin + sl];
                        const bool keep = o.w < q.thr;
                        x = (uint32_t)(keep ? q.self : q.alias);
                        if constexpr (PROP) {
                            const float2 cr = a.corr[begin + sl];
                            logw = logw + (WT)(keep ? cr.x : cr.y);
                        }
                        ++ju;
                        const RowRec rr = a.rows[x];
                        inv_r = rr.inv_r;
                        deg = rr.deg;
                        begin = rr.begin;
                        dx = load_d<FP32>(a, x);
                    } else {
                        fin = true;
                    }
                }
                if (fin) {
                    logw = logw + final_term<MODE, FP32>(dx, s, ka, a);
                    const double f = (double)(wexp<FP32>(logw) * load_v<FP32>(a.v, x));
                    if (!isfinite(f)) err |= F_OVERFLOW;
                    const double df = f - K;
                    acc1 += df;
                    acc2 += df * df;
                    evs += ev;
                    jus += ju;
                    if constexpr (TRACE) {
                        const int64_t ti = wbase + wl;
                        a.tr_x[ti] = (int32_t)x;
                        a.tr_ev[ti] = ev;
                        a.tr_ju[ti] = ju;
                        a.tr_f[ti] = f;
                    }
                }
            }
            const unsigned long long fmask = __ballot(fin);
            if (fin) {
                wl = next + (uint32_t)__popcll(fmask & lanemask_lt);
                if (wl < cnt) {
                    x = (uint32_t)node;
                    s = 0.0;
                    logw = (WT)0;
                    ev = 0;
                    ju = 0;
                    ka = 0;
                    inv_r = r0.inv_r;
                    deg = r0.deg;
                    begin = r0.begin;
                    dx = d0;
                } else {
                    active = false;
                }
            }
            next += (uint32_t)__popcll(fmask);
        }

        acc1 = wave_sum(acc1);
        acc2 = wave_sum(acc2);
        evs = wave_sum_u64(evs);
        jus = wave_sum_u64(jus);
        const unsigned long long emask = __ballot(err != 0);
        if (emask) {
            if (err) atomicOr(a.flags, err);
        }
        if (lane == 0) {
            if (a.chunks == 1) {
                const double nw = (double)a.nwalk;
                a.est[e] = K + acc1 / nw;
                if (a.se) {
                    double var = a.nwalk > 1 ? (acc2 - acc1 * acc1 / nw) / (nw - 1.0) : 0.0;
                    a.se[e] = sqrt((var > 0.0 ? var : 0.0) / nw);
                }
            } else {
                a.part[(e * a.chunks + c) * 2] = acc1;
                a.part[(e * a.chunks + c) * 2 + 1] = acc2;
                if (c == 0) a.shift[e] = K;
            }
            if (a.counters) {
                atomicAdd(&a.counters[0], evs);
                atomicAdd(&a.counters[1], jus);
            }
        }
    }
}

// Combine the chunk partials of every entry in chunk order.
__global__ void k_finalize(WalkArgs a) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a.k) return;
    double s1 = 0.0, s2 = 0.0;
    const double *p = a.part + e * a.chunks * 2;
    for (int64_t c = 0; c < a.chunks; ++c) {
        s1 += p[2 * c];
        s2 += p[2 * c + 1];
    }
    const double nw = (double)a.nwalk;
    a.est[e] = a.shift[e] + s1 / nw;
    if (a.se) {
        double var = a.nwalk > 1 ? (s2 - s1 * s1 / nw) / (nw - 1.0) : 0.0;
        a.se[e] = sqrt((var > 0.0 ? var : 0.0) / nw);
    }
}

template <int MODE, bool FP32, bool PROP, bool TRACE>
hipError_t launch_t(const WalkArgs &a, int block, hipStream_t s) {
    const int64_t waves_per_block = block / WAVE;
    int64_t grid = (a.ntasks + waves_per_block - 1) / waves_per_block;
    const int64_t max_grid = 1 << 16;
    if (grid > max_grid) grid = max_grid;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL((k_walk<MODE, FP32, PROP, TRACE>), dim3((unsigned)grid), dim3(block), 0, s,
                       a);
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
    if (a.chunks <= 1 || a.k == 0) return hipSuccess;
    const int block = 256;
    const int64_t grid = (a.k + block - 1) / block;
    hipLaunchKernelGGL(k_finalize, dim3((unsigned)grid), dim3(block), 0, s, a);
    return hipGetLastError();
}

}  // namespace mc
