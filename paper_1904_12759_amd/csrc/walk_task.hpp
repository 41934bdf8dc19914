// Device code shared by the single-instance and batched walk kernels: the
// Philox generator, the logarithm, weight quadratures, the Chan merge and the
// per-task walker loop (run_task).  Included by walk.hip and batch.hip only.
#pragma once

#include <math.h>

#include "mc_internal.hpp"

namespace mc {

// ------------------------------------------------------------- primitives
namespace detail {

constexpr int WAVE = 64;

// ln 2 split so that e * kLn2Hi is exact for |e| < 2^11 (low 21 bits zero).
constexpr double kLn2Hi = 0x1.62e42fee00000p-1;
constexpr double kLn2Lo = 0x1.a39ef35793c76p-33;

// Natural logarithm of u in (0, 1].  With u = m 2^e, m in [1/sqrt2, sqrt2),
// log u = e ln2 + 2 atanh(f), f = (m-1)/(m+1), |f| < 0.1716, and atanh(f)/f is
// the Taylor series sum_k f^{2k}/(2k+1), kept to f^24 (truncation < 1e-19).
// Within about 2 ulp of the correctly rounded logarithm.
__device__ __forceinline__ double log_unit(double u) {
    int e;
    double m = frexp(u, &e);
    if (m < 0.70710678118654752440) {
        m = m + m;
        e -= 1;
    }
    const double f = (m - 1.0) / (m + 1.0);
    const double f2 = f * f;
    double p = 1.0 / 25.0;
    p = fma(p, f2, 1.0 / 23.0);
    p = fma(p, f2, 1.0 / 21.0);
    p = fma(p, f2, 1.0 / 19.0);
    p = fma(p, f2, 1.0 / 17.0);
    p = fma(p, f2, 1.0 / 15.0);
    p = fma(p, f2, 1.0 / 13.0);
    p = fma(p, f2, 1.0 / 11.0);
    p = fma(p, f2, 1.0 / 9.0);
    p = fma(p, f2, 1.0 / 7.0);
    p = fma(p, f2, 1.0 / 5.0);
    p = fma(p, f2, 1.0 / 3.0);
    p = fma(p, f2, 1.0);
    const double de = (double)e;
    return fma(de, kLn2Hi, fma(de, kLn2Lo, 2.0 * f * p));
}

__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        // three-input XOR in one v_bitop3_b32 (truth table 0x96)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        c0 = n0;
        c1 = (uint32_t)p1;
        c2 = n2;
        c3 = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

template <bool FP32>
struct WeightT {
    using T = double;
};
template <>
struct WeightT<true> {
    using T = float;
};

// Grid index K(s) = min(N, ceil(s * N / t)): the grid points k*dt with
// K(s_a) <= k < K(s_b) lie in the holding interval [s_a, s_b).
__device__ __forceinline__ int32_t grid_index(double s, double inv_dt, int32_t ngrid) {
    const double g = ceil(s * inv_dt);
    return g >= (double)ngrid ? ngrid : (int32_t)g;
}

// Sum of quadrature coefficients c_k over the grid points ka..kb (kb >= ka-1).
// STRANG (trapezoid): c_0 = c_N = 1/2, else 1.  LIE (right Riemann sum of
// Eq. (deff)): c_0 = 0, else 1.
template <int MODE>
__device__ __forceinline__ double grid_coef_sum(int32_t ka, int32_t kb, int32_t ngrid) {
    const int32_t count = kb - ka + 1;
    if (count <= 0) return 0.0;
    double c = (double)count;
    if (ka == 0) c -= (MODE == MC_STRANG) ? 0.5 : 1.0;
    if (MODE == MC_STRANG && kb == ngrid) c -= 0.5;
    return c;
}

template <bool FP32>
__device__ __forceinline__ typename WeightT<FP32>::T load_v(const void *v, uint32_t i) {
    if constexpr (FP32)
        return static_cast<const float *>(v)[i];
    else
        return static_cast<const double *>(v)[i];
}

template <bool FP32>
__device__ __forceinline__ typename WeightT<FP32>::T load_d(const InstArgs &P, uint32_t i) {
    if constexpr (FP32)
        return P.d32[i];
    else
        return P.d64[i];
}

template <bool FP32>
__device__ __forceinline__ typename WeightT<FP32>::T wexp(typename WeightT<FP32>::T x) {
    if constexpr (FP32)
        return expf(x);
    else
        return exp(x);
}

// Log-weight of the last holding interval [s, t] in a state with exponent dx.
template <int MODE, bool FP32>
__device__ __forceinline__ typename WeightT<FP32>::T final_term(typename WeightT<FP32>::T dx,
                                                                double s, int32_t ka,
                                                                const InstArgs &P) {
    using WT = typename WeightT<FP32>::T;
    if constexpr (MODE == MC_EXACT) {
        return dx * (WT)(P.t - s);
    } else {
        const double c = grid_coef_sum<MODE>(ka, P.ngrid, P.ngrid);
        return dx * (WT)(c * P.dt);
    }
}

// Merge (nb, mb, qb) into (na, ma, qa): count, mean and sum of squared
// deviations of the union (Chan, Golub, LeVeque 1979).
__device__ __forceinline__ void chan_merge(double &na, double &ma, double &qa, double nb,
                                           double mb, double qb) {
    const double n = na + nb;
    if (nb == 0.0) return;
    if (na == 0.0) {
        na = nb;
        ma = mb;
        qa = qb;
        return;
    }
    const double delta = mb - ma;
    const double w = nb / n;
    ma = ma + delta * w;
    qa = qa + qb + delta * delta * na * w;
    na = n;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, WAVE);
    return x;
}

}  // namespace detail

using namespace detail;

// ----------------------------------------------------------- one task
// Runs walkers ord0 .. ord0+cnt-1 from `node` on the calling wavefront and
// leaves, in every lane, the wave's (count, mean, M2) of W * v[X_t] plus the
// event and jump totals.  All lanes of the wave must call it together.
// `list` is this wave's LDS scratch of at least cnt words.
//
// Two phases.  When a walker's first holding time outlasts t with fair
// probability (e^{-r t} >= 1/8), phase 1 draws only the first event of every
// walker: those that stay return exactly K (the no-jump value), so they are
// counted as one group (n0, K, 0); the ordinals of the others are compacted
// into `list`.  Phase 2 runs the complete walk, with lane refill, on the
// listed walkers only (their first event is drawn again from the same
// counter), so the rarely needed logarithm, jump and exp code runs on lanes
// that need it instead of masked lanes of a mostly idle wave.
template <int MODE, bool FP32, bool PROP, bool TRACE>
__device__ __forceinline__ TaskResult run_task(const InstArgs &P, uint32_t node, uint32_t ord0,
                                               uint32_t cnt, const TraceOut &tr,
                                               uint32_t *list) {
    using WT = typename WeightT<FP32>::T;
    const int lane = threadIdx.x & (WAVE - 1);
    const unsigned long long lanemask_lt = (1ull << lane) - 1ull;
    const double t = P.t;

    // start row: the same for every walker of the task
    const RowRec r0 = P.rows[node];
    const WT d0 = load_d<FP32>(P, node);
    const WT v0 = load_v<FP32>(P.v, node);
    // K: the value of a walker that never leaves the start node
    const double K = (double)(wexp<FP32>(final_term<MODE, FP32>(d0, 0.0, 0, P)) * v0);
    // U below e0 means the first holding time certainly outlasts t: then
    // -log(U)/r0 > t + 2^-40/r0, far beyond the rounding of the log-based test.
    const double e0 = r0.deg ? exp(-t / r0.inv_r) * (1.0 - 0x1p-40) : 0.0;

    uint32_t n0 = 0;              // walkers that never jump (value K), wave-uniform
    unsigned long long evs = 0, jus = 0;
    uint32_t todo = cnt;          // walkers for phase 2
    bool use_list = false;
    if (r0.deg == 0) {
        // no exit rate at the start: every walker holds until t
        n0 = cnt;
        todo = 0;
        if (lane == 0) evs = cnt;
        if constexpr (TRACE) {
            for (uint32_t w = lane; w < cnt; w += WAVE) {
                tr.x[tr.base + w] = (int32_t)node;
                tr.ev[tr.base + w] = 1;
                tr.ju[tr.base + w] = 0;
                tr.f[tr.base + w] = K;
            }
        }
    } else if (e0 >= 0.125) {
        use_list = true;
        uint32_t nlist = 0;
        // U >= e0  <=>  m + 1 >= e0 * 2^53 (exact: U = (m+1) 2^-53), i.e. m + 1 >= ceil(e0 2^53)
        const uint64_t m_thr = (uint64_t)ceil(e0 * 0x1p53);
        for (uint32_t b = 0; b < cnt; b += WAVE) {
            const uint32_t w = b + (uint32_t)lane;
            const bool valid = w < cnt;
            bool go = false;
            if (valid) {
                const U4 o = philox(0u, ord0 + w, node, P.inst, P.key0, P.key1);
                const uint64_t m = ((uint64_t)o.x << 21) | ((uint64_t)o.y >> 11);
                go = m + 1ull >= m_thr;
            }
            const unsigned long long gmask = __ballot(go);
            const unsigned long long smask = __ballot(valid && !go);
            if (go) list[nlist + (uint32_t)__popcll(gmask & lanemask_lt)] = w;
            nlist += (uint32_t)__popcll(gmask);
            n0 += (uint32_t)__popcll(smask);
            if constexpr (TRACE) {
                if (valid && !go) {
                    tr.x[tr.base + w] = (int32_t)node;
                    tr.ev[tr.base + w] = 1;
                    tr.ju[tr.base + w] = 0;
                    tr.f[tr.base + w] = K;
                }
            }
        }
        if (lane == 0) evs = n0;
        todo = nlist;
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }

    // ---- phase 2: full walks with lane refill over `todo` walkers
    uint32_t wl = (uint32_t)lane;
    bool active = wl < todo;
    uint32_t ow = 0;              // walker ordinal within the task
    if (active) ow = use_list ? list[wl] : wl;
    uint32_t x = node;
    double s = 0.0;
    WT logw = (WT)0;
    uint32_t ev = 0, ju = 0;
    int32_t ka = 0;
    double inv_r = r0.inv_r;
    uint32_t deg = r0.deg, begin = r0.begin;
    WT dx = d0;

    uint32_t nl = 0;
    double kl = 0.0, s1 = 0.0, s2 = 0.0;
    uint32_t next = WAVE;
    uint32_t err = 0;

    while (__ballot(active) != 0ull) {
        bool fin = false;
        if (active) {
            if (deg == 0) {
                ++ev;                    // no exit rate: holds until t
                fin = true;
            } else if (ev >= P.max_events) {
                err |= F_WALK_LIMIT;
                fin = true;
            } else {
                const U4 o = philox(ev, ord0 + ow, node, P.inst, P.key0, P.key1);
                ++ev;
                const uint64_t m = ((uint64_t)o.x << 21) | ((uint64_t)o.y >> 11);
                const double U = (double)(m + 1ull) * 0x1p-53;
                bool jump = false;
                double S = 0.0, sn = 0.0;
                if (ju != 0 || U >= e0) {
                    S = -log_unit(U) * inv_r;
                    sn = s + S;
                    jump = sn < t;
                }
                if (jump) {
                    if constexpr (MODE == MC_EXACT) {
                        logw = logw + dx * (WT)S;
                    } else {
                        const int32_t kb = grid_index(sn, P.inv_dt, P.ngrid);
                        const double cs = grid_coef_sum<MODE>(ka, kb - 1, P.ngrid);
                        logw = logw + dx * (WT)(cs * P.dt);
                        ka = kb;
                    }
                    s = sn;
                    const uint32_t sl = (uint32_t)(((uint64_t)o.z * (uint64_t)deg) >> 32);
                    const SlotRec q = P.slots[begin + sl];
                    const bool keep = o.w < q.thr;
                    x = (uint32_t)(keep ? q.self : q.alias);
                    if constexpr (PROP) {
                        const float2 cr = P.corr[begin + sl];
                        logw = logw + (WT)(keep ? cr.x : cr.y);
                    }
                    ++ju;
                    const RowRec rr = P.rows[x];
                    inv_r = rr.inv_r;
                    deg = rr.deg;
                    begin = rr.begin;
                    dx = load_d<FP32>(P, x);
                } else {
                    fin = true;
                }
            }
            if (fin) {
                double f = K;            // never left the start node
                if (ju != 0) {
                    logw = logw + final_term<MODE, FP32>(dx, s, ka, P);
                    f = (double)(wexp<FP32>(logw) * load_v<FP32>(P.v, x));
                    if (!isfinite(f)) err |= F_OVERFLOW;
                }
                if (nl == 0) kl = f;
                const double df = f - kl;
                s1 += df;
                s2 += df * df;
                ++nl;
                evs += ev;
                jus += ju;
                if constexpr (TRACE) {
                    const int64_t ti = tr.base + ow;
                    tr.x[ti] = (int32_t)x;
                    tr.ev[ti] = ev;
                    tr.ju[ti] = ju;
                    tr.f[ti] = f;
                }
            }
        }
        const unsigned long long fmask = __ballot(fin);
        if (fin) {
            wl = next + (uint32_t)__popcll(fmask & lanemask_lt);
            if (wl < todo) {
                ow = use_list ? list[wl] : wl;
                x = node;
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

    // lane -> (count, mean, M2), then pairwise across the wave
    double n = (double)nl, mean = 0.0, q = 0.0;
    if (nl) {
        mean = kl + s1 / n;
        q = s2 - s1 * (s1 / n);
        if (q < 0.0) q = 0.0;
    }
#pragma unroll
    for (int off = 1; off < WAVE; off <<= 1) {
        const double nb = __shfl_xor(n, off, WAVE);
        const double mb = __shfl_xor(mean, off, WAVE);
        const double qb = __shfl_xor(q, off, WAVE);
        // both lanes of a pair merge (lower, upper) in that order
        if (lane & off) {
            double n2 = nb, m2 = mb, q2 = qb;
            chan_merge(n2, m2, q2, n, mean, q);
            n = n2;
            mean = m2;
            q = q2;
        } else {
            chan_merge(n, mean, q, nb, mb, qb);
        }
    }
    // the walkers that never jumped: n0 copies of K
    double nn = (double)n0, mm = K, qq = 0.0;
    chan_merge(nn, mm, qq, n, mean, q);
    TaskResult res;
    res.n = nn;
    res.mean = mm;
    res.m2 = qq;
    res.events = wave_sum_u64(evs);
    res.jumps = wave_sum_u64(jus);
    res.err = err;
    return res;
}

}  // namespace mc
