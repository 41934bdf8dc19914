// Device code shared by the single-instance and batched walk kernels: the
// Philox generator, the logarithm, weight quadratures, the Chan merge and the
// per-task walker loop (run_group).  Included by walk.hip and batch.hip only.
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

// An FP64 constant materialised in a scalar register pair where it is used.
// Without this the compiler keeps the logarithm's coefficients live in vector
// registers across the whole walk loop, which costs a wave of occupancy.
__device__ __forceinline__ double sconst(double c) {
    asm volatile("" : "+s"(c));
    return c;
}

// Predicates of the compiler's lane-mask comparisons (the integer comparison
// codes of its IR): unsigned >= and unsigned <.
constexpr int kCmpUge = 35;
constexpr int kCmpUlt = 36;

// The lanes of the wave where b holds, as a 64-bit mask.
__device__ __forceinline__ unsigned long long lanes_where(bool b) {
    return __builtin_amdgcn_ballot_w64(b);
}

// Number of lanes below this one whose bit is set in mask (mbcnt on the two halves).
__device__ __forceinline__ uint32_t set_below(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Natural logarithm of u in (0, 1].  With u = m 2^e, m in [1/sqrt2, sqrt2),
// log u = e ln2 + 2 atanh(f), f = (m-1)/(m+1), |f| < 0.1716, and atanh(f)/f is
// the Taylor series sum_k f^{2k}/(2k+1), kept to f^24 (truncation < 1e-19).
// Within 3 ulp of the correctly rounded logarithm (the largest errors, about
// 2.5 ulp, where e ln2 and 2 atanh(f) partly cancel, u just below 1/sqrt2).
__device__ __forceinline__ double log_unit(double u) {
    int e;
    double m = frexp(u, &e);
    if (m < sconst(0.70710678118654752440)) {
        m = m + m;
        e -= 1;
    }
    // f = (m - 1) / (m + 1), m + 1 in [1.7, 2.5): the hardware reciprocal, two
    // Newton steps and a residual correction (within an ulp of the quotient; no
    // operand scaling or special cases are needed in this range)
    const double a = m - 1.0, b = m + 1.0;
    double y = __builtin_amdgcn_rcp(b);
    y = fma(fma(-b, y, 1.0), y, y);
    y = fma(fma(-b, y, 1.0), y, y);
    const double q0 = a * y;
    const double f = fma(fma(-b, q0, a), y, q0);
    const double f2 = f * f;
    double p = sconst(1.0 / 25.0);
    p = fma(p, f2, sconst(1.0 / 23.0));
    p = fma(p, f2, sconst(1.0 / 21.0));
    p = fma(p, f2, sconst(1.0 / 19.0));
    p = fma(p, f2, sconst(1.0 / 17.0));
    p = fma(p, f2, sconst(1.0 / 15.0));
    p = fma(p, f2, sconst(1.0 / 13.0));
    p = fma(p, f2, sconst(1.0 / 11.0));
    p = fma(p, f2, sconst(1.0 / 9.0));
    p = fma(p, f2, sconst(1.0 / 7.0));
    p = fma(p, f2, sconst(1.0 / 5.0));
    p = fma(p, f2, sconst(1.0 / 3.0));
    p = fma(p, f2, 1.0);
    const double de = (double)e;
    return fma(de, sconst(kLn2Hi), fma(de, sconst(kLn2Lo), 2.0 * f * p));
}

// e^x in FP64: Cody-Waite reduction x = k ln2 + r, |r| <= ln2/2 (k ln2 taken
// as k*kLn2Hi, exact for |k| < 2^11, plus k*kLn2Lo), the Taylor series of e^r
// to r^13 (truncation below 2^-56 relative), then scaling by 2^k.  Within
// about 2 ulp of the correctly rounded value; NaN stays NaN, x < -1100 gives
// 0 and x > 1100 gives +inf.
__device__ __forceinline__ double exp_f64(double x) {
    if (!(x >= -1100.0)) return x != x ? x : 0.0;
    if (x > 1100.0) return __longlong_as_double(0x7ff0000000000000ll);
    const double k = rint(x * sconst(0x1.71547652b82fep+0));   // x log2(e)
    const double r = fma(-k, sconst(kLn2Lo), fma(-k, sconst(kLn2Hi), x));
    double p = sconst(1.0 / 6227020800.0);                       // 1/13!
    p = fma(p, r, sconst(1.0 / 479001600.0));
    p = fma(p, r, sconst(1.0 / 39916800.0));
    p = fma(p, r, sconst(1.0 / 3628800.0));
    p = fma(p, r, sconst(1.0 / 362880.0));
    p = fma(p, r, sconst(1.0 / 40320.0));
    p = fma(p, r, sconst(1.0 / 5040.0));
    p = fma(p, r, sconst(1.0 / 720.0));
    p = fma(p, r, sconst(1.0 / 120.0));
    p = fma(p, r, sconst(1.0 / 24.0));
    p = fma(p, r, sconst(1.0 / 6.0));
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return ldexp(p, (int)k);
}

// 1 - e^{-y} for y >= 0 without cancellation: for y below ln2/2 the series
// y (1 - y/2! + y^2/3! - ...) to y^14 (truncation below 2^-56 relative),
// otherwise 1 - e^{-y} with exp_f64 (e^{-y} <= 0.71, so the difference loses
// no more than a bit).
__device__ __forceinline__ double one_minus_exp_neg(double y) {
    if (y >= sconst(0.34657359027997264)) return 1.0 - exp_f64(-y);
    const double r = -y;
    double p = sconst(1.0 / 87178291200.0);                      // 1/14!
    p = fma(p, r, sconst(1.0 / 6227020800.0));
    p = fma(p, r, sconst(1.0 / 479001600.0));
    p = fma(p, r, sconst(1.0 / 39916800.0));
    p = fma(p, r, sconst(1.0 / 3628800.0));
    p = fma(p, r, sconst(1.0 / 362880.0));
    p = fma(p, r, sconst(1.0 / 40320.0));
    p = fma(p, r, sconst(1.0 / 5040.0));
    p = fma(p, r, sconst(1.0 / 720.0));
    p = fma(p, r, sconst(1.0 / 120.0));
    p = fma(p, r, sconst(1.0 / 24.0));
    p = fma(p, r, sconst(1.0 / 6.0));
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    return y * p;                                                // -(r P(r)) = -expm1(r)
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

// First-event words of walker w from the randomised rank-1 lattice: with
// o = Philox of the replicate's shift counter, B = 2^b and j = the b bits of
// w mod B reversed (radical-inverse order: the first 2^k walkers of a replicate
// are the 2^k-point sub-lattice),
//   64-bit word of U:  j 2^(64-b) + (o.x 2^32 + o.y)   mod 2^64
//   slot word:         j g1 2^(32-b) + o.z             mod 2^32
//   alias word:        j g2 2^(32-b) + o.w             mod 2^32
// with (1, g1, g2) = (1, a, a^2 mod B): every coordinate is a uniform shift of
// the lattice point modulo 1.
__device__ __forceinline__ U4 lattice_words(U4 o, uint32_t w, uint32_t b) {
    const uint32_t g1 = b == 9u ? 119u : 149u;
    const uint32_t g2 = (g1 * g1) & ((1u << b) - 1u);
    const uint32_t j = __builtin_bitreverse32(w) >> (32u - b);
    const uint64_t u0 = ((uint64_t)j << (64u - b)) + (((uint64_t)o.x << 32) | o.y);
    return U4{(uint32_t)(u0 >> 32), (uint32_t)u0, ((j * g1) << (32u - b)) + o.z,
              ((j * g2) << (32u - b)) + o.w};
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

// Row record and weight exponent of walk id x.  With LOC (relabelled rows),
// the hot rows x < P.hot come from their LDS copy.
template <bool LOC>
__device__ __forceinline__ RowRec row_at(const InstArgs &P, uint32_t x) {
    if constexpr (LOC)
        if (x < P.hot) return P.lrows[x];
    return P.rows[x];
}

template <bool FP32, bool LOC>
__device__ __forceinline__ typename WeightT<FP32>::T d_at(const InstArgs &P, uint32_t x) {
    if constexpr (LOC)
        if (x < P.hot) return static_cast<const typename WeightT<FP32>::T *>(P.ld)[x];
    return load_d<FP32>(P, x);
}

// A jump from slot js with alias word w: the destination x and its row and d.
// jump_sep reads the slot, then the destination's row and d; jump_fat reads the
// 64-byte slot that holds both destinations' rows and d.  Same values either way.
template <bool FP32, bool LOC>
__device__ __forceinline__ bool jump_sep(const InstArgs &P, uint32_t js, uint32_t w, uint32_t &x,
                                         double &inv_r, uint32_t &deg, uint32_t &begin,
                                         typename WeightT<FP32>::T &dx) {
    const SlotRec q = P.slots[js];
    const bool keep = w < q.thr;
    x = (uint32_t)(keep ? q.self : q.alias);
    const RowRec rr = row_at<LOC>(P, x);
    inv_r = rr.inv_r;
    deg = rr.deg;
    begin = rr.begin;
    dx = d_at<FP32, LOC>(P, x);
    return keep;
}

template <bool FP32>
__device__ __forceinline__ bool jump_fat(const InstArgs &P, uint32_t js, uint32_t w, uint32_t &x,
                                         double &inv_r, uint32_t &deg, uint32_t &begin,
                                         typename WeightT<FP32>::T &dx) {
    const FatSlot q = P.fat[js];
    const bool keep = w < q.s.thr;
    x = (uint32_t)(keep ? q.s.self : q.s.alias);
    inv_r = keep ? q.rs.inv_r : q.ra.inv_r;
    deg = keep ? q.rs.deg : q.ra.deg;
    begin = keep ? q.rs.begin : q.ra.begin;
    dx = (typename WeightT<FP32>::T)(keep ? q.ds : q.da);
    return keep;
}

// Matrix-free 7-point stencil: the jump from x by the inverse-CDF rule over its
// six faces in column order (-z, -y, -x, +x, +y, +z): the first face whose running
// sum of rates exceeds u r, u = o2 2^-32 in [0, 1), or the last face with a rate
// when rounding leaves u r at or above the sum.  The state's thresholds turn that
// into a count of integer comparisons; meta and e0 (the face word and the first
// threshold) came with the row record, the other four are read here.  The
// neighbour comes from the index.
__device__ __forceinline__ uint32_t stencil_jump(const InstArgs &P, uint32_t x, uint32_t meta,
                                                 uint32_t e0, uint32_t o2) {
    const uint4 e = P.stail[x];
    const uint32_t m = (o2 > e0 ? 1u : 0u) + (o2 > e.x ? 1u : 0u) + (o2 > e.y ? 1u : 0u) +
                       (o2 > e.z ? 1u : 0u) + (o2 > e.w ? 1u : 0u);
    const uint32_t face = (meta >> (3u + 3u * m)) & 7u;
    // |x offset| 1, nx or nx ny for the x, y or z axis, selected without branches
    const bool lower = face < 3u;
    const uint32_t axis = lower ? 2u - face : face - 3u;          // 0: x, 1: y, 2: z
    const uint32_t step = 1u + ((P.nx - 1u) & (0u - (uint32_t)(axis != 0u))) +
                          ((P.nxy - P.nx) & (0u - (uint32_t)(axis == 2u)));
    return x + (lower ? 0u - step : step);
}

// Walk id of an original node, and back (identity without relabelling).
template <bool LOC>
__device__ __forceinline__ uint32_t walk_id(const InstArgs &P, uint32_t node) {
    if constexpr (LOC) return P.perm[node];
    return node;
}
template <bool LOC>
__device__ __forceinline__ uint32_t orig_id(const InstArgs &P, uint32_t x) {
    if constexpr (LOC) return P.inv[x];
    return x;
}

// Position that the walker in this lane takes when the wave's walkers are sorted
// by current walk id (lanes without a walker last, ties in lane order): each
// lane returns the lane whose walker sorts to it.  A bitonic network over the
// 64 keys (x << 6 | lane), exchanged with lane shuffles; the calling wave must
// be converged.
__device__ __forceinline__ uint32_t sorted_source(uint32_t x, bool active, int lane) {
    unsigned long long key =
        ((unsigned long long)(active ? x : 0xFFFFFFFFu) << 6) | (unsigned long long)lane;
    for (int k = 2; k <= WAVE; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            const unsigned long long o = __shfl_xor(key, j, WAVE);
            const bool ascending = (lane & k) == 0;
            const bool lower = (lane & j) == 0;
            const unsigned long long lo = key < o ? key : o;
            const unsigned long long hi = key < o ? o : key;
            key = lower == ascending ? lo : hi;
        }
    }
    return (uint32_t)(key & (WAVE - 1));
}

// e^x in FP32 for the FP32 weights: x log2(e) = p + c exactly to about 2^-48
// (p the rounded product, c its rounding error by an FMA plus x times the low
// part of log2(e)), k = rint(p), then 2^((p - k) + c) from the hardware exp2
// (|p - k + c| <= 1/2) scaled by 2^k.  Within 2 ulp; a finite x beyond the
// range gives +inf through the scaling, x below -104 (past the smallest
// denormal, and -inf) gives 0, NaN and +inf give NaN.  k is clamped to
// [-512, 512] before its conversion to an integer (a no-op wherever the result
// is kept), so that the conversion is defined for every x.
__device__ __forceinline__ float exp_f32(float x) {
    const float p = x * 1.44269502f;
    const float c = fmaf(x, 1.92596299e-8f, fmaf(x, 1.44269502f, -p));
    const float k = rintf(p);
    const float y = __builtin_amdgcn_exp2f((p - k) + c);
    const float r = ldexpf(y, (int)__builtin_amdgcn_fmed3f(k, -512.0f, 512.0f));
    return x < -104.0f ? 0.0f : r;
}

template <bool FP32>
__device__ __forceinline__ typename WeightT<FP32>::T wexp(typename WeightT<FP32>::T x) {
    if constexpr (FP32)
        return exp_f32(x);
    else
        return exp_f64(x);
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

// Cross-lane moves within a row of 16 lanes (DPP), on the two 32-bit halves of
// a 64-bit value.  CTRL: 0xB1 swaps neighbouring lanes (quad_perm 1,0,3,2),
// 0x4E swaps lane pairs (quad_perm 2,3,0,1), 0x141 mirrors each half row of 8,
// 0x140 mirrors the row.  All lanes of the row must be active.
template <int CTRL>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t b) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xF, 0xF, false);
    const uint32_t hi =
        (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
    return ((uint64_t)hi << 32) | lo;
}

// Merge of one entry's chunk partials p[3c .. 3c+2] = (count, mean, M2),
// c < chunks, by the L lanes sub = 0 .. L-1 of a group aligned to L in the
// block, in a fixed order: lane sub takes chunks sub, sub + L, sub + 2L, ...
// (so that a wave's loads cover consecutive partials), eight at a time as a
// pairwise tree whose result it merges into its running total; then lane sub
// takes in the total of lane sub + off for off = 1, 2, 4, ... (across waves
// through lds, one (count, mean, M2) per wave).  The result is in sub-lane 0.
// Every thread of the block must call it (it holds a barrier), all lanes of a
// wave with the same L, all lanes of a group with the same p and chunks (p
// may be null when chunks is 0).
__device__ __forceinline__ void fin_merge(const double *p, int64_t chunks, uint32_t L, uint32_t sub,
                                          double (*lds)[3], double &n, double &mean, double &m2) {
    n = 0.0;
    mean = 0.0;
    m2 = 0.0;
    // a lane's partials fetched together (past the end: its first chunk read again,
    // in bounds, and taken as empty, which merges as a no-op), so that the loads
    // overlap, and merged as a tree of depth three
    constexpr int B = 8;
    for (int64_t c = sub; c < chunks; c += (int64_t)B * L) {
        double bn[B], bm[B], bq[B];
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const int64_t ck = c + (int64_t)k * L;
            const bool in = ck < chunks;
            const int64_t cl = in ? ck : c;
            bn[k] = in ? p[3 * cl] : 0.0;
            bm[k] = p[3 * cl + 1];
            bq[k] = p[3 * cl + 2];
        }
#pragma unroll
        for (int s = 1; s < B; s <<= 1)
#pragma unroll
            for (int k = 0; k < B; k += 2 * s) chan_merge(bn[k], bm[k], bq[k], bn[k + s], bm[k + s], bq[k + s]);
        chan_merge(n, mean, m2, bn[0], bm[0], bq[0]);
    }
    const uint32_t W = L < WAVE ? L : WAVE;
    for (uint32_t off = 1; off < W; off <<= 1) {
        const double nb = __shfl_down(n, off, (int)W);
        const double mb = __shfl_down(mean, off, (int)W);
        const double qb = __shfl_down(m2, off, (int)W);
        if ((sub & (2 * off - 1)) == 0) chan_merge(n, mean, m2, nb, mb, qb);
    }
    const uint32_t wave = threadIdx.x / WAVE;
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        lds[wave][0] = n;
        lds[wave][1] = mean;
        lds[wave][2] = m2;
    }
    __syncthreads();
    if (L > WAVE && sub == 0 && chunks > 0) {
        // the group's waves wave .. wave + L/64 - 1, merged pairwise in place (an
        // empty group leaves lds alone: its waves may belong to other groups)
        const uint32_t nw = L / WAVE;
        for (uint32_t s = 1; s < nw; s <<= 1)
            for (uint32_t k = 0; k < nw; k += 2 * s)
                chan_merge(lds[wave + k][0], lds[wave + k][1], lds[wave + k][2], lds[wave + k + s][0],
                           lds[wave + k + s][1], lds[wave + k + s][2]);
        n = lds[wave][0];
        mean = lds[wave][1];
        m2 = lds[wave][2];
    }
}

__device__ __forceinline__ uint64_t readlane_u64(uint64_t b, int l) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ double readlane_f64(double x, int l) {
    return __longlong_as_double((long long)readlane_u64((uint64_t)__double_as_longlong(x), l));
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
    return __longlong_as_double((long long)dpp_u64<CTRL>((uint64_t)__double_as_longlong(x)));
}

// Sum over each row of 16 lanes: the first four steps of wave_sum_f64, after
// which every lane of a row holds the row's sum.  Every lane of the wave must be
// active.
__device__ __forceinline__ double row_sum_f64(double x) {
    x = x + dpp_f64<0xB1>(x);
    x = x + dpp_f64<0x4E>(x);
    x = x + dpp_f64<0x141>(x);
    x = x + dpp_f64<0x140>(x);
    return x;
}

// Sum over the 64 lanes of a wavefront in a fixed tree: neighbours, pairs,
// half rows and rows of 16 lanes by DPP (each step adds two equal partial sums
// in both orders, which commutativity makes bitwise equal), then the four row
// sums as (r0 + r1) + (r2 + r3).  The result is uniform.  Every lane of the
// wave must be active.
__device__ __forceinline__ double wave_sum_f64(double x) {
    x = x + dpp_f64<0xB1>(x);
    x = x + dpp_f64<0x4E>(x);
    x = x + dpp_f64<0x141>(x);
    x = x + dpp_f64<0x140>(x);
    return (readlane_f64(x, 0) + readlane_f64(x, 16)) + (readlane_f64(x, 32) + readlane_f64(x, 48));
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
    uint64_t x = v;
    x += dpp_u64<0xB1>(x);
    x += dpp_u64<0x4E>(x);
    x += dpp_u64<0x141>(x);
    x += dpp_u64<0x140>(x);
    return (readlane_u64(x, 0) + readlane_u64(x, 16)) + (readlane_u64(x, 32) + readlane_u64(x, 48));
}

}  // namespace detail

using namespace detail;

// ----------------------------------------------------------- one task
// Per-wave LDS scratch of run_group (16-byte aligned size: the hot-row copies
// that may follow the wave scratch are read as 16-byte records).
template <typename WT, bool COND = false>
struct alignas(16) GroupLds {
    static constexpr uint32_t C = chunk_walkers(sizeof(WT) == sizeof(float));
    WT fval[C];                   // W v[X_t] of list[i]
    double K[kGroupMax];          // value of a walker that never leaves the start node
                                  // (first-jump conditioning: e^{-rt} times that value)
    uint32_t node[kGroupMax];     // start node of each entry (UINT32_MAX: out of range)
    uint32_t n0[kGroupMax];       // walkers of entry g that never jump | its walker count << 16
    uint32_t ord0[kGroupMax];     // first walker ordinal of entry g's chunk
    uint16_t seg[kGroupMax + 1];  // entry g's jumpers are list[seg[g] .. seg[g+1])
    uint16_t list[C];             // jumpers: (entry << 10) | ordinal, entry-major, ordinal order
    double q[COND ? kGroupMax : 1];  // first-jump conditioning: 1 - e^{-rt} of the start node
};
static_assert(kGroupMax <= 64 && kChunkMax <= 1024, "list codes are 6 + 10 bits");

// Where a task's per-entry results go: entry e_first + g, one of `chunks` chunks.
// With var_task set, the task's "entries" are the chunk slots s0 .. s0+G-1 of
// entries with their own walker counts (slot s is chunk s - var_task[e] of the
// entry e with var_task[e] <= s < var_task[e+1], of var_nwalk[e] walkers), and
// every slot writes its partial to part[s].
struct GroupOut {
    double *est, *se, *part;
    int64_t e_first, chunks;
    int64_t pbase;             // partial of entry e_first + g at this chunk: pbase + g * chunks
    const int64_t *var_task = nullptr, *var_nwalk = nullptr;
    int64_t s0 = 0, k = 0;
};

// Runs walkers ord0 .. ord0+cnt-1 of G entries on the calling wavefront and
// writes each entry's estimate (or its chunk's (count, mean, M2)).  All lanes
// of the wave call it together; lds is this wave's scratch.
//
// Phase 1 draws only the first event of every walker of the entries whose
// no-jump probability e^{-r t} is at least 1/8: a walker with U below
// e0 = e^{-rt}(1 - 2^-16), evaluated in FP32 (error below 1e-6, so e0 stays
// below e^{-rt}(1 - 2^-17)), certainly holds past t (-log(U)/r > t + 2^-17/r,
// far beyond the logarithm's rounding) and returns exactly K, so only a count
// is kept; the others are appended to a list, as are all walkers of the other
// entries.  Phase 2 runs the complete walk for the listed walkers with lane
// refill (their first event drawn again from the same counter), so the rarely
// needed logarithm, jump and exp code runs on lanes that need it.  Every
// finished walker writes its value to the slot of its list position, and each
// entry's mean and M2 come from a two-pass reduction over its slots in a fixed
// order plus its n0 copies of K: the result does not depend on which lane ran
// which walker, nor on how many entries share the task.  When the entries'
// listed walkers do not all fit the list at once, phases 1 and 2 alternate in
// sessions (see below); with RESORT (relabelled tables only) the wave re-sorts
// its walkers by current node every P.resort events.
// Entries whose listed walkers are summed by one lane, or by one row of 16
// lanes, rather than by the whole wave.
constexpr uint32_t kShortSeg = 32;
constexpr uint32_t kRowSeg = 256;

// An entry's statistics: the estimate and standard error, or its (count, mean,
// M2) partial when it spans several chunks or has its own walker count.
__device__ __forceinline__ void put_stats(const GroupOut &out, uint32_t g, double mean, double m2,
                                          double count) {
    if (out.var_task) {
        double *pp = out.part + (out.s0 + (int64_t)g) * 3;
        pp[0] = count;
        pp[1] = mean;
        pp[2] = m2;
    } else if (out.chunks == 1) {
        const int64_t e = out.e_first + g;
        out.est[e] = mean;
        if (out.se) out.se[e] = count > 1.0 ? sqrt(m2 / (count - 1.0) / count) : 0.0;
    } else {
        double *pp = out.part + (out.pbase + (int64_t)g * out.chunks) * 3;
        pp[0] = count;
        pp[1] = mean;
        pp[2] = m2;
    }
}

template <int MODE, bool FP32, bool PROP, bool TRACE, bool LOC, bool COND, bool RESORT = false,
          int FAT = 0, bool QMC = false, bool STENCIL = false>
__device__ __forceinline__ void run_group(const InstArgs &P, const int64_t *idx, int64_t n,
                                          uint32_t G, uint32_t ord0, uint32_t cnt,
                                          const TraceOut &tr, const GroupOut &out,
                                          GroupLds<typename WeightT<FP32>::T, COND> &L,
                                          unsigned long long &my_events,
                                          unsigned long long &my_jumps, uint32_t &err_out) {
    using WT = typename WeightT<FP32>::T;
    const int lane = threadIdx.x & (WAVE - 1);
    const double t = P.t;
    uint32_t err = 0;
    // the task's shape is the same in every lane: scalar registers and scalar branches
    G = __builtin_amdgcn_readfirstlane(G);
    ord0 = __builtin_amdgcn_readfirstlane(ord0);
    cnt = __builtin_amdgcn_readfirstlane(cnt);

    constexpr uint32_t C = GroupLds<WT, COND>::C;

    // ---- per-entry setup, one lane per entry (or per chunk slot)
    double e0 = 0.0;
    if (lane < (int)G) {
        int64_t e = out.e_first + lane;
        uint32_t ordg = ord0, cntg = cnt;
        if (out.var_task) {
            const int64_t sl = out.s0 + lane;
            int64_t lo = 0, hi = out.k - 1;
            while (lo < hi) {
                const int64_t mid = (lo + hi + 1) >> 1;
                if (out.var_task[mid] <= sl) lo = mid;
                else hi = mid - 1;
            }
            e = lo;
            const int64_t c = sl - out.var_task[lo];
            const int64_t rem = out.var_nwalk[lo] - c * (int64_t)C;
            cntg = (uint32_t)(rem < (int64_t)C ? rem : (int64_t)C);
            ordg = ord0 + (uint32_t)(c * (int64_t)C);
        }
        L.ord0[lane] = ordg;
        L.n0[lane] = cntg << 16;
        const int64_t nd = idx ? idx[e] : e;
        uint32_t node = 0xFFFFFFFFu;
        double K = 0.0;
        if (nd >= 0 && nd < n) {
            node = (uint32_t)nd;
            const uint32_t x0 = walk_id<LOC>(P, node);
            RowRec r0;
            WT d0;
            r0 = row_at<LOC>(P, x0);
            d0 = d_at<FP32, LOC>(P, x0);
            const WT v0 = load_v<FP32>(P.v, node);
            K = (double)(wexp<FP32>(final_term<MODE, FP32>(d0, 0.0, 0, P)) * v0);
            // first-jump conditioning (start nodes with exits and r t <= cond_max_rt):
            // every walker is sampled given a jump before t and the no-jump event
            // enters as e^{-rt} K; q = 1 - e^{-rt} > 0 marks such an entry
            double q = 0.0;
            if (COND && r0.deg && t <= P.cond_max_rt * r0.inv_r) {
                const double rt = t / r0.inv_r;
                q = one_minus_exp_neg(rt);
            }
            if constexpr (COND) L.q[lane] = q;
            if (q > 0.0) {
                K = exp_f64(-t / r0.inv_r) * K;
                e0 = 0.0;                 // list every walker
            } else {
                // e^{-rt} in FP32 (relative error below 1e-6 where e0 >= 1/8 matters),
                // lowered by 2^-16; 2: never jumps
                e0 = r0.deg ? (double)exp2f((float)(-t / r0.inv_r) * 1.44269504f) * (1.0 - 0x1p-16)
                            : 2.0;
            }
        } else {
            err |= F_OUT_OF_RANGE;
        }
        L.node[lane] = node;
        L.K[lane] = K;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    // ---- sessions: phase 1 appends the possibly-jumping walkers of consecutive
    // entries to the LDS pool while they fit; a full pool is flushed (phase 2 and
    // the statistics of its entries) and the entry that did not fit is redone in
    // an empty pool, where it always fits (cnt <= C).  An entry's values and its
    // reduction do not depend on which session it falls in.
    uint32_t nlist = 0, g_begin = 0;
    unsigned long long evs = 0, jus = 0;
    uint32_t g = 0;
    for (;;) {
        for (; g < G;) {
            // LDS values the whole wave shares, read into scalar registers
            const uint32_t node = __builtin_amdgcn_readfirstlane(L.node[g]);
            const uint32_t cg = __builtin_amdgcn_readfirstlane(L.n0[g]) >> 16;   // its walkers
            const uint32_t og = __builtin_amdgcn_readfirstlane(L.ord0[g]);      // first ordinal
            const double eg = readlane_f64(e0, (int)g);
            const uint32_t start = nlist;
            if (lane == 0) L.seg[g] = start;
            if (node == 0xFFFFFFFFu) {
                ++g;
                continue;
            }
            if (eg >= 1.5) {
                // no exit rate: every walker holds until t, one holding interval each
                if (lane == 0) {
                    L.n0[g] = cg | (cg << 16);
                    evs += cg;
                }
                if constexpr (TRACE) {
                    for (uint32_t w = lane; w < cg; w += WAVE) {
                        tr.x[tr.base + w] = (int32_t)node;
                        tr.ev[tr.base + w] = 1;
                        tr.ju[tr.base + w] = 0;
                        tr.f[tr.base + w] = L.K[g];
                    }
                }
                ++g;
                continue;
            }
            bool fits = true;
            uint32_t stay = 0;
            if (eg < 0.125) {
                // most walkers leave: list them all
                if (nlist + cg > C) {
                    fits = false;
                } else {
                    for (uint32_t w = lane; w < cg; w += WAVE) L.list[nlist + w] = (uint16_t)((g << 10) | w);
                    nlist += cg;
                }
            } else {
                // U >= e0  <=>  m + 1 >= e0 2^53 (U = (m+1) 2^-53 exactly), i.e. m + 1 >= ceil(e0 2^53)
                const uint64_t m_thr = (uint64_t)ceil(eg * 0x1p53);
                const uint64_t t_pair = (((m_thr - 1ull) >> 21) << 32) | (((m_thr - 1ull) & 0x1FFFFFull) << 11);
                // lattice first events: a chunk starting on a replicate boundary is one
                // replicate (every run but a per-walker trace from an unaligned
                // ordinal), whose shift the whole entry shares
                const uint32_t qb = qmc_bits(FP32);
                const bool one_rep = QMC && (og & ((1u << qb) - 1u)) == 0u;
                const U4 shift = one_rep ? philox(kQmcShiftMark, og >> qb, node, P.inst, P.key0,
                                                  P.key1)
                                         : U4{0u, 0u, 0u, 0u};
                for (uint32_t b = 0; b < cg; b += WAVE) {
                    if (nlist + WAVE > C) {
                        fits = false;
                        break;
                    }
                    const uint32_t w = b + (uint32_t)lane;
                    const bool valid = w < cg;
                    // drawn in every lane (a lane past the entry's walkers would idle
                    // under the exec mask anyway), so that `go` needs no branch
                    const uint32_t wo = og + w;
                    U4 o;
                    if constexpr (QMC) {
                        o = lattice_words(one_rep ? shift
                                                  : philox(kQmcShiftMark, wo >> qb, node, P.inst,
                                                           P.key0, P.key1),
                                          wo, qb);
                    } else {
                        o = philox(0u, wo, node, P.inst, P.key0, P.key1);
                    }
                    // m = o.x 2^21 + (o.y >> 11) >= T = m_thr - 1 compared without forming
                    // m: with T = A 2^21 + B (B < 2^21) it holds iff o.x > A, or o.x = A
                    // and o.y >= B 2^11, i.e. iff the word pair (o.x, o.y) >= (A, B 2^11)
                    const bool up = (((uint64_t)o.x << 32) | o.y) >= t_pair;
                    const bool go = valid && up;
                    // ballots of single comparisons, combined on the scalar unit
                    const unsigned long long vmask = lanes_where(valid);
                    // (the ballot taken by the comparison itself: a ballot of the bool
                    // `up` would turn it into a vector value and back)
                    const unsigned long long gmask =
                        vmask & __builtin_amdgcn_uicmpl(((uint64_t)o.x << 32) | o.y, t_pair,
                                                        kCmpUge);
                    if (go) L.list[nlist + set_below(gmask)] = (uint16_t)((g << 10) | w);
                    nlist += (uint32_t)__popcll(gmask);
                    stay += (uint32_t)__popcll(vmask & ~gmask);
                    if constexpr (TRACE) {
                        if (valid && !go) {
                            tr.x[tr.base + w] = (int32_t)node;
                            tr.ev[tr.base + w] = 1;
                            tr.ju[tr.base + w] = 0;
                            tr.f[tr.base + w] = L.K[g];
                        }
                    }
                }
            }
            if (!fits) {
                nlist = start;            // roll back entry g: it opens the next session
                break;
            }
            if (lane == 0) {
                L.n0[g] = stay | (cg << 16);
                evs += stay;
            }
            ++g;
        }
        const uint32_t g_end = g;
        if (lane == 0) L.seg[g_end] = nlist;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // ---- phase 2: full walks with lane refill over the list
        uint32_t wl = (uint32_t)lane;
        bool active = wl < nlist;
        uint32_t code = active ? L.list[wl] : 0u;
        uint32_t node = active ? L.node[code >> 10] : 0u;     // original id: RNG counter
        uint32_t wb = active ? L.ord0[code >> 10] : 0u;       // first ordinal of its chunk
        uint32_t x = walk_id<LOC>(P, node);                      // walk id
        double s = 0.0;
        WT logw = (WT)0;
        uint32_t ev = 0, ju = 0;
        int32_t ka = 0;
        double inv_r = 0.0;
        uint32_t deg = 0, begin = 0;
        WT dx = (WT)0;
        if (active) {
            const RowRec rr = row_at<LOC>(P, x);
            inv_r = rr.inv_r;
            deg = rr.deg;
            begin = rr.begin;
            dx = d_at<FP32, LOC>(P, x);
        }
        uint32_t next = WAVE;
        uint32_t since_sort = 0;

        // (tested at the bottom: lane 0 is active iff the list is not empty)
        if (nlist > 0) do {
            if constexpr (LOC && RESORT) {
                // relabelled tables: every P.resort events the walkers move to the
                // lanes of their sorted current walk ids, so that neighbouring lanes
                // gather neighbouring rows; each walker's whole state moves with it
                // (its list slot included), so no value changes
                if (++since_sort >= P.resort) {
                    since_sort = 0;
                    const int src = (int)sorted_source(x, active, lane);
                    wl = __shfl(wl, src, WAVE);
                    active = __shfl((int)active, src, WAVE) != 0;
                    code = __shfl(code, src, WAVE);
                    node = __shfl(node, src, WAVE);
                    wb = __shfl(wb, src, WAVE);
                    x = __shfl(x, src, WAVE);
                    s = __shfl(s, src, WAVE);
                    logw = __shfl(logw, src, WAVE);
                    ev = __shfl(ev, src, WAVE);
                    ju = __shfl(ju, src, WAVE);
                    ka = __shfl(ka, src, WAVE);
                    inv_r = __shfl(inv_r, src, WAVE);
                    deg = __shfl(deg, src, WAVE);
                    begin = __shfl(begin, src, WAVE);
                    dx = __shfl(dx, src, WAVE);
                }
            }
            bool fin = false;
            if (active) {
                // the rare walkers (no exit rate: holds until t; at the walk-length
                // cap) draw like the others and are settled after the draw, which
                // keeps the event block out of a nested branch
                const bool live = deg != 0 && ev < P.max_events;
                {
                    const uint32_t wo = wb + (code & 1023u);
                    U4 o;
                    if constexpr (QMC) {
                        const bool lat = ev == 0;
                        o = philox(lat ? kQmcShiftMark : ev, lat ? wo >> qmc_bits(FP32) : wo, node,
                                   P.inst, P.key0, P.key1);
                        if (lat) o = lattice_words(o, wo, qmc_bits(FP32));
                    } else {
                        o = philox(ev, wo, node, P.inst, P.key0, P.key1);
                    }
                    ev += (live || deg == 0) ? 1u : 0u;
                    const uint64_t m = ((uint64_t)o.x << 21) | ((uint64_t)o.y >> 11);
                    double S;
                    bool forced = false;
                    if constexpr (COND) {
                        const double qe = ev == 1 ? L.q[code >> 10] : 0.0;
                        if (qe > 0.0) {
                            // first holding time given a jump before t: inverse of the
                            // exponential law truncated to [0, t), U in [0, 1)
                            const double U = (double)m * 0x1p-53;
                            S = -log_unit(1.0 - U * qe) * inv_r;
                            forced = true;
                        } else {
                            S = -log_unit((double)(m + 1ull) * 0x1p-53) * inv_r;
                        }
                    } else {
                        const double U = (double)(m + 1ull) * 0x1p-53;
                        S = -log_unit(U) * inv_r;
                    }
                    const double sn = s + S;
                    if (live && (forced || sn < t)) {
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
                        const uint32_t js = begin + sl;
                        // FAT: 0 separate tables, 1 64-byte slots, 2 whichever P holds
                        bool keep = true;
                        if constexpr (STENCIL) {
                            x = stencil_jump(P, x, deg, begin, o.z);
                            const RowRec rr = row_at<false>(P, x);
                            inv_r = rr.inv_r;
                            deg = rr.deg;
                            begin = rr.begin;
                            dx = d_at<FP32, false>(P, x);
                        } else if constexpr (FAT == 1)
                            keep = jump_fat<FP32>(P, js, o.w, x, inv_r, deg, begin, dx);
                        else if constexpr (FAT == 2)
                            keep = P.fat ? jump_fat<FP32>(P, js, o.w, x, inv_r, deg, begin, dx)
                                         : jump_sep<FP32, LOC>(P, js, o.w, x, inv_r, deg, begin, dx);
                        else
                            keep = jump_sep<FP32, LOC>(P, js, o.w, x, inv_r, deg, begin, dx);
                        if constexpr (PROP) {
                            const float2 cr = P.corr[js];
                            logw = logw + (WT)(keep ? cr.x : cr.y);
                        }
                        ++ju;
                    } else {
                        fin = true;
                        if (!live && deg != 0) err |= F_WALK_LIMIT;
                    }
                }
                if (fin) {
                    WT f;
                    if (ju == 0) {
                        f = (WT)L.K[code >> 10];         // never left the start node
                    } else {
                        logw = logw + final_term<MODE, FP32>(dx, s, ka, P);
                        f = wexp<FP32>(logw) * load_v<FP32>(P.v, orig_id<LOC>(P, x));
                        if constexpr (COND) {
                            const uint32_t e = code >> 10;
                            if (L.q[e] > 0.0) f = (WT)(L.K[e] + L.q[e] * (double)f);
                        }
                    }
                    L.fval[wl] = f;
                    evs += ev;
                    jus += ju;
                    if constexpr (TRACE) {
                        const int64_t ti = tr.base + (code & 1023u);
                        tr.x[ti] = (int32_t)orig_id<LOC>(P, x);
                        tr.ev[ti] = ev;
                        tr.ju[ti] = ju;
                        tr.f[ti] = (double)f;
                    }
                }
            }
            const unsigned long long fmask = lanes_where(fin);
            if (fin) {
                wl = next + set_below(fmask);
                if (wl < nlist) {
                    code = L.list[wl];
                    node = L.node[code >> 10];
                    wb = L.ord0[code >> 10];
                    x = walk_id<LOC>(P, node);
                    s = 0.0;
                    logw = (WT)0;
                    ev = 0;
                    ju = 0;
                    ka = 0;
                    const RowRec rr = row_at<LOC>(P, x);
                    inv_r = rr.inv_r;
                    deg = rr.deg;
                    begin = rr.begin;
                    dx = d_at<FP32, LOC>(P, x);
                } else {
                    active = false;
                }
            }
            next += (uint32_t)__popcll(fmask);
        } while (__builtin_amdgcn_uicmp(wl, nlist, kCmpUlt) != 0ull);   // = lanes_where(active)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // ---- per-entry statistics: slots in a fixed order, plus n0 copies of K.
        // Entries with at most kShortSeg listed walkers: one lane each (a session
        // holds at most 64 entries), sums in slot order; up to kRowSeg: one row of
        // 16 lanes each; the others: the whole wave, lanes striding the segment,
        // then a fixed tree.  Which one depends only on the entry's own walkers,
        // so packing changes no result.
        // lane l looks at entry g_begin + l (a session holds at most 64 entries) and
        // the wave learns which entries take the row tree and which the wave tree
        unsigned long long rowm, widem;
        {
            const uint32_t g = g_begin + (uint32_t)lane;
            const bool in = g < g_end;
            const uint32_t b0 = in ? L.seg[g] : 0u, J = in ? L.seg[g + 1] - b0 : 0u;
            rowm = lanes_where(in && J > kShortSeg && J <= kRowSeg);
            widem = lanes_where(in && J > kRowSeg);
            if (in && J <= kShortSeg) {
                double mean, m2, count;
                if (L.node[g] == 0xFFFFFFFFu) {
                    mean = NAN;
                    m2 = NAN;
                    count = 1.0;
                } else {
                    const double K = L.K[g];
                    const uint32_t n0w = L.n0[g];
                    const uint32_t n0 = n0w & 0xFFFFu;
                    const double nn0 = (double)n0;
                    count = (double)(n0w >> 16);
                    if (n0 && !isfinite(K)) err |= F_OVERFLOW;
                    double s1 = 0.0;
                    for (uint32_t i = 0; i < J; ++i) s1 += (double)L.fval[b0 + i];
                    if (!isfinite(s1)) err |= F_OVERFLOW;      // a walker's value is not finite
                    mean = n0 ? (nn0 * K + s1) / count : s1 / count;
                    double s2 = 0.0;
                    for (uint32_t i = 0; i < J; ++i) {
                        const double dv = (double)L.fval[b0 + i] - mean;
                        s2 += dv * dv;
                    }
                    const double dk = K - mean;
                    m2 = n0 ? s2 + nn0 * dk * dk : s2;
                }
                put_stats(out, g, mean, m2, count);
            }
        }
        // entries of kShortSeg+1 .. kRowSeg listed walkers: four at a time, one per
        // row of 16 lanes (lanes of a row stride the segment, then the row tree)
        while (rowm) {
            // the next (up to) four of them, lowest first
            const uint32_t sel0 = g_begin + (uint32_t)__builtin_ctzll(rowm);
            rowm &= rowm - 1ull;
            uint32_t sel1 = sel0, sel2 = sel0, sel3 = sel0, m = 1;
            if (rowm) {
                sel1 = g_begin + (uint32_t)__builtin_ctzll(rowm);
                rowm &= rowm - 1ull;
                m = 2;
            }
            if (rowm) {
                sel2 = g_begin + (uint32_t)__builtin_ctzll(rowm);
                rowm &= rowm - 1ull;
                m = 3;
            }
            if (rowm) {
                sel3 = g_begin + (uint32_t)__builtin_ctzll(rowm);
                rowm &= rowm - 1ull;
                m = 4;
            }
            const uint32_t r = (uint32_t)lane >> 4, rl = (uint32_t)lane & 15u;
            const bool act = r < m;          // rows past m repeat the first entry, unwritten
            const uint32_t g = r == 1 ? sel1 : r == 2 ? sel2 : r == 3 ? sel3 : sel0;
            const uint32_t b0 = L.seg[g], J = L.seg[g + 1] - b0;
            const bool bad = L.node[g] == 0xFFFFFFFFu;
            const double K = L.K[g];
            const uint32_t n0w = L.n0[g];
            const uint32_t n0 = n0w & 0xFFFFu;
            const double nn0 = (double)n0;
            double count = (double)(n0w >> 16);
            if (act && !bad && n0 && !isfinite(K)) err |= F_OVERFLOW;
            double s1 = 0.0;
            for (uint32_t i = rl; i < J; i += 16) s1 += (double)L.fval[b0 + i];
            s1 = row_sum_f64(s1);
            if (act && !isfinite(s1)) err |= F_OVERFLOW;
            double mean = n0 ? (nn0 * K + s1) / count : s1 / count;
            double s2 = 0.0;
            for (uint32_t i = rl; i < J; i += 16) {
                const double dv = (double)L.fval[b0 + i] - mean;
                s2 += dv * dv;
            }
            s2 = row_sum_f64(s2);
            const double dk = K - mean;
            double m2 = n0 ? s2 + nn0 * dk * dk : s2;
            if (bad) {
                mean = NAN;
                m2 = NAN;
                count = 1.0;
            }
            if (act && rl == 0) put_stats(out, g, mean, m2, count);
        }
        for (; widem; widem &= widem - 1ull) {
            const uint32_t g = g_begin + (uint32_t)__builtin_ctzll(widem);
            const uint32_t b0 = __builtin_amdgcn_readfirstlane(L.seg[g]);
            const uint32_t b1 = __builtin_amdgcn_readfirstlane(L.seg[g + 1]);
            double mean, m2, count;
            if (L.node[g] == 0xFFFFFFFFu) {
                mean = NAN;
                m2 = NAN;
                count = 1.0;
            } else {
                const double K = L.K[g];
                const uint32_t n0w = __builtin_amdgcn_readfirstlane(L.n0[g]);
                const uint32_t n0 = n0w & 0xFFFFu;
                const double nn0 = (double)n0;
                count = (double)(n0w >> 16);
                // K enters only through the walkers that stayed: without any, an
                // infinite K (e^{td} v beyond the FP32 range, taken by no walker)
                // must not turn 0 * K into NaN; with some, it is an overflow
                if (n0 && !isfinite(K)) err |= F_OVERFLOW;
                // lanes stride from the segment start, so the summation tree depends only on
                // the entry's own walkers
                const uint32_t J = b1 - b0;
                double s1 = 0.0;
                for (uint32_t i = lane; i < J; i += WAVE) s1 += (double)L.fval[b0 + i];
                s1 = wave_sum_f64(s1);
                if (!isfinite(s1)) err |= F_OVERFLOW;
                mean = n0 ? (nn0 * K + s1) / count : s1 / count;
                double s2 = 0.0;
                for (uint32_t i = lane; i < J; i += WAVE) {
                    const double dv = (double)L.fval[b0 + i] - mean;
                    s2 += dv * dv;
                }
                s2 = wave_sum_f64(s2);
                const double dk = K - mean;
                m2 = n0 ? s2 + nn0 * dk * dk : s2;
            }
            if (lane == 0) put_stats(out, g, mean, m2, count);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (g_end >= G) break;
        nlist = 0;
        g_begin = g_end;
    }
    my_events += wave_sum_u64(evs);
    my_jumps += wave_sum_u64(jus);
    err_out |= err;
}

}  // namespace mc
