// The forward estimator of the full vector (paper Lemma 2, Theorem 2 and
// Algorithm 2): walkers start at node j with probability |v_j| / V,
// V = sum_l |v_l|, evolve forward in time under the same jump law (the
// generator is symmetric, so forward and backward chains coincide), and add
// V sign(v_j) W to the entry of the state where they stop at t.  The value
// credited to node i is then an unbiased estimate of (e^{tA^T} v)_i, which is
// (e^{tA} v)_i for the symmetric A the paper assumes (the library checks it).
//
// Random numbers: walker w draws its start from the Philox counter
// (0, w, 0xFFFFFFFF, instance) and its k-th holding interval (k = 1, 2, ...)
// from (k, w, 0xFFFFFFFF, instance); 0xFFFFFFFF is never a node id, so these
// streams are disjoint from every backward walk.
//
// Work decomposition: a task is a chunk of kFwdChunk consecutive walker
// ordinals, one wavefront per task, one walker per lane with lane refill.
// Each finished walker adds Y and Y^2 to its end node with FP64 atomics (so
// per-node sums are exact up to the order of the additions) and writes Y to
// the LDS slot of its ordinal; the chunk's (count, mean, M2) of Y comes from a
// fixed-order two-pass sum and the chunks merge in order, so the estimate of
// sum_i x_i is bitwise reproducible.
#include <math.h>


#include "walk_task.hpp"

namespace mc {

namespace {

constexpr uint32_t kFwdMark = 0xFFFFFFFFu;

// Sum of the grid coefficients c_{N-k} over ka <= k <= kb: the backward
// coefficients read in reverse time order.
template <int MODE>
__device__ __forceinline__ double grid_coef_sum_rev(int32_t ka, int32_t kb, int32_t ngrid) {
    if (kb < ka) return 0.0;
    return grid_coef_sum<MODE>(ngrid - kb, ngrid - ka, ngrid);
}

// Guide-table cell of a cumulative value c: min(G, floor(c G / V)), non-decreasing
// in c (all the lookup relies on).
__device__ __forceinline__ int64_t guide_cell(double c, double scale, int64_t G) {
    const double k = floor(c * scale);
    return k >= (double)G ? G : (int64_t)k;
}

// Start node of walker w: the first j with cdf[j] >= U V.  The guide table
// (Chen and Asau, 1974) holds for every cell k the first node j whose cell is
// >= k; the answer's cell is >= the target's, so the search walks forward from
// guide[cell(target)], over about n / G nodes (one or two cache lines).  cdf is
// the device's parallel prefix sum; should its rounding ever make a node of
// zero weight the answer, the next node of non-zero weight is taken instead.
__device__ __forceinline__ uint32_t draw_start(const FwdArgs &a, uint32_t w, double V,
                                               double scale, double &vj) {
    const U4 o = philox(0u, w, kFwdMark, a.P.inst, a.P.key0, a.P.key1);
    const uint64_t m = ((uint64_t)o.x << 21) | ((uint64_t)o.y >> 11);
    const double target = (double)(m + 1ull) * 0x1p-53 * V;
    int64_t j = a.guide[guide_cell(target, scale, a.gcells)];
    while (a.cdf[j] < target) ++j;          // stops at n - 1 at the latest: cdf[n-1] = V
    // the sign of v[j] is needed anyway; v[j] = 0 only where the scan's rounding made
    // the sums non-increasing, and then the nearest node with weight is taken
    int8_t sg = a.vsign[j];
    if (sg == 0) {
        int64_t k = j;
        while (k < a.n - 1 && a.absv[k] == 0.0) ++k;
        if (a.absv[k] == 0.0)
            while (k > 0 && a.absv[k] == 0.0) --k;
        j = k;
        sg = a.vsign[j];
    }
    vj = (double)sg;
    return (uint32_t)j;
}

template <int MODE, bool FP32, bool TRACE>
__global__ __launch_bounds__(64) void k_forward(FwdArgs a) {
    using WT = typename WeightT<FP32>::T;
    __shared__ double ys[kFwdChunk];
    const int lane = threadIdx.x & (WAVE - 1);
    const InstArgs &P = a.P;
    const double t = P.t;
    const double V = a.n > 0 ? a.cdf[a.n - 1] : 0.0;
    const double gscale = (double)a.gcells / V;
    unsigned long long evs = 0, jus = 0;
    uint32_t err = 0;
    for (int64_t c = blockIdx.x; c < a.chunks; c += gridDim.x) {
        const int64_t wbase = c * (int64_t)kFwdChunk;
        const int64_t rem = a.nwalk - wbase;
        const uint32_t cnt = (uint32_t)(rem < (int64_t)kFwdChunk ? rem : (int64_t)kFwdChunk);
        const uint32_t ord0 = (uint32_t)(a.w0 + wbase);
        if (!(V > 0.0)) {
            // v = 0: every walker contributes 0
            for (uint32_t i = lane; i < cnt; i += WAVE) {
                ys[i] = 0.0;
                if constexpr (TRACE) {
                    a.t_start[wbase + i] = -1;
                    a.t_end[wbase + i] = -1;
                    a.t_ev[wbase + i] = 0;
                    a.t_ju[wbase + i] = 0;
                    a.t_y[wbase + i] = 0.0;
                }
            }
        } else {
            // walker state of this lane
            uint32_t wl = (uint32_t)lane;
            bool active = wl < cnt;
            uint32_t j = 0, x = 0, ev = 0, ju = 0, deg = 0, begin = 0;
            double s = 0.0, inv_r = 0.0, sgn = 1.0;
            int32_t ka = 0;
            WT logw = (WT)0, dx = (WT)0;
            auto start = [&](uint32_t i) {
                double vj;
                j = draw_start(a, ord0 + i, V, gscale, vj);
                sgn = vj > 0.0 ? 1.0 : -1.0;
                x = P.perm ? P.perm[j] : j;
                const FwdRow fr = a.frows[x];
                inv_r = fr.inv_r;
                deg = fr.deg;
                begin = fr.begin;
                dx = FP32 ? (WT)fr.d32 : (WT)fr.d64;
                s = 0.0;
                logw = (WT)0;
                ev = 0;
                ju = 0;
                ka = 0;
            };
            if (active) start(wl);
            uint32_t next = WAVE;
            // (tested at the bottom: lane 0 is active iff the chunk has walkers)
            if (cnt > 0) do {
                bool fin = false;
                if (active) {
                    if (deg == 0) {
                        ++ev;
                        fin = true;
                    } else if (ev >= P.max_events) {
                        err |= F_WALK_LIMIT;
                        fin = true;
                    } else {
                        const U4 o = philox(ev + 1u, ord0 + wl, kFwdMark, P.inst, P.key0, P.key1);
                        ++ev;
                        const uint64_t m = ((uint64_t)o.x << 21) | ((uint64_t)o.y >> 11);
                        const double U = (double)(m + 1ull) * 0x1p-53;
                        const double S = -log_unit(U) * inv_r;
                        const double sn = s + S;
                        if (sn < t) {
                            if constexpr (MODE == MC_EXACT) {
                                logw = logw + dx * (WT)S;
                            } else {
                                const int32_t kb = grid_index(sn, P.inv_dt, P.ngrid);
                                const double cs = grid_coef_sum_rev<MODE>(ka, kb - 1, P.ngrid);
                                logw = logw + dx * (WT)(cs * P.dt);
                                ka = kb;
                            }
                            s = sn;
                            const uint32_t sl = (uint32_t)(((uint64_t)o.z * (uint64_t)deg) >> 32);
                            const SlotRec q = P.slots[begin + sl];
                            x = (uint32_t)(o.w < q.thr ? q.self : q.alias);
                            ++ju;
                            const FwdRow fr = a.frows[x];
                            inv_r = fr.inv_r;
                            deg = fr.deg;
                            begin = fr.begin;
                            dx = FP32 ? (WT)fr.d32 : (WT)fr.d64;
                        } else {
                            fin = true;
                        }
                    }
                    if (fin) {
                        if constexpr (MODE == MC_EXACT) {
                            logw = logw + dx * (WT)(t - s);
                        } else {
                            const double cs = grid_coef_sum_rev<MODE>(ka, P.ngrid, P.ngrid);
                            logw = logw + dx * (WT)(cs * P.dt);
                        }
                        const double y = V * sgn * (double)wexp<FP32>(logw);
                        if (!isfinite(y)) err |= F_OVERFLOW;
                        const uint32_t xe = P.inv ? P.inv[x] : x;
                        if (a.acc1) unsafeAtomicAdd(a.acc1 + xe, y);
                        if (a.acc2) unsafeAtomicAdd(a.acc2 + xe, y * y);
                        ys[wl] = y;
                        evs += ev;
                        jus += ju;
                        if constexpr (TRACE) {
                            a.t_start[wbase + wl] = (int32_t)j;
                            a.t_end[wbase + wl] = (int32_t)xe;
                            a.t_ev[wbase + wl] = ev;
                            a.t_ju[wbase + wl] = ju;
                            a.t_y[wbase + wl] = y;
                        }
                    }
                }
                const unsigned long long fmask = lanes_where(fin);
                if (fin) {
                    wl = next + set_below(fmask);
                    if (wl < cnt) start(wl);
                    else active = false;
                }
                next += (uint32_t)__popcll(fmask);
            } while (lanes_where(active) != 0ull);
        }
        __syncthreads();
        // chunk statistics of Y in ordinal order: two passes, fixed DPP tree
        double s1 = 0.0;
        for (uint32_t i = lane; i < cnt; i += WAVE) s1 += ys[i];
        const double mean = wave_sum_f64(s1) / (double)cnt;
        double s2 = 0.0;
        for (uint32_t i = lane; i < cnt; i += WAVE) {
            const double dv = ys[i] - mean;
            s2 += dv * dv;
        }
        const double m2 = wave_sum_f64(s2);
        if (lane == 0) {
            a.part[3 * c] = (double)cnt;
            a.part[3 * c + 1] = mean;
            a.part[3 * c + 2] = m2;
        }
        __syncthreads();
    }
    for (int off = 1; off < WAVE; off <<= 1) err |= __shfl_xor(err, off, WAVE);
    if (err && lane == 0) atomicOr(a.flags, err);
    const unsigned long long e = wave_sum_u64(evs), jn = wave_sum_u64(jus);
    if (lane == 0) {
        a.counters[2 * blockIdx.x] = e;
        a.counters[2 * blockIdx.x + 1] = jn;
    }
}

// Guide table: for every cell k = 0..G, the first node j with cell(cdf[j]) >= k
// (binary search; n - 1 when there is none).  One thread per cell, no races.
__global__ void k_fwd_guide(int64_t n, int64_t G, const double *__restrict__ cdf,
                            int32_t *__restrict__ guide) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k > G) return;
    const double V = cdf[n - 1];
    if (!(V > 0.0)) return;
    const double scale = (double)G / V;
    int64_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (guide_cell(cdf[mid], scale, G) >= k) hi = mid;
        else lo = mid + 1;
    }
    guide[k] = (int32_t)lo;
}

// The forward walks' merged state records.
__global__ void k_fwd_rows(int64_t n, const RowRec *__restrict__ rows, const double *__restrict__ d64,
                           const float *__restrict__ d32, FwdRow *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const RowRec r = rows[i];
    FwdRow f;
    f.inv_r = r.inv_r;
    f.deg = r.deg;
    f.begin = r.begin;
    f.d64 = d64[i];
    f.d32 = d32[i];
    f.pad = 0u;
    out[i] = f;
}

// acc1 = acc2 = 0 (a kernel, so the sequence can be captured in a graph).
__global__ void k_fwd_zero(int64_t n, double *acc1, double *acc2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    acc1[i] = 0.0;
    if (acc2) acc2[i] = 0.0;
}

// Inclusive sums of |v| in FP64, written here rather than taken from a library so
// that their order is fixed and visible.  Tiles of kScanTile values, kScanItems
// consecutive ones per thread: a thread's values are summed left to right, the
// thread sums of a tile are scanned left to right by one lane (so the last prefix of
// a thread equals the next thread's starting sum bit for bit, and the tile's last
// prefix its total), and the tile totals are scanned left to right by one lane.  A
// prefix is offset(tile) + (start of its thread + running sum within the thread):
// non-decreasing in i (every step adds a non-negative value to one summand, and
// rounding is monotone) and deterministic; its rounding differs from a plain
// left-to-right sum in the last bits.  The first pass also writes |v| and the sign
// of each entry.
constexpr int kScanItems = 16;
constexpr int kScanThreads = 256;
constexpr int64_t kScanTile = (int64_t)kScanItems * kScanThreads;

int64_t scan_tiles(int64_t n) { return (n + kScanTile - 1) / kScanTile; }

template <bool FP32>
__global__ __launch_bounds__(kScanThreads) void k_fwd_scan_tiles(int64_t n, const void *v,
                                                                 double *__restrict__ absv,
                                                                 int8_t *__restrict__ sign,
                                                                 double *__restrict__ local,
                                                                 double *__restrict__ tsum) {
    // the tile passes through LDS so that global loads and stores stay coalesced
    // (position p = 256 k + t for lane t) while each thread scans its own 16
    // consecutive values (row p / 16, padded to 17 against bank conflicts)
    __shared__ double tile[kScanThreads * (kScanItems + 1)];
    __shared__ double sh[kScanThreads + 1];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int p = k * kScanThreads + t;
        const int64_t i = base + p;
        double a = 0.0;
        if (i < n) {
            const double x = (double)load_v<FP32>(v, (uint32_t)i);
            a = fabs(x);
            absv[i] = a;
            sign[i] = x > 0.0 ? (int8_t)1 : (x < 0.0 ? (int8_t)-1 : (int8_t)0);
        }
        tile[(p / kScanItems) * (kScanItems + 1) + p % kScanItems] = a;
    }
    __syncthreads();
    double run = 0.0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        run = run + tile[t * (kScanItems + 1) + j];
        tile[t * (kScanItems + 1) + j] = run;
    }
    sh[t] = run;
    __syncthreads();
    if (t == 0) {
        double e = 0.0;
        for (int u = 0; u < kScanThreads; ++u) {
            const double su = sh[u];
            sh[u] = e;
            e = e + su;
        }
        sh[kScanThreads] = e;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int p = k * kScanThreads + t;
        const int64_t i = base + p;
        const int owner = p / kScanItems;
        if (i < n) local[i] = sh[owner] + tile[owner * (kScanItems + 1) + p % kScanItems];
    }
    if (t == 0) tsum[blockIdx.x] = sh[kScanThreads];
}

// Tile offsets: off[b] = sum of the totals of tiles 0 .. b-1, left to right (the
// totals pass through LDS 1024 at a time; one lane adds).
__global__ __launch_bounds__(256) void k_fwd_scan_offsets(int64_t tiles, const double *__restrict__ tsum,
                                                         double *__restrict__ off) {
    __shared__ double sh[1024];
    double e = 0.0;
    for (int64_t b0 = 0; b0 < tiles; b0 += 1024) {
        const int64_t m = tiles - b0 < 1024 ? tiles - b0 : 1024;
        for (int64_t u = threadIdx.x; u < m; u += blockDim.x) sh[u] = tsum[b0 + u];
        __syncthreads();
        if (threadIdx.x == 0)
            for (int64_t u = 0; u < m; ++u) {
                const double su = sh[u];
                sh[u] = e;
                e = e + su;
            }
        __syncthreads();
        for (int64_t u = threadIdx.x; u < m; u += blockDim.x) off[b0 + u] = sh[u];
        __syncthreads();
    }
}

// cdf[i] = off[tile of i] + local[i], in place.
__global__ void k_fwd_scan_add(int64_t n, const double *__restrict__ off, double *__restrict__ cdf) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    cdf[i] = off[i / kScanTile] + cdf[i];
}

// Per-node mean and standard error from the sums of Y and Y^2, in place.
__global__ void k_fwd_finish(int64_t n, int64_t m, double *acc1, double *acc2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double mean = acc1[i] / (double)m;
    acc1[i] = mean;
    if (acc2) {
        if (m > 1) {
            const double var = (acc2[i] - (double)m * mean * mean) / (double)(m - 1);
            acc2[i] = sqrt((var > 0.0 ? var : 0.0) / (double)m);
        } else {
            acc2[i] = 0.0;
        }
    }
}

// Mean and standard error of Y over all walkers: 1024 threads each merge a
// contiguous range of chunk partials in order, then neighbouring ranges merge
// pairwise in LDS (thread i takes in thread i + off), keeping chunk order.
__global__ __launch_bounds__(1024) void k_fwd_total(int64_t chunks, const double *part,
                                                    double *sum_out) {
    __shared__ double sn[1024], sm[1024], sq[1024];
    const int64_t T = blockDim.x;
    const int64_t i = threadIdx.x;
    const int64_t q = (chunks + T - 1) / T;
    const int64_t c0 = i * q, c1 = c0 + q < chunks ? c0 + q : chunks;
    double n = 0.0, mean = 0.0, m2 = 0.0;
    for (int64_t c = c0; c < c1; ++c) chan_merge(n, mean, m2, part[3 * c], part[3 * c + 1], part[3 * c + 2]);
    sn[i] = n;
    sm[i] = mean;
    sq[i] = m2;
    __syncthreads();
    for (int64_t off = 1; off < T; off <<= 1) {
        if ((i & (2 * off - 1)) == 0 && i + off < T) {
            double a = sn[i], b = sm[i], c = sq[i];
            chan_merge(a, b, c, sn[i + off], sm[i + off], sq[i + off]);
            sn[i] = a;
            sm[i] = b;
            sq[i] = c;
        }
        __syncthreads();
    }
    if (i == 0) {
        sum_out[0] = sm[0];
        sum_out[1] = sn[0] > 1.0 ? sqrt(sq[0] / (sn[0] - 1.0) / sn[0]) : 0.0;
    }
}

// A == A^T: for every stored off-diagonal position (i, j), the sum of the
// stored entries (i, j) equals the sum of the stored entries (j, i).
__global__ void k_check_symmetric(int64_t nnz, const int64_t *__restrict__ rowptr,
                                  const int32_t *__restrict__ rowof,
                                  const int32_t *__restrict__ col, const double *__restrict__ val,
                                  uint32_t *flag) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nnz) return;
    const int32_t i = rowof[p], j = col[p];
    if (i == j) return;
    double sij = 0.0, sji = 0.0;
    for (int64_t q = rowptr[i]; q < rowptr[i + 1]; ++q)
        if (col[q] == j) sij += val[q];
    for (int64_t q = rowptr[j]; q < rowptr[j + 1]; ++q)
        if (col[q] == i) sji += val[q];
    if (!(sij == sji)) atomicOr(flag, 1u);
}

}  // namespace

hipError_t launch_check_symmetric(int64_t nnz, const int64_t *rowptr, const int32_t *rowof,
                                  const int32_t *col, const double *val, uint32_t *flag,
                                  hipStream_t s) {
    if (nnz == 0) return hipSuccess;
    hipLaunchKernelGGL(k_check_symmetric, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, s, nnz,
                       rowptr, rowof, col, val, flag);
    return hipGetLastError();
}

hipError_t launch_fwd_rows(int64_t n, const InstArgs &P, FwdRow *frows, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fwd_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, P.rows,
                       P.d64, P.d32, frows);
    return hipGetLastError();
}

hipError_t launch_fwd_cdf(int64_t n, const void *v, bool fp32, double *absv, int8_t *vsign, double *cdf,
                          int32_t *guide, void *temp, size_t &temp_bytes, hipStream_t s) {
    const int64_t tiles = scan_tiles(n);
    if (!temp) {
        temp_bytes = sizeof(double) * 2 * (size_t)tiles;
        return hipSuccess;
    }
    if (n <= 0) return hipSuccess;
    if (tiles > 0x7FFFFFFF || temp_bytes < sizeof(double) * 2 * (size_t)tiles) return hipErrorInvalidValue;
    double *tsum = static_cast<double *>(temp), *off = tsum + tiles;
    if (fp32)
        hipLaunchKernelGGL(k_fwd_scan_tiles<true>, dim3((unsigned)tiles), dim3(kScanThreads), 0, s, n, v,
                           absv, vsign, cdf, tsum);
    else
        hipLaunchKernelGGL(k_fwd_scan_tiles<false>, dim3((unsigned)tiles), dim3(kScanThreads), 0, s, n, v,
                           absv, vsign, cdf, tsum);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fwd_scan_offsets, dim3(1), dim3(256), 0, s, tiles, tsum, off);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fwd_scan_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, off, cdf);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t G = guide_cells(n);
    hipLaunchKernelGGL(k_fwd_guide, dim3((unsigned)((G + 256) / 256)), dim3(256), 0, s, n, G, cdf,
                       guide);
    return hipGetLastError();
}

int forward_grid(int64_t chunks) {
    int64_t g = chunks < (int64_t)kMaxWalkGrid ? chunks : (int64_t)kMaxWalkGrid;
    return (int)(g < 1 ? 1 : g);
}

hipError_t launch_forward(const FwdArgs &a, int mode, bool fp32, bool trace, double *sum_out,
                          hipStream_t s) {
    const unsigned gz = (unsigned)((a.n + 255) / 256);
    if (a.n > 0 && a.acc1) {
        hipLaunchKernelGGL(k_fwd_zero, dim3(gz), dim3(256), 0, s, a.n, a.acc1, a.acc2);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const dim3 grid((unsigned)forward_grid(a.chunks)), block(64);
#define MC_FWD(M, F, T) hipLaunchKernelGGL((k_forward<M, F, T>), grid, block, 0, s, a)
    switch (mode * 4 + (fp32 ? 2 : 0) + (trace ? 1 : 0)) {
        case MC_EXACT * 4 + 0: MC_FWD(MC_EXACT, false, false); break;
        case MC_EXACT * 4 + 1: MC_FWD(MC_EXACT, false, true); break;
        case MC_EXACT * 4 + 2: MC_FWD(MC_EXACT, true, false); break;
        case MC_EXACT * 4 + 3: MC_FWD(MC_EXACT, true, true); break;
        case MC_STRANG * 4 + 0: MC_FWD(MC_STRANG, false, false); break;
        case MC_STRANG * 4 + 1: MC_FWD(MC_STRANG, false, true); break;
        case MC_STRANG * 4 + 2: MC_FWD(MC_STRANG, true, false); break;
        case MC_STRANG * 4 + 3: MC_FWD(MC_STRANG, true, true); break;
        case MC_LIE * 4 + 0: MC_FWD(MC_LIE, false, false); break;
        case MC_LIE * 4 + 1: MC_FWD(MC_LIE, false, true); break;
        case MC_LIE * 4 + 2: MC_FWD(MC_LIE, true, false); break;
        case MC_LIE * 4 + 3: MC_FWD(MC_LIE, true, true); break;
        default: return hipErrorInvalidValue;
    }
#undef MC_FWD
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.n > 0 && a.acc1) {
        hipLaunchKernelGGL(k_fwd_finish, dim3(gz), dim3(256), 0, s, a.n, a.nwalk, a.acc1, a.acc2);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (sum_out) {
        hipLaunchKernelGGL(k_fwd_total, dim3(1), dim3(1024), 0, s, a.chunks, a.part, sum_out);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace mc
