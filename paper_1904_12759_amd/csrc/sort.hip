// Stable sort of (64-bit key, 32-bit value) pairs by ascending key: least-
// significant-digit radix sort, eight passes of 8-bit digits.  Used where the
// library needs an order (relabelling rows hot-first, the rankings of the isim
// measure); written here so that the library carries no sort of someone else's.
//
// A pass over tiles of kSortTile pairs (256 threads x 16 items, item k of thread t at
// tile position 256 k + t, so loads are coalesced and positions run in (k, t)
// order):
//   1. every tile counts its digits (LDS atomics; counts do not depend on order),
//      stored digit-major: cnt[d * tiles + b];
//   2. one block turns the counts into exclusive offsets (integer sums, exact);
//   3. every tile places its pairs: for each k, the 256 pairs at positions
//      256 k .. 256 k + 255 are ranked among equal digits by position (within a
//      wave by matching the 8 digit bits with ballots, across the four waves by
//      the waves' digit counts in wave order), after the equal digits of the
//      tile's earlier items; pair p goes to offset[d][tile] + that rank.
// Equal keys keep their input order (each pass is stable), so the sort is stable.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mc_internal.hpp"

namespace mc {

namespace {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int64_t kSortTile = (int64_t)kSortThreads * kSortItems;
constexpr int kDigits = 256;
constexpr int kSortWaves = kSortThreads / 64;

__device__ __forceinline__ uint32_t digit_of(unsigned long long key, int shift) {
    return (uint32_t)(key >> shift) & (kDigits - 1);
}

__global__ __launch_bounds__(kSortThreads) void k_sort_count(int64_t n, int64_t tiles,
                                                             const unsigned long long *__restrict__ keys,
                                                             int shift, uint32_t *__restrict__ cnt) {
    __shared__ uint32_t h[kDigits];
    const int t = threadIdx.x;
    h[t] = 0u;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t i = base + (int64_t)k * kSortThreads + t;
        if (i < n) atomicAdd(&h[digit_of(keys[i], shift)], 1u);
    }
    __syncthreads();
    cnt[(int64_t)t * tiles + blockIdx.x] = h[t];
}

// Exclusive prefix sums of cnt[0 .. len) in place: thread j sums a contiguous run,
// the run totals are scanned by one lane, then every run is rewritten.
__global__ __launch_bounds__(1024) void k_sort_offsets(int64_t len, uint32_t *__restrict__ cnt) {
    __shared__ uint32_t run[1024];
    const int j = threadIdx.x;
    const int64_t per = (len + 1023) / 1024;
    const int64_t lo = (int64_t)j * per;
    const int64_t hi = lo + per < len ? lo + per : len;
    uint32_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += cnt[i];
    run[j] = s;
    __syncthreads();
    if (j == 0) {
        uint32_t e = 0;
        for (int u = 0; u < 1024; ++u) {
            const uint32_t v = run[u];
            run[u] = e;
            e += v;
        }
    }
    __syncthreads();
    uint32_t e = run[j];
    for (int64_t i = lo; i < hi; ++i) {
        const uint32_t v = cnt[i];
        cnt[i] = e;
        e += v;
    }
}

__global__ __launch_bounds__(kSortThreads) void k_sort_place(
    int64_t n, int64_t tiles, const unsigned long long *__restrict__ kin,
    const uint32_t *__restrict__ vin, unsigned long long *__restrict__ kout,
    uint32_t *__restrict__ vout, int shift, const uint32_t *__restrict__ off) {
    __shared__ uint32_t base_d[kDigits];                 // next free slot of each digit
    __shared__ uint32_t wcnt[kSortWaves][kDigits];       // this round's digit counts per wave
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int w = t >> 6;
    const unsigned long long lt = (1ull << lane) - 1ull;
    base_d[t] = off[(int64_t)t * tiles + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int k = 0; k < kSortItems; ++k) {
        for (int u = t; u < kSortWaves * kDigits; u += kSortThreads) (&wcnt[0][0])[u] = 0u;
        __syncthreads();
        const int64_t i = base + (int64_t)k * kSortThreads + t;
        const bool valid = i < n;
        unsigned long long key = 0;
        uint32_t val = 0, d = 0;
        if (valid) {
            key = kin[i];
            val = vin[i];
            d = digit_of(key, shift);
        }
        // lanes of this wave with the same digit
        unsigned long long same = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const unsigned long long set = __ballot(valid && ((d >> b) & 1u));
            same &= ((d >> b) & 1u) ? set : ~set;
        }
        const uint32_t in_wave = (uint32_t)__popcll(same & lt);
        if (valid && in_wave == 0) wcnt[w][d] = (uint32_t)__popcll(same);
        __syncthreads();
        if (valid) {
            uint32_t before = 0;
            for (int x = 0; x < w; ++x) before += wcnt[x][d];
            const uint32_t dst = base_d[d] + before + in_wave;
            kout[dst] = key;
            vout[dst] = val;
        }
        __syncthreads();
        base_d[t] += wcnt[0][t] + wcnt[1][t] + wcnt[2][t] + wcnt[3][t];
        __syncthreads();
    }
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

// Sorts n pairs (kin, vin) into (kout, vout) on stream s.  With temp == null only
// the scratch size (alternate key and value buffers and the digit counts) is written
// to temp_bytes; otherwise temp must hold that many bytes.  kin / vin are not changed.
hipError_t sort_pairs_u64(void *temp, size_t &temp_bytes, const unsigned long long *kin,
                          unsigned long long *kout, const uint32_t *vin, uint32_t *vout, int64_t n,
                          hipStream_t s) {
    static_assert(kSortWaves == 4, "place kernel sums four wave counts");
    if (n < 0 || n > 0x7FFFFFFFll) return hipErrorInvalidValue;
    const int64_t tiles = (n + kSortTile - 1) / kSortTile;
    const size_t kbytes = align_up(sizeof(unsigned long long) * (size_t)n);
    const size_t vbytes = align_up(sizeof(uint32_t) * (size_t)n);
    const size_t cbytes = align_up(sizeof(uint32_t) * (size_t)kDigits * (size_t)tiles);
    const size_t need = kbytes + vbytes + cbytes;
    if (!temp) {
        temp_bytes = need > 0 ? need : 1;
        return hipSuccess;
    }
    if (temp_bytes < need) return hipErrorInvalidValue;
    if (n == 0) return hipSuccess;
    char *p = static_cast<char *>(temp);
    unsigned long long *ktmp = reinterpret_cast<unsigned long long *>(p);
    uint32_t *vtmp = reinterpret_cast<uint32_t *>(p + kbytes);
    uint32_t *cnt = reinterpret_cast<uint32_t *>(p + kbytes + vbytes);
    // passes 0..7 write tmp, out, tmp, ..., out: the last one lands in kout / vout
    const unsigned long long *ks = kin;
    const uint32_t *vs = vin;
    for (int pass = 0; pass < 8; ++pass) {
        unsigned long long *kd = (pass & 1) ? kout : ktmp;
        uint32_t *vd = (pass & 1) ? vout : vtmp;
        const int shift = 8 * pass;
        hipLaunchKernelGGL(k_sort_count, dim3((unsigned)tiles), dim3(kSortThreads), 0, s, n, tiles, ks,
                           shift, cnt);
        hipLaunchKernelGGL(k_sort_offsets, dim3(1), dim3(1024), 0, s, (int64_t)kDigits * tiles, cnt);
        hipLaunchKernelGGL(k_sort_place, dim3((unsigned)tiles), dim3(kSortThreads), 0, s, n, tiles, ks,
                           vs, kd, vd, shift, cnt);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        ks = kd;
        vs = vd;
    }
    return hipSuccess;
}

}  // namespace mc
