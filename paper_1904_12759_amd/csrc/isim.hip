// Intersection similarity of two rankings (the isim measure the paper uses in
// Sec. 6 to compare the node rankings of two computed communicability
// vectors): isim_K(x, y) = (1/K) sum_{i=1..K} |X_i delta Y_i| / (2i), X_i the i
// nodes with the largest x.
//
// With rank_x(j), rank_y(j) the 0-based positions of node j in the two
// descending orders and m_j = max(rank_x(j), rank_y(j)), node j lies in
// X_i and Y_i exactly when m_j < i, so |X_i cap Y_i| = #{j : m_j < i} and
// |X_i delta Y_i| = 2i - 2 |X_i cap Y_i|: one histogram of m over [0, K) and its
// prefix sums give every term.  Orders are stable radix sorts (sort.hip) of keys
// that order the values descending (node index as payload), so ties keep the lower
// index first; -0 is read as +0.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "alloc.hpp"
#include "mc_internal.hpp"

namespace mc {

namespace {

constexpr int kSumThreads = 1024;

// 64-bit key whose ascending order is the descending order of the double a
// (finite; -0 already mapped to +0): flip the ordering of the IEEE bits.
__device__ __forceinline__ unsigned long long desc_key(double a) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(a);
    const unsigned long long asc = (b >> 63) ? ~b : (b | 0x8000000000000000ull);
    return ~asc;
}

// keys: x then y (+0.0 maps -0 to +0); payload: node index; flag: non-finite input
__global__ void k_isim_init(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
                            unsigned long long *__restrict__ keys, uint32_t *__restrict__ vals,
                            uint32_t *__restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double a = x[i], b = y[i];
    if (!isfinite(a) || !isfinite(b)) atomicOr(flag, 1u);
    keys[i] = desc_key(a + 0.0);
    keys[n + i] = desc_key(b + 0.0);
    vals[i] = (uint32_t)i;
    vals[n + i] = (uint32_t)i;
}

// rank of every node in both orders
__global__ void k_isim_rank(int64_t n, const uint32_t *__restrict__ order, int32_t *__restrict__ rank) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    rank[order[r]] = (int32_t)r;
    rank[n + order[n + r]] = (int32_t)r;
}

// histogram of m_j = max(rank_x(j), rank_y(j)) over [0, K)
__global__ void k_isim_hist(int64_t n, int64_t K, const int32_t *__restrict__ rank,
                            int32_t *__restrict__ cnt) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int32_t m = max(rank[j], rank[n + j]);
    if (m < K) atomicAdd(cnt + m, 1);
}

// Inclusive prefix sums of the histogram (integers, exact): thread j sums a
// contiguous run, one lane scans the run totals, every run is rewritten.
__global__ __launch_bounds__(1024) void k_isim_cum(int64_t K, const int32_t *__restrict__ cnt,
                                                   int32_t *__restrict__ cum) {
    __shared__ int32_t run[1024];
    const int j = threadIdx.x;
    const int64_t per = (K + 1023) / 1024;
    const int64_t lo = (int64_t)j * per;
    const int64_t hi = lo + per < K ? lo + per : K;
    int32_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += cnt[i];
    run[j] = s;
    __syncthreads();
    if (j == 0) {
        int32_t e = 0;
        for (int u = 0; u < 1024; ++u) {
            const int32_t v = run[u];
            run[u] = e;
            e += v;
        }
    }
    __syncthreads();
    int32_t e = run[j];
    for (int64_t i = lo; i < hi; ++i) {
        e += cnt[i];
        cum[i] = e;
    }
}

// (1/K) sum_{i=1..K} (1 - c_i / i), c_i = cum[i-1] = |X_i cap Y_i|: every thread sums
// its strided terms in order, then a fixed tree, so the result is reproducible
__global__ __launch_bounds__(kSumThreads) void k_isim_sum(int64_t K, const int32_t *__restrict__ cum,
                                                          double *__restrict__ out) {
    __shared__ double part[kSumThreads];
    double s = 0.0;
    for (int64_t i = (int64_t)threadIdx.x + 1; i <= K; i += kSumThreads)
        s += 1.0 - (double)cum[i - 1] / (double)i;
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = kSumThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = part[0] / (double)K;
}

mc_status status_of(hipError_t e) {
    if (e == hipSuccess) return MC_OK;
    if (e == hipErrorOutOfMemory) return MC_ERR_NO_MEMORY;
    (void)hipGetLastError();
    return MC_ERR_DEVICE;
}

}  // namespace

}  // namespace mc

extern "C" mc_status mc_isim(int64_t n, const double *x, const double *y, int64_t k, double *out,
                             void *stream) {
    using namespace mc;
    fault_scope_begin();
    if (!x || !y || !out || n < 1 || n > 0x7FFFFFFFll || k < 1 || k > n) return MC_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    unsigned long long *keys = nullptr, *keys_sorted = nullptr;
    double *res = nullptr;
    uint32_t *vals = nullptr, *order = nullptr;
    int32_t *rank = nullptr, *cnt = nullptr, *cum = nullptr;
    uint32_t *flag = nullptr;
    void *temp = nullptr;
    size_t temp_bytes = 0;
    hipError_t e = sort_pairs_u64(nullptr, temp_bytes, nullptr, nullptr, nullptr, nullptr, n, s);
    if (e == hipSuccess) e = dev_malloc((void **)&keys, sizeof(unsigned long long) * 2 * (size_t)n);
    if (e == hipSuccess) e = dev_malloc((void **)&keys_sorted, sizeof(unsigned long long) * 2 * (size_t)n);
    if (e == hipSuccess) e = dev_malloc((void **)&vals, sizeof(uint32_t) * 2 * (size_t)n);
    if (e == hipSuccess) e = dev_malloc((void **)&order, sizeof(uint32_t) * 2 * (size_t)n);
    if (e == hipSuccess) e = dev_malloc((void **)&rank, sizeof(int32_t) * 2 * (size_t)n);
    if (e == hipSuccess) e = dev_malloc((void **)&cnt, sizeof(int32_t) * (size_t)k);
    if (e == hipSuccess) e = dev_malloc((void **)&cum, sizeof(int32_t) * (size_t)k);
    if (e == hipSuccess) e = dev_malloc((void **)&res, sizeof(double));
    if (e == hipSuccess) e = dev_malloc((void **)&flag, sizeof(uint32_t));
    if (e == hipSuccess) e = dev_malloc(&temp, temp_bytes);
    const unsigned g = (unsigned)((n + 255) / 256);
    if (e == hipSuccess) e = hipMemsetAsync(flag, 0, sizeof(uint32_t), s);
    if (e == hipSuccess) e = hipMemsetAsync(cnt, 0, sizeof(int32_t) * (size_t)k, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_isim_init, dim3(g), dim3(256), 0, s, n, x, y, keys, vals, flag);
        e = hipGetLastError();
    }
    size_t tb = temp_bytes;
    if (e == hipSuccess) e = sort_pairs_u64(temp, tb, keys, keys_sorted, vals, order, n, s);
    tb = temp_bytes;
    if (e == hipSuccess)
        e = sort_pairs_u64(temp, tb, keys + n, keys_sorted + n, vals + n, order + n, n, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_isim_rank, dim3(g), dim3(256), 0, s, n, order, rank);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_isim_hist, dim3(g), dim3(256), 0, s, n, k, rank, cnt);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_isim_cum, dim3(1), dim3(1024), 0, s, k, cnt, cum);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_isim_sum, dim3(1), dim3(kSumThreads), 0, s, k, cum, res);
        e = hipGetLastError();
    }
    uint32_t f = 0;
    double r = 0.0;
    if (e == hipSuccess) e = hipMemcpyAsync(&f, flag, sizeof(f), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&r, res, sizeof(r), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    mc_status st = status_of(e);
    (void)hipStreamSynchronize(s);
    (void)hipFree(keys);
    (void)hipFree(keys_sorted);
    (void)hipFree(vals);
    (void)hipFree(order);
    (void)hipFree(rank);
    (void)hipFree(cnt);
    (void)hipFree(cum);
    (void)hipFree(res);
    (void)hipFree(flag);
    (void)hipFree(temp);
    if (st != MC_OK) return st;
    if (f) return MC_ERR_NONFINITE;
    *out = r;
    return MC_OK;
}
