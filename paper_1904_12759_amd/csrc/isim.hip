// Intersection similarity of two rankings (the isim measure the paper uses in
// Sec. 6 to compare the node rankings of two computed communicability
// vectors): isim_K(x, y) = (1/K) sum_{i=1..K} |X_i delta Y_i| / (2i), X_i the i
// nodes with the largest x.
//
// With rank_x(j), rank_y(j) the 0-based positions of node j in the two
// descending orders and m_j = max(rank_x(j), rank_y(j)), node j lies in
// X_i and Y_i exactly when m_j < i, so |X_i cap Y_i| = #{j : m_j < i} and
// |X_i delta Y_i| = 2i - 2 |X_i cap Y_i|: one histogram of m over [0, K) and its
// prefix sums give every term.  Orders are stable radix sorts of the values
// (node index as payload), so ties keep the lower index first; -0 is read as +0.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <hipcub/hipcub.hpp>

#include "alloc.hpp"
#include "mc_internal.hpp"

namespace mc {

namespace {

constexpr int kSumThreads = 1024;

// keys: x then y (+0.0 maps -0 to +0); payload: node index; flag: non-finite input
__global__ void k_isim_init(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
                            double *__restrict__ keys, int32_t *__restrict__ vals,
                            uint32_t *__restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double a = x[i], b = y[i];
    if (!isfinite(a) || !isfinite(b)) atomicOr(flag, 1u);
    keys[i] = a + 0.0;
    keys[n + i] = b + 0.0;
    vals[i] = (int32_t)i;
    vals[n + i] = (int32_t)i;
}

// rank of every node in both orders
__global__ void k_isim_rank(int64_t n, const int32_t *__restrict__ order, int32_t *__restrict__ rank) {
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
    double *keys = nullptr, *keys_sorted = nullptr, *res = nullptr;
    int32_t *vals = nullptr, *order = nullptr, *rank = nullptr, *cnt = nullptr, *cum = nullptr;
    uint32_t *flag = nullptr;
    void *temp = nullptr;
    size_t sort_bytes = 0, scan_bytes = 0;
    const int nn = (int)n, kk = (int)k;
    hipError_t e = hipcub::DeviceRadixSort::SortPairsDescending(nullptr, sort_bytes, keys, keys_sorted,
                                                                vals, order, nn, 0, 64, s);
    if (e == hipSuccess) e = hipcub::DeviceScan::InclusiveSum(nullptr, scan_bytes, cnt, cum, kk, s);
    if (e == hipSuccess) e = dev_malloc((void **)&keys, sizeof(double) * 2 * (size_t)n);
    if (e == hipSuccess) e = dev_malloc((void **)&keys_sorted, sizeof(double) * 2 * (size_t)n);
    if (e == hipSuccess) e = dev_malloc((void **)&vals, sizeof(int32_t) * 2 * (size_t)n);
    if (e == hipSuccess) e = dev_malloc((void **)&order, sizeof(int32_t) * 2 * (size_t)n);
    if (e == hipSuccess) e = dev_malloc((void **)&rank, sizeof(int32_t) * 2 * (size_t)n);
    if (e == hipSuccess) e = dev_malloc((void **)&cnt, sizeof(int32_t) * (size_t)k);
    if (e == hipSuccess) e = dev_malloc((void **)&cum, sizeof(int32_t) * (size_t)k);
    if (e == hipSuccess) e = dev_malloc((void **)&res, sizeof(double));
    if (e == hipSuccess) e = dev_malloc((void **)&flag, sizeof(uint32_t));
    const size_t temp_bytes = sort_bytes > scan_bytes ? sort_bytes : scan_bytes;
    if (e == hipSuccess) e = dev_malloc(&temp, temp_bytes ? temp_bytes : 1);
    const unsigned g = (unsigned)((n + 255) / 256);
    if (e == hipSuccess) e = hipMemsetAsync(flag, 0, sizeof(uint32_t), s);
    if (e == hipSuccess) e = hipMemsetAsync(cnt, 0, sizeof(int32_t) * (size_t)k, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_isim_init, dim3(g), dim3(256), 0, s, n, x, y, keys, vals, flag);
        e = hipGetLastError();
    }
    size_t tb = temp_bytes;
    if (e == hipSuccess)
        e = hipcub::DeviceRadixSort::SortPairsDescending(temp, tb, keys, keys_sorted, vals, order, nn,
                                                         0, 64, s);
    tb = temp_bytes;
    if (e == hipSuccess)
        e = hipcub::DeviceRadixSort::SortPairsDescending(temp, tb, keys + n, keys_sorted + n, vals + n,
                                                         order + n, nn, 0, 64, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_isim_rank, dim3(g), dim3(256), 0, s, n, order, rank);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_isim_hist, dim3(g), dim3(256), 0, s, n, k, rank, cnt);
        e = hipGetLastError();
    }
    tb = temp_bytes;
    if (e == hipSuccess) e = hipcub::DeviceScan::InclusiveSum(temp, tb, cnt, cum, kk, s);
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
