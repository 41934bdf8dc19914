// Table construction on the device: validation of the CSR matrix, the split of
// every row into diagonal, exit rate and jump law (paper Sec. 2 and Eq.
// (paths)), and one Vose alias table per row so that a jump costs one draw and
// one gather instead of the row scan discussed in Sec. 4.
#include <math.h>


#include "mc_internal.hpp"

namespace mc {
namespace {

// rowptr must be a valid row-offset array before any row is read.
__global__ void k_check_rowptr(int64_t n, int64_t nnz, const int64_t *__restrict__ rowptr,
                               uint32_t *flags) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    const int64_t p = rowptr[i];
    bool bad = p < 0 || p > nnz;
    if (i == 0) bad |= p != 0;
    if (i == n) bad |= p != nnz;
    if (i < n) bad |= rowptr[i + 1] < p;
    if (bad) atomicOr(flags, F_INVALID_ARG);
}

// One thread per row.  Slots of row i occupy CSR positions rowptr[i] ..
// rowptr[i]+deg-1 (the positive off-diagonal entries, in CSR order).
//   plain   (bias == null): a_s = a_ij,          r = sum a_s,  d = a_ii + r
//   tilted  (bias != null): a_s = a_ij exp(b_ij), r~ = sum a_s, d~ = d + (r~ - r)
// The alias table follows Vose (IEEE TSE 1991): scaled probabilities
// q_s = a_s * deg / r, two LIFO work lists filled by scanning the slots in
// order, and for each "small" slot the threshold floor(q * 2^32) of keeping
// its own column; slots left over keep their own column with certainty.
__global__ void k_setup_rows(int64_t n, const int64_t *__restrict__ rowptr,
                             const int32_t *__restrict__ col, const double *__restrict__ val,
                             const float *__restrict__ bias, const double *__restrict__ base_r,
                             const double *__restrict__ base_d, RowRec *__restrict__ rows,
                             double *__restrict__ d64, float *__restrict__ d32,
                             double *__restrict__ rr, SlotRec *__restrict__ slots,
                             float2 *__restrict__ corr, double *__restrict__ q,
                             int32_t *__restrict__ small, int32_t *__restrict__ large,
                             uint32_t *flags) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t p0 = rowptr[i], p1 = rowptr[i + 1];
    double diag = 0.0, rate = 0.0;
    int64_t deg = 0;
    uint32_t err = 0;
    for (int64_t p = p0; p < p1; ++p) {
        const int32_t j = col[p];
        const double a = val[p];
        if (j < 0 || j >= n) {
            err |= F_INVALID_ARG;
            continue;
        }
        if (!isfinite(a)) {
            err |= F_NONFINITE;
            continue;
        }
        if (j == i) {
            diag = diag + a;
        } else if (a < 0.0) {
            err |= F_NOT_METZLER;
        } else if (a > 0.0) {
            double at = a;
            const int64_t s = p0 + deg;
            if (bias) {
                const float b = bias[p];
                at = a * exp((double)b);
                if (!isfinite(b) || !isfinite(at) || !(at > 0.0)) err |= F_NONFINITE;
                corr[s] = make_float2(-b, 0.0f);
            }
            q[s] = at;
            slots[s] = SlotRec{0xFFFFFFFFu, j, j, (uint32_t)deg};
            rate = rate + at;
            ++deg;
        }
    }
    double d = bias ? base_d[i] + (rate - base_r[i]) : diag + rate;
    double inv_r = 0.0;
    if (deg > 0) {
        inv_r = 1.0 / rate;
        if (!isfinite(inv_r)) err |= F_INVALID_ARG;
    }
    if (!isfinite(d)) err |= F_NONFINITE;
    if (err) {
        atomicOr(flags, err);
        return;
    }
    rows[i] = RowRec{inv_r, (uint32_t)deg, (uint32_t)p0};
    d64[i] = d;
    d32[i] = (float)d;
    rr[i] = rate;
    if (deg <= 1) {
        if (bias && deg == 1) corr[p0].y = corr[p0].x;
        return;
    }
    bool uniform = true;
    for (int64_t s = 1; s < deg && uniform; ++s) uniform = q[p0 + s] == q[p0];
    if (!uniform) {
        int64_t ns = 0, nl = 0;
        for (int64_t s = 0; s < deg; ++s) {
            const double qs = (q[p0 + s] * (double)deg) / rate;
            q[p0 + s] = qs;
            if (qs < 1.0)
                small[p0 + ns++] = (int32_t)s;
            else
                large[p0 + nl++] = (int32_t)s;
        }
        while (ns > 0 && nl > 0) {
            const int32_t l = small[p0 + --ns];
            const int32_t g = large[p0 + --nl];
            const double ql = q[p0 + l];
            SlotRec rec = slots[p0 + l];
            rec.thr = (uint32_t)(ql * 4294967296.0);
            rec.alias = slots[p0 + g].self;
            rec.aslot = (uint32_t)g;
            slots[p0 + l] = rec;
            const double qg = (q[p0 + g] + ql) - 1.0;
            q[p0 + g] = qg;
            if (qg < 1.0)
                small[p0 + ns++] = g;
            else
                large[p0 + nl++] = g;
        }
    }
    if (bias) {
        for (int64_t s = 0; s < deg; ++s) {
            const uint32_t a = slots[p0 + s].aslot;
            corr[p0 + s].y = corr[p0 + a].x;
        }
    }
}

// Relabelling: sort key ~bits(r_i) orders rows by descending exit rate (the
// bit pattern of a non-negative double is monotone in its value); the radix
// sort is stable, so equal rates keep index order.
__global__ void k_relabel_keys(int64_t n, const double *__restrict__ r,
                               unsigned long long *__restrict__ keys, uint32_t *__restrict__ vals) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    keys[i] = ~(unsigned long long)__double_as_longlong(r[i]);
    vals[i] = (uint32_t)i;
}

__global__ void k_relabel_perm(int64_t n, const uint32_t *__restrict__ inv, uint32_t *__restrict__ perm) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) perm[inv[k]] = (uint32_t)k;
}

// Walk-order copies of the row records and weight exponents.
__global__ void k_relabel_rows(int64_t n, const uint32_t *__restrict__ inv,
                               const RowRec *__restrict__ rows, const double *__restrict__ d64,
                               const float *__restrict__ d32, RowRec *__restrict__ wrows,
                               double *__restrict__ wd64, float *__restrict__ wd32) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const uint32_t i = inv[k];
    wrows[k] = rows[i];
    wd64[k] = d64[i];
    wd32[k] = d32[i];
}

// Rename the columns held in row i's slots (one thread per original row; only
// the deg slots in use are touched).
__global__ void k_relabel_slots(int64_t n, const int64_t *__restrict__ rowptr,
                                const RowRec *__restrict__ rows, const uint32_t *__restrict__ perm,
                                SlotRec *__restrict__ slots) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t p0 = rowptr[i];
    const uint32_t deg = rows[i].deg;
    for (uint32_t s = 0; s < deg; ++s) {
        SlotRec q = slots[p0 + s];
        q.self = (int32_t)perm[q.self];
        q.alias = (int32_t)perm[q.alias];
        slots[p0 + s] = q;
    }
}

// 64-byte slots from the final tables (rows, d and slots in walk order): slot
// position j gets slot j and the rows and d of its two destinations.  Positions
// that hold no slot (the diagonal, zero entries) may hold any bits; they get
// empty rows unless both destinations are in range, and no walk reads them.
__global__ void k_fat_slots(int64_t nnz, int64_t n, const SlotRec *__restrict__ slots,
                            const RowRec *__restrict__ rows, const double *__restrict__ d64,
                            const float *__restrict__ d32, int fp32, FatSlot *__restrict__ fat) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nnz) return;
    FatSlot f{};
    f.s = slots[j];
    const uint32_t a = (uint32_t)f.s.self, b = (uint32_t)f.s.alias;
    if (a < (uint64_t)n && b < (uint64_t)n) {
        f.rs = rows[a];
        f.ra = rows[b];
        f.ds = fp32 ? (double)d32[a] : d64[a];
        f.da = fp32 ? (double)d32[b] : d64[b];
    }
    fat[j] = f;
}

}  // namespace

hipError_t launch_fat_slots(int64_t n, int64_t nnz, const Tables &tb, bool walk_order, bool fp32,
                            hipStream_t s) {
    if (nnz == 0) return hipSuccess;
    const int64_t grid = (nnz + 255) / 256;
    if (grid > 0x7FFFFFFF) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fat_slots, dim3((unsigned)grid), dim3(256), 0, s, nnz, n, tb.slots,
                       walk_order ? tb.wrows : tb.rows, walk_order ? tb.wd64 : tb.d64,
                       walk_order ? tb.wd32 : tb.d32, fp32 ? 1 : 0, tb.fat);
    return hipGetLastError();
}

hipError_t launch_relabel_keys(int64_t n, const double *r, unsigned long long *keys, uint32_t *vals,
                               hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_relabel_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, r, keys,
                       vals);
    return hipGetLastError();
}

hipError_t launch_relabel_apply(int64_t n, const int64_t *rowptr, const uint32_t *inv,
                                uint32_t *perm, Tables &tb, bool build_perm, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const unsigned g = (unsigned)((n + 255) / 256);
    if (build_perm) hipLaunchKernelGGL(k_relabel_perm, dim3(g), dim3(256), 0, s, n, inv, perm);
    hipLaunchKernelGGL(k_relabel_rows, dim3(g), dim3(256), 0, s, n, inv, tb.rows, tb.d64, tb.d32,
                       tb.wrows, tb.wd64, tb.wd32);
    hipLaunchKernelGGL(k_relabel_slots, dim3(g), dim3(256), 0, s, n, rowptr, tb.rows, perm, tb.slots);
    return hipGetLastError();
}

// Largest o in [0, 2^32) with (o 2^-32) r < c, for c > 0 (o = 0 always
// qualifies): the product rounds monotonically in o, so the o that keep u r below
// c form a prefix and bisection finds its end.  Both multiplications are the ones
// the inverse-CDF rule makes (the first is exact).
__device__ uint32_t cdf_threshold(double c, double r) {
    uint64_t lo = 0, hi = 1ull << 32;    // (lo 2^-32) r < c; hi == 2^32 or fails
    while (hi - lo > 1) {
        const uint64_t mid = (lo + hi) >> 1;
        if (((double)mid * 0x1p-32) * r < c) lo = mid;
        else hi = mid;
    }
    return (uint32_t)lo;
}

// One thread per node of the 7-point stencil: its three face rates checked
// (finite, >= 0, and 0 on the last plane of their axis, where no neighbour
// exists) and a_xx finite; two slots counted per positive face (an exit in each
// direction); and its state record: r summed over the six faces in column order
// (-z, -y, -x, +x, +y, +z) as the row split sums the same matrix in CSR form, 1/r
// when the node has an exit, the faces with a rate, the jump thresholds of the
// inverse-CDF rule over the running sums (all but the last such face), and
// d = a_xx + r.  The faces toward lower indices are the neighbours' own, which
// their threads check.
__global__ void k_stencil_rows(int64_t n, int64_t nx, int64_t ny, const double *__restrict__ fx,
                               const double *__restrict__ fy, const double *__restrict__ fz,
                               const double *__restrict__ diag, RowRec *__restrict__ rows,
                               uint4 *__restrict__ stail, double *__restrict__ d64,
                               float *__restrict__ d32, uint32_t *flags,
                               unsigned long long *nslots) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t nxy = nx * ny;
    const int64_t x = i % nx, y = (i / nx) % ny, z = i / nxy;
    const int64_t nz = n / nxy;
    const double up[3] = {fx[i], fy[i], fz[i]};
    const bool last[3] = {x == nx - 1, y == ny - 1, z == nz - 1};
    uint32_t bad = 0;
    unsigned long long cnt = 0;
    for (int a = 0; a < 3; ++a) {
        if (!isfinite(up[a])) bad |= F_NONFINITE;
        else if (up[a] < 0.0) bad |= F_NOT_METZLER;
        else if (up[a] > 0.0 && last[a]) bad |= F_INVALID_ARG;
        if (up[a] > 0.0) cnt += 2;
    }
    const double f[6] = {i >= nxy ? fz[i - nxy] : 0.0, i >= nx ? fy[i - nx] : 0.0,
                         i >= 1 ? fx[i - 1] : 0.0, up[0], up[1], up[2]};
    double r = 0.0;
    uint32_t deg = 0;
    for (int k = 0; k < 6; ++k) {
        r = r + f[k];
        deg += f[k] > 0.0 ? 1u : 0u;
    }
    double inv_r = 0.0;
    uint32_t meta = deg;
    uint32_t e[5] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu};
    if (deg > 0 && !bad) {
        inv_r = 1.0 / r;
        if (!isfinite(inv_r)) bad |= F_INVALID_ARG;
        double cum = 0.0;
        uint32_t j = 0;
        for (int k = 0; k < 6; ++k) {
            cum = cum + f[k];
            if (f[k] > 0.0) {
                meta |= (uint32_t)k << (3 + 3 * j);
                if (j + 1 < deg) e[j] = cdf_threshold(cum, r);
                ++j;
            }
        }
    }
    const double d = diag[i] + r;
    if (!isfinite(d)) bad |= F_NONFINITE;
    if (bad) atomicOr(flags, bad);
    if (cnt) atomicAdd(nslots, cnt);
    rows[i] = RowRec{inv_r, meta, e[0]};
    stail[i] = make_uint4(e[1], e[2], e[3], e[4]);
    d64[i] = d;
    d32[i] = (float)d;
}

hipError_t launch_stencil_rows(int64_t n, int64_t nx, int64_t ny, const double *fx, const double *fy,
                               const double *fz, const double *diag, RowRec *rows, uint4 *stail,
                               double *d64, float *d32, uint32_t *flags, unsigned long long *nslots,
                               hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int64_t grid = (n + 255) / 256;
    hipLaunchKernelGGL(k_stencil_rows, dim3((unsigned)grid), dim3(256), 0, s, n, nx, ny, fx, fy, fz,
                       diag, rows, stail, d64, d32, flags, nslots);
    return hipGetLastError();
}

hipError_t launch_check_rowptr(int64_t n, int64_t nnz, const int64_t *rowptr, uint32_t *flags,
                               hipStream_t s) {
    const int64_t threads = n + 1;
    const int block = 256;
    const int64_t grid = (threads + block - 1) / block;
    hipLaunchKernelGGL(k_check_rowptr, dim3((unsigned)grid), dim3(block), 0, s, n, nnz, rowptr,
                       flags);
    return hipGetLastError();
}

hipError_t launch_setup_rows(int64_t n, const int64_t *rowptr, const int32_t *col,
                             const double *val, const float *bias, const Tables &base,
                             Tables &out, double *q_scratch, int32_t *stack_small,
                             int32_t *stack_large, uint32_t *flags, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int block = 128;
    const int64_t grid = (n + block - 1) / block;
    hipLaunchKernelGGL(k_setup_rows, dim3((unsigned)grid), dim3(block), 0, s, n, rowptr, col,
                       val, bias, base.r, base.d64, out.rows, out.d64, out.d32, out.r,
                       out.slots, out.corr, q_scratch, stack_small, stack_large, flags);
    return hipGetLastError();
}

}  // namespace mc
