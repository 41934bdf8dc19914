// The learned proposal's network: node features, the 8 -> 64 -> 64 -> 1 MLP
// that maps an edge's two node-feature vectors to a tilt b_ij of its jump
// rate, its training step (forward, backward, deterministic gradient
// reduction, Adam) and its inference over every edge.
//
// Variance reduction is the remedy the paper names for the statistical error
// (Sec. 5); tilting jump rates with an importance-weight correction is this
// library's way of doing it.  The network is small (4801 parameters) but its
// 64 x 64 layer is a dense contraction over many edges, so that layer runs on
// the matrix cores with bfloat16 operands and FP32 accumulation: the forward
// product and the backward dL/da1 = W2^T dL/dz2 on gfx950's
// v_mfma_f32_16x16x32_bf16 (two per 16 x 16 output tile), the weight gradient
// dW2 = dz2 a1^T, a contraction over a tile's 16 edges, on
// v_mfma_f32_16x16x16_bf16.
//
// Register layout.  A wave handles tiles of 16 edges.  Lane l works on edge
// e = l % 16 and owns the hidden features 16*k + 4*(l/16) + i (k, i < 4): the
// rows of the MFMA result D[m][n] (lane n + 16*(m/4), element m%4) that fall to
// it.  A 16x16x32 operand gives lane m + 16*(kk/8) (A) or n + 16*(kk/8) (B) the
// eight elements kk%8 of its contraction index; a contraction does not depend on
// which feature stands at which kk as long as A and B agree, so element j of
// K-block kb is taken to be the lane's own feature of tile 2*kb + j/4 (index
// j%4).  Then layer 1's output is layer 2's B operand and layer 2's output (D)
// is the backward product's B operand without moving between lanes; only dW2
// goes through LDS.
#include "walk_task.hpp"
#include "mlp.hpp"

namespace mc {
namespace {

constexpr int H = 64;
constexpr int NIN = 8;
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + H * NIN;
constexpr int OFF_W2 = OFF_B1 + H;
constexpr int OFF_B2 = OFF_W2 + H * H;
constexpr int OFF_W3 = OFF_B2 + H;
constexpr int OFF_B3 = OFF_W3 + H;
static_assert(OFF_B3 + 1 == kMlpParams, "parameter layout");
constexpr int GSTRIDE = kMlpParams + 2;   // gradient partial row: params, sum p(b-t)^2, sum p
constexpr int WAVES = 4;                  // waves per block

typedef short v4s __attribute__((ext_vector_type(4)));
typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Hidden feature at element j of K-block kb of a lane in quarter q (see above).
__device__ __forceinline__ int kfeat(int kb, int q, int j) {
    return 16 * (2 * kb + (j >> 2)) + 4 * q + (j & 3);
}

__device__ __forceinline__ v4f mfma32(v8s a, v8s b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a),
                                                  __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
}

// float -> bfloat16, round to nearest even
__device__ __forceinline__ uint16_t f2bf(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ---------------------------------------------------------------- features
// The row of every CSR position, 16 lanes per row (a hub's row is long).
__global__ void k_rowof(int64_t n, const int64_t *__restrict__ rowptr, int32_t *__restrict__ rowof) {
    const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
    if (i >= n) return;
    for (int64_t p = rowptr[i] + (threadIdx.x & 15); p < rowptr[i + 1]; p += 16) rowof[p] = (int32_t)i;
}

// raw features [log1p deg, r, v, log1p(mean target degree)] in FP64
// One row of 16 lanes per node: lanes stride the row's entries, then the row's
// fixed DPP tree, so a hub's many neighbours are summed by 16 lanes instead of one
// thread (whose serial loop set the time of the whole launch on power-law graphs).
__global__ __launch_bounds__(256) void k_feat_raw(int64_t n, const int64_t *__restrict__ rowptr,
                                                  const int32_t *__restrict__ col,
                                                  const double *__restrict__ val,
                                                  const RowRec *__restrict__ rows,
                                                  const double *__restrict__ r, const void *v,
                                                  int v_fp32, double *__restrict__ raw) {
    const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
    const int rl = threadIdx.x & 15;
    const bool in = i < n;                   // whole rows share `in`; all lanes stay for the tree
    // neighbour degrees are integers: their sum is exact in any order
    uint64_t dsum = 0;
    if (in) {
        const int64_t p1 = rowptr[i + 1];
#pragma unroll 4
        for (int64_t p = rowptr[i] + rl; p < p1; p += 16) {
            const int32_t j = col[p];
            if (j != i && val[p] > 0.0) dsum += rows[j].deg;
        }
    }
    const double nsum = row_sum_f64((double)dsum);
    if (!in || rl != 0) return;
    const uint32_t deg = rows[i].deg;
    const double vi = v_fp32 ? (double)static_cast<const float *>(v)[i]
                             : static_cast<const double *>(v)[i];
    raw[4 * i + 0] = log1p((double)deg);
    raw[4 * i + 1] = r[i];
    raw[4 * i + 2] = vi;
    raw[4 * i + 3] = log1p(deg ? nsum / (double)deg : 0.0);
}

// Column means and population standard deviations, two passes, each over many
// blocks: thread t of block b adds rows b*256 + t, + grid*256, ... in order, the
// block's fixed tree gives its partial, and one block adds the partials in block
// order (deterministic; one block alone read the 32 MB of a 1e6-node graph twice at
// a single CU's bandwidth).
__global__ __launch_bounds__(256) void k_feat_colsum(int64_t n, const double *__restrict__ raw,
                                                     const double *__restrict__ stats,
                                                     double *__restrict__ part) {
    __shared__ double sh[256][4];
    const int tid = threadIdx.x;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * 256 + tid; i < n; i += (int64_t)gridDim.x * 256)
        for (int c = 0; c < 4; ++c) {
            const double x = raw[4 * i + c];
            if (stats) {
                const double d = x - stats[c];
                acc[c] += d * d;
            } else {
                acc[c] += x;
            }
        }
    for (int c = 0; c < 4; ++c) sh[tid][c] = acc[c];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w)
            for (int c = 0; c < 4; ++c) sh[tid][c] += sh[tid + w][c];
        __syncthreads();
    }
    if (tid < 4) part[4 * blockIdx.x + tid] = sh[0][tid];
}

// sd == false: stats[c] = mean; true: stats[4 + c] = population sd (1 if 0).  One
// block of kStatBlocks threads: thread b takes block b's partials, then a fixed tree.
__global__ __launch_bounds__(kStatBlocks) void k_feat_colfin(int64_t n, const double *__restrict__ part,
                                                            double *__restrict__ stats, int sd) {
    __shared__ double sh[kStatBlocks][4];
    const int b = threadIdx.x;
    for (int c = 0; c < 4; ++c) sh[b][c] = part[4 * b + c];
    __syncthreads();
    for (int w = kStatBlocks / 2; w > 0; w >>= 1) {
        if (b < w)
            for (int c = 0; c < 4; ++c) sh[b][c] += sh[b + w][c];
        __syncthreads();
    }
    if (b < 4) {
        const double s = sh[0][b];
        if (!sd) {
            stats[b] = s / (double)n;
        } else {
            const double v = sqrt(s / (double)n);
            stats[4 + b] = v > 0.0 ? v : 1.0;
        }
    }
}

__global__ void k_feat_norm(int64_t n, const double *__restrict__ raw,
                            const double *__restrict__ stats, float *__restrict__ feats) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 4 * n) return;
    const int c = (int)(k & 3);
    feats[k] = (float)((raw[k] - stats[c]) / stats[4 + c]);
}

// log h_i = 0.5 log(second moment of W v[X_t]) from a plain run's mean and
// standard error with nwalk walkers per node.
__global__ void k_log_h(int64_t n, const double *__restrict__ est, const double *__restrict__ se,
                        double nwalk, float *__restrict__ lh) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double var = se[i] * se[i] * nwalk;
    double m2 = var * (nwalk - 1.0) / nwalk + est[i] * est[i];
    if (!(m2 > 1e-300)) m2 = 1e-300;
    lh[i] = (float)(0.5 * log(m2));
}

// ------------------------------------------------------------------- network
struct NetArgs {
    const uint16_t *wbf;       // bfloat16 parameters [kMlpParams]
    const float *feats;        // [n * 4]
    const int32_t *rowof;      // [nnz] row of each CSR position
    const int32_t *col;        // [nnz]
    const double *val;         // [nnz]
    const double *r;           // [n] exit rates
    const float *lh;           // [n] log h (training only)
    int64_t p0, p1;            // only CSR positions in [p0, p1) are edges of this batch
    int64_t tile0, ntile;      // tiles visited: (tile0 + t * stride) mod tmod, t < ntile;
    int64_t stride, tmod;      // tile T covers CSR positions 16 T .. 16 T + 15
    float *out_b;              // [nnz] (inference) tilt per CSR position, 0 off the edges
    float *gpart;              // [waves][GSTRIDE] (training) per-wave gradient partials
};

// Forward (TRAIN = false: write b for every position; TRAIN = true: also
// back-propagate the weighted squared error and accumulate per-wave gradients).
template <bool TRAIN>
__global__ __launch_bounds__(256, TRAIN ? 1 : 2) void k_net(NetArgs a) {
    __shared__ float s_w1[H * NIN], s_b1[H], s_b2[H], s_w3[H], s_b3;
    __shared__ uint16_t s_a1[WAVES][H][16];    // a1 (bf16), [feature][edge]
    __shared__ uint16_t s_dz2[WAVES][H][16];   // dL/dz2 (bf16), [feature][edge]
    __shared__ float s_dz1[WAVES][H][16];      // dL/dz1, [feature][edge]
    __shared__ float s_x[WAVES][NIN][16];      // inputs, [feature][edge]
    __shared__ float s_g[TRAIN ? GSTRIDE : 1]; // the block's gradient partial

    for (int k = threadIdx.x; k < H * NIN; k += blockDim.x) s_w1[k] = bf2f(a.wbf[OFF_W1 + k]);
    for (int k = threadIdx.x; k < H; k += blockDim.x) {
        s_b1[k] = bf2f(a.wbf[OFF_B1 + k]);
        s_b2[k] = bf2f(a.wbf[OFF_B2 + k]);
        s_w3[k] = bf2f(a.wbf[OFF_W3 + k]);
    }
    if (threadIdx.x == 0) s_b3 = bf2f(a.wbf[OFF_B3]);
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int e = lane & 15;
    const int q = lane >> 4;
    // layer-2 weights as A operands: w2f[mt][kb][j] = W2[16 mt + e][kfeat(kb, q, j)]
    v8s w2f[4][2];
    for (int mt = 0; mt < 4; ++mt)
        for (int kb = 0; kb < 2; ++kb)
            for (int j = 0; j < 8; ++j)
                w2f[mt][kb][j] = (short)a.wbf[OFF_W2 + (16 * mt + e) * H + kfeat(kb, q, j)];
    // and transposed for the backward product: W2^T[16 mt + e][kfeat(kb, q, j)]
    v8s w2t[4][2];
    if constexpr (TRAIN) {
        for (int mt = 0; mt < 4; ++mt)
            for (int kb = 0; kb < 2; ++kb)
                for (int j = 0; j < 8; ++j)
                    w2t[mt][kb][j] = (short)a.wbf[OFF_W2 + kfeat(kb, q, j) * H + 16 * mt + e];
    }

    // layer-1 weights as 16x16x4 A operands: lane (e, q) holds W1[16 ks + e][q] and
    // W1[16 ks + e][4 + q]
    float w1a[4], w1b[4];
    for (int ks = 0; ks < 4; ++ks) {
        w1a[ks] = s_w1[(16 * ks + e) * NIN + q];
        w1b[ks] = s_w1[(16 * ks + e) * NIN + 4 + q];
    }

    v4f gw2[4][4];
    float gw3[16], gb2[16], gw1[NIN], gb1 = 0.0f, gb3 = 0.0f, lsum = 0.0f, psum = 0.0f;
    if constexpr (TRAIN) {
        for (int mt = 0; mt < 4; ++mt)
            for (int nk = 0; nk < 4; ++nk) gw2[mt][nk] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
        for (int k = 0; k < 16; ++k) gw3[k] = gb2[k] = 0.0f;
        for (int c = 0; c < NIN; ++c) gw1[c] = 0.0f;
    }

    const int64_t wave_id = (int64_t)blockIdx.x * WAVES + wv;
    const int64_t nwaves = (int64_t)gridDim.x * WAVES;
    for (int64_t t = wave_id; t < a.ntile; t += nwaves) {
        const int64_t tile = (a.tile0 + t * a.stride) % a.tmod;
        const int64_t pos = tile * 16 + e;
        const bool inside = pos >= a.p0 && pos < a.p1;
        bool valid = inside;
        int32_t src = 0, dst = 0;
        if (valid) {
            src = a.rowof[pos];
            dst = a.col[pos];
            valid = dst != src && a.val[pos] > 0.0;
        }
        // the edge's inputs: lane q holds x[q] (source feature q) and x[4 + q]
        // (destination feature q), the B operands of layer 1's two K-steps
        const float xs = valid ? a.feats[4 * (int64_t)src + q] : 0.0f;
        const float xd = valid ? a.feats[4 * (int64_t)dst + q] : 0.0f;
        // layer 1 (MFMA, FP32 16x16x4, the bias as accumulator): z1[16 ks + 4 q + i]
        uint32_t m1 = 0;
        v8s a1b[2];                  // a1b[kb][j]: feature kfeat(kb, q, j)
        for (int ks = 0; ks < 4; ++ks) {
            v4f z = {s_b1[16 * ks + 4 * q], s_b1[16 * ks + 4 * q + 1], s_b1[16 * ks + 4 * q + 2],
                     s_b1[16 * ks + 4 * q + 3]};
            z = __builtin_amdgcn_mfma_f32_16x16x4f32(w1a[ks], xs, z, 0, 0, 0);
            z = __builtin_amdgcn_mfma_f32_16x16x4f32(w1b[ks], xd, z, 0, 0, 0);
            for (int i = 0; i < 4; ++i) {
                const float av = z[i] > 0.0f ? z[i] : 0.0f;
                if (z[i] > 0.0f) m1 |= 1u << (4 * ks + i);
                const uint16_t hb = f2bf(av);
                a1b[ks >> 1][4 * (ks & 1) + i] = (short)hb;
            }
        }
        // layer 2 (MFMA): z2[16 mt + 4 q + i] for edge e
        float a2[16];
        uint32_t m2 = 0;
        for (int mt = 0; mt < 4; ++mt) {
            v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
            for (int kb = 0; kb < 2; ++kb) acc = mfma32(w2f[mt][kb], a1b[kb], acc);
            for (int i = 0; i < 4; ++i) {
                const int f = 16 * mt + 4 * q + i;
                const float z = acc[i] + s_b2[f];
                a2[4 * mt + i] = z > 0.0f ? z : 0.0f;
                if (z > 0.0f) m2 |= 1u << (4 * mt + i);
            }
        }
        // layer 3 and the bounded tilt
        float y = 0.0f;
        for (int mt = 0; mt < 4; ++mt)
            for (int i = 0; i < 4; ++i) y += s_w3[16 * mt + 4 * q + i] * a2[4 * mt + i];
        y += __shfl_xor(y, 16, 64);
        y += __shfl_xor(y, 32, 64);
        y += s_b3;
        const float th = tanhf(y * 0.125f);
        const float b = 8.0f * th;
        if constexpr (!TRAIN) {
            if (q == 0 && inside) a.out_b[pos] = valid ? b : 0.0f;
        } else {
            // d/dy of p (b - target)^2 (the division by sum p happens after reduction)
            float gy = 0.0f;
            if (valid) {
                const float tgt = a.lh[dst] - a.lh[src];
                const float pe = (float)(a.val[pos] / a.r[src]);
                const float diff = b - tgt;
                gy = 2.0f * pe * diff * (1.0f - th * th);
                if (q == 0) {
                    lsum += pe * diff * diff;
                    psum += pe;
                }
            }
            if (q == 0) gb3 += gy;
            v8s dz2b[2];             // dz2b[kb][j]: feature kfeat(kb, q, j)
            for (int mt = 0; mt < 4; ++mt)
                for (int i = 0; i < 4; ++i) {
                    const int k = 4 * mt + i;
                    const int f = 16 * mt + 4 * q + i;
                    gw3[k] += gy * a2[k];
                    const float dz = (m2 >> k) & 1u ? gy * s_w3[f] : 0.0f;
                    gb2[k] += dz;
                    const uint16_t db = f2bf(dz);
                    dz2b[mt >> 1][4 * (mt & 1) + i] = (short)db;
                    s_dz2[wv][f][e] = db;
                    s_a1[wv][f][e] = (uint16_t)a1b[mt >> 1][4 * (mt & 1) + i];
                }
            // dL/da1 = W2^T dL/dz2 (MFMA), masked by layer 1's ReLU
            for (int mt = 0; mt < 4; ++mt) {
                v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
                for (int kb = 0; kb < 2; ++kb) acc = mfma32(w2t[mt][kb], dz2b[kb], acc);
                for (int i = 0; i < 4; ++i) {
                    const int k = 4 * mt + i;
                    s_dz1[wv][16 * mt + 4 * q + i][e] = (m1 >> k) & 1u ? acc[i] : 0.0f;
                }
            }
            s_x[wv][q][e] = xs;
            s_x[wv][4 + q][e] = xd;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // dW2 += dz2 a1^T over the tile's 16 edges (MFMA, K = edges)
            v4s afr[4], bfr[4];
            for (int t = 0; t < 4; ++t)
                for (int i = 0; i < 4; ++i) {
                    afr[t][i] = (short)s_dz2[wv][16 * t + e][4 * q + i];
                    bfr[t][i] = (short)s_a1[wv][16 * t + e][4 * q + i];
                }
            for (int mt = 0; mt < 4; ++mt)
                for (int nk = 0; nk < 4; ++nk)
                    gw2[mt][nk] =
                        __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(afr[mt], bfr[nk], gw2[mt][nk], 0, 0, 0);
            // dW1 and db1 (VALU): lane l owns hidden unit l
            for (int ee = 0; ee < 16; ++ee) {
                const float d = s_dz1[wv][lane][ee];
                gb1 += d;
                for (int c = 0; c < NIN; ++c) gw1[c] += d * s_x[wv][c][ee];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }

    if constexpr (TRAIN) {
        // per-feature sums over the 16 edges of each quarter
        for (int k = 0; k < 16; ++k) {
            float s3 = gw3[k], s2 = gb2[k];
            for (int off = 1; off < 16; off <<= 1) {
                s3 += __shfl_xor(s3, off, 64);
                s2 += __shfl_xor(s2, off, 64);
            }
            gw3[k] = s3;
            gb2[k] = s2;
        }
        for (int off = 1; off < 64; off <<= 1) {
            gb3 += __shfl_xor(gb3, off, 64);
            lsum += __shfl_xor(lsum, off, 64);
            psum += __shfl_xor(psum, off, 64);
        }
        // the block's partial: the waves' partials added into LDS in wave order
        for (int step = 0; step < WAVES; ++step) {
            if (wv == step) {
                const bool first = step == 0;
                auto put = [&](int j, float x) { s_g[j] = first ? x : s_g[j] + x; };
                for (int c = 0; c < NIN; ++c) put(OFF_W1 + lane * NIN + c, gw1[c]);
                put(OFF_B1 + lane, gb1);
                for (int mt = 0; mt < 4; ++mt)
                    for (int nk = 0; nk < 4; ++nk)
                        for (int i = 0; i < 4; ++i)
                            put(OFF_W2 + (16 * mt + 4 * q + i) * H + 16 * nk + e, gw2[mt][nk][i]);
                if (e == 0)
                    for (int k = 0; k < 16; ++k) {
                        const int f = 16 * (k >> 2) + 4 * q + (k & 3);
                        put(OFF_W3 + f, gw3[k]);
                        put(OFF_B2 + f, gb2[k]);
                    }
                if (lane == 0) {
                    put(OFF_B3, gb3);
                    put(kMlpParams, lsum);
                    put(kMlpParams + 1, psum);
                }
            }
            __syncthreads();
        }
        float *g = a.gpart + (int64_t)blockIdx.x * GSTRIDE;
        for (int j = threadIdx.x; j < GSTRIDE; j += blockDim.x) g[j] = s_g[j];
    }
}

// Sum the per-block partials (FP64) in a fixed order: thread (column j, split s)
// of a block adds the partials of blocks s, s + RS, s + 2 RS, ... of its column,
// then the RS split sums of a column meet in a fixed tree in LDS.  16 columns
// (parameters, then sum p (b - t)^2 and sum p) per block.
constexpr int RS = 16;
__global__ __launch_bounds__(256) void k_grad_reduce(int64_t nparts, const float *__restrict__ gpart,
                                                     double *__restrict__ gsum) {
    __shared__ double sh[RS][16];
    const int pl = threadIdx.x & 15, sp = threadIdx.x >> 4;
    const int j = blockIdx.x * 16 + pl;
    double acc = 0.0;
    if (j < GSTRIDE)
        for (int64_t w = sp; w < nparts; w += RS) acc += (double)gpart[w * GSTRIDE + j];
    sh[sp][pl] = acc;
    __syncthreads();
    for (int h = RS / 2; h > 0; h >>= 1) {
        if (sp < h) sh[sp][pl] += sh[sp + h][pl];
        __syncthreads();
    }
    if (sp == 0 && j < GSTRIDE) gsum[j] = sh[0][pl];
}

// Gradient and loss: the sums divided by sum p, rounded to FP32.
__global__ void k_grad_scale(const double *__restrict__ gsum, float *__restrict__ grad,
                             float *__restrict__ loss) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= kMlpParams + 1) return;
    const double ps = gsum[kMlpParams + 1];
    const int col = j < kMlpParams ? j : kMlpParams;
    const double v = ps > 0.0 ? gsum[col] / ps : 0.0;
    if (j < kMlpParams) grad[j] = (float)v;
    else if (loss) *loss = (float)v;
}

// Adam (Kingma & Ba 2015) on the FP32 master weights, then the bf16 copy.
__global__ void k_adam(const float *__restrict__ grad, float *__restrict__ w, float *__restrict__ m,
                       float *__restrict__ v, uint16_t *__restrict__ wbf, float lr, float beta1,
                       float beta2, float eps, float bc1, float bc2) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= kMlpParams) return;
    const float g = grad[j];
    const float mj = beta1 * m[j] + (1.0f - beta1) * g;
    const float vj = beta2 * v[j] + (1.0f - beta2) * g * g;
    m[j] = mj;
    v[j] = vj;
    const float wj = w[j] - lr * (mj / bc1) / (sqrtf(vj / bc2) + eps);
    w[j] = wj;
    wbf[j] = f2bf(wj);
}

// He-uniform weights (bound sqrt(6 / fan_in)) from Philox, zero biases, and a
// small last layer so that training starts from an almost untilted walk.
__global__ void k_mlp_init(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                           uint16_t *__restrict__ wbf, uint32_t k0, uint32_t k1) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= kMlpParams) return;
    const U4 o = philox((uint32_t)j, 0u, 0u, 0x4d4c5031u, k0, k1);
    const float u = (float)(o.x >> 8) * 0x1p-24f;       // [0, 1)
    float bound = 0.0f;
    if (j < OFF_B1) bound = sqrtf(6.0f / NIN);
    else if (j >= OFF_W2 && j < OFF_B2) bound = sqrtf(6.0f / H);
    else if (j >= OFF_W3 && j < OFF_B3) bound = 0.01f;
    const float x = (2.0f * u - 1.0f) * bound;
    w[j] = x;
    m[j] = 0.0f;
    v[j] = 0.0f;
    wbf[j] = f2bf(x);
}

__global__ void k_params_bf16(const float *__restrict__ w, uint16_t *__restrict__ wbf) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < kMlpParams) wbf[j] = f2bf(w[j]);
}

}  // namespace

// ------------------------------------------------------------- launchers
int mlp_grad_stride() { return GSTRIDE; }

hipError_t launch_rowof(int64_t n, const int64_t *rowptr, int32_t *rowof, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int64_t g = (16 * n + 255) / 256;
    if (g > 0x7FFFFFFF) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_rowof, dim3((unsigned)g), dim3(256), 0, s, n, rowptr, rowof);
    return hipGetLastError();
}

hipError_t launch_features(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                           const RowRec *rows, const double *r, const void *v, int v_fp32,
                           double *raw, double *stats, float *feats, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int64_t g = (16 * n + 255) / 256;
    if (g > 0x7FFFFFFF) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_feat_raw, dim3((unsigned)g), dim3(256), 0, s, n, rowptr, col, val, rows, r, v,
                       v_fp32, raw);
    // partials after the 8 statistics words
    double *part = stats + 8;
    hipLaunchKernelGGL(k_feat_colsum, dim3(kStatBlocks), dim3(256), 0, s, n, raw,
                       (const double *)nullptr, part);
    hipLaunchKernelGGL(k_feat_colfin, dim3(1), dim3(kStatBlocks), 0, s, n, part, stats, 0);
    hipLaunchKernelGGL(k_feat_colsum, dim3(kStatBlocks), dim3(256), 0, s, n, raw, stats, part);
    hipLaunchKernelGGL(k_feat_colfin, dim3(1), dim3(kStatBlocks), 0, s, n, part, stats, 1);
    hipLaunchKernelGGL(k_feat_norm, dim3((unsigned)((4 * n + 255) / 256)), dim3(256), 0, s, n, raw,
                       stats, feats);
    return hipGetLastError();
}

hipError_t launch_log_h(int64_t n, const double *est, const double *se, double nwalk, float *lh,
                        hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_log_h, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, est, se, nwalk,
                       lh);
    return hipGetLastError();
}

// Blocks for ntile tiles: one wave per tile, at most max_blocks.
int mlp_blocks(int64_t ntile, int max_blocks) {
    int64_t b = (ntile + WAVES - 1) / WAVES;
    if (b > max_blocks) b = max_blocks;
    if (b < 1) b = 1;
    return (int)b;
}

hipError_t launch_net_forward(const uint16_t *wbf, const float *feats, const int32_t *rowof,
                              const int32_t *col, const double *val, const double *r, int64_t nnz,
                              float *out_b, hipStream_t s) {
    if (nnz <= 0) return hipSuccess;
    const int64_t nt = (nnz + 15) / 16;
    NetArgs a{wbf, feats, rowof, col, val, r, nullptr, 0, nnz, 0, nt, 1, nt, out_b, nullptr};
    hipLaunchKernelGGL(k_net<false>, dim3((unsigned)mlp_blocks(nt, 4096)), dim3(64 * WAVES), 0, s,
                       a);
    return hipGetLastError();
}

hipError_t launch_net_gradient(const uint16_t *wbf, const float *feats, const int32_t *rowof,
                               const int32_t *col, const double *val, const double *r,
                               const float *lh, int64_t p0, int64_t p1, int64_t tile0,
                               int64_t ntile, int64_t stride, int64_t tmod, int blocks,
                               float *gpart, double *gsum, float *grad, float *loss,
                               hipStream_t s) {
    NetArgs a{wbf, feats, rowof, col, val, r, lh, p0, p1, tile0, ntile, stride, tmod, nullptr, gpart};
    hipLaunchKernelGGL(k_net<true>, dim3((unsigned)blocks), dim3(64 * WAVES), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_grad_reduce, dim3((GSTRIDE + 15) / 16), dim3(256), 0, s, (int64_t)blocks,
                       gpart, gsum);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_grad_scale, dim3((kMlpParams + 1 + 255) / 256), dim3(256), 0, s, gsum, grad,
                       loss);
    return hipGetLastError();
}

hipError_t launch_adam(const float *grad, float *w, float *m, float *v, uint16_t *wbf, float lr,
                       int step, hipStream_t s) {
    const float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
    const float bc1 = (float)(1.0 - pow(0.9, step));
    const float bc2 = (float)(1.0 - pow(0.999, step));
    hipLaunchKernelGGL(k_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, grad, w, m, v, wbf, lr,
                       beta1, beta2, eps, bc1, bc2);
    return hipGetLastError();
}

hipError_t launch_mlp_init(float *w, float *m, float *v, uint16_t *wbf, uint64_t seed,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_init, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, w, m, v, wbf,
                       (uint32_t)seed, (uint32_t)(seed >> 32));
    return hipGetLastError();
}

hipError_t launch_params_bf16(const float *w, uint16_t *wbf, hipStream_t s) {
    hipLaunchKernelGGL(k_params_bf16, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, w, wbf);
    return hipGetLastError();
}

}  // namespace mc
