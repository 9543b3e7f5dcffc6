// Quantiser set-up and encoding for the quantisation-aware fine-tuning of Sec. 3.3:
//   * gamma, beta of the LSQ+ covariance codes from the range of each slot (beta = min,
//     gamma = the least float32 >= (max - min) / (2^b - 1));
//   * the residual-VQ codebooks by K-means (Lloyd iterations, Sec. 4.1 uses 5) per stage on the
//     residual colours, seeded with the points at indices floor(j N / B), a centroid whose
//     cluster empties staying put; distances and means in float64, partial sums per block added
//     in block order (deterministic); the moving average's running state (Sec. 3.4) starts at
//     each final centroid's count of nearest residuals and that count times the entry;
//   * encoding of float records into the codec layout of include/gi.h with the same fake
//     quantiser the fine-tuning renders with.
#include <hip/hip_runtime.h>

#include "gi_common.h"

namespace gi {

namespace {

constexpr int QB = 256;

// per-block min and max of slots 2..4: part[block][6] = min0..2, max0..2
__global__ __launch_bounds__(QB) void k_slot_range(const float4 *__restrict__ params, int64_t n,
                                                   float *__restrict__ part) {
    __shared__ float s[QB / 64][6];
    const int64_t i = (int64_t)blockIdx.x * QB + threadIdx.x;
    float v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    if (i < n) {
        const float4 a = params[2 * i], b = params[2 * i + 1];
        const float l[3] = {a.z, a.w, b.x};
        for (int k = 0; k < 3; ++k) {
            v[k] = l[k];
            v[3 + k] = l[k];
        }
    }
    for (int d = 32; d >= 1; d >>= 1)
        for (int k = 0; k < 3; ++k) {
            v[k] = fminf(v[k], __shfl_xor(v[k], d, 64));
            v[3 + k] = fmaxf(v[3 + k], __shfl_xor(v[3 + k], d, 64));
        }
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < 6; ++k) s[threadIdx.x >> 6][k] = v[k];
    __syncthreads();
    if (threadIdx.x < 6) {
        float r = s[0][threadIdx.x];
        for (int w = 1; w < QB / 64; ++w)
            r = threadIdx.x < 3 ? fminf(r, s[w][threadIdx.x]) : fmaxf(r, s[w][threadIdx.x]);
        part[(int64_t)blockIdx.x * 6 + threadIdx.x] = r;
    }
}

__global__ void k_lsq_init(const float *__restrict__ part, int64_t blocks, int32_t bits,
                           float *__restrict__ quant) {
    const int k = threadIdx.x;
    if (k >= 3) return;
    float lo = INFINITY, hi = -INFINITY;
    for (int64_t b = 0; b < blocks; ++b) {
        lo = fminf(lo, part[b * 6 + k]);
        hi = fmaxf(hi, part[b * 6 + 3 + k]);
    }
    const double top = (double)((1 << bits) - 1);
    const double exact = hi > lo ? ((double)hi - (double)lo) / top : 1.0;
    float g = (float)exact;
    if ((double)g < exact) g = nextafterf(g, INFINITY);
    quant[k] = g;
    quant[3 + k] = lo;
}

// residual colours of stage 0 = the record colours
__global__ __launch_bounds__(QB) void k_resid_init(const float4 *__restrict__ params, int64_t n,
                                                   double *__restrict__ resid) {
    const int64_t i = (int64_t)blockIdx.x * QB + threadIdx.x;
    if (i >= n) return;
    const float4 b = params[2 * i + 1];
    resid[3 * i] = b.y;
    resid[3 * i + 1] = b.z;
    resid[3 * i + 2] = b.w;
}

__global__ void k_kmeans_seed(const double *__restrict__ resid, int64_t n, int32_t k,
                              double *__restrict__ cent) {
    const int j = threadIdx.x;
    if (j >= k) return;
    const int64_t src = ((int64_t)j * n) / k;
    for (int c = 0; c < 3; ++c) cent[3 * j + c] = resid[3 * src + c];
}

__device__ inline int nearest(const double *cent, int k, double r0, double r1, double r2) {
    int best = 0;
    double bd = 0.0;
    for (int j = 0; j < k; ++j) {
        const double d0 = r0 - cent[3 * j], d1 = r1 - cent[3 * j + 1], d2 = r2 - cent[3 * j + 2];
        const double d = (d0 * d0 + d1 * d1) + d2 * d2;
        if (j == 0 || d < bd) {
            bd = d;
            best = j;
        }
    }
    return best;
}

// assignment and per-block sums per centroid: part[k][4][block] = (sum x, sum y, sum z, count)
// (entry-major, so that the update reads each entry's block sums contiguously)
__global__ __launch_bounds__(QB) void k_kmeans_assign(const double *__restrict__ resid,
                                                      int64_t n, int32_t k,
                                                      const double *__restrict__ cent,
                                                      double *__restrict__ part) {
#pragma clang fp contract(off)
    __shared__ double pts[QB][3];
    __shared__ int32_t lab[QB];
    __shared__ double sc[QAT_KMAX * 3];
    for (int t = threadIdx.x; t < 3 * k; t += QB) sc[t] = cent[t];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * QB + threadIdx.x;
    lab[threadIdx.x] = -1;
    if (i < n) {
        const double r0 = resid[3 * i], r1 = resid[3 * i + 1], r2 = resid[3 * i + 2];
        pts[threadIdx.x][0] = r0;
        pts[threadIdx.x][1] = r1;
        pts[threadIdx.x][2] = r2;
        lab[threadIdx.x] = nearest(sc, k, r0, r1, r2);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < 4 * k; t += QB) {
        const int j = t >> 2, c = t & 3;
        double acc = 0.0;
        for (int p = 0; p < QB; ++p)
            if (lab[p] == j) acc += c < 3 ? pts[p][c] : 1.0;
        part[(int64_t)t * gridDim.x + blockIdx.x] = acc;
    }
}

// one block of four waves: wave w adds the block sums of entries w, w + 4, ... (lanes in a
// fixed strided order, then a fixed shuffle tree)
__global__ __launch_bounds__(256) void k_kmeans_update(const double *__restrict__ part,
                                                       int64_t blocks, int32_t k,
                                                       double *__restrict__ cent) {
    __shared__ double tot[QAT_KMAX * 4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int t = wave; t < 4 * k; t += 4) {
        double acc = 0.0;
        for (int64_t b = lane; b < blocks; b += 64) acc += part[(int64_t)t * blocks + b];
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
        if (lane == 0) tot[t] = acc;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < 3 * k; t += blockDim.x) {
        const int j = t / 3, c = t % 3;
        const double cnt = tot[4 * j + 3];
        if (cnt > 0.0) cent[t] = tot[4 * j + c] / cnt;
    }
}

// running state of the codebooks' moving average at stage m: the number of residuals nearest
// each final centroid (the assignment sums of k_kmeans_assign, added in the fixed order of
// k_kmeans_update) and that count times the float32 entry
__global__ __launch_bounds__(256) void k_ema_init(const double *__restrict__ part, int64_t blocks,
                                                  int32_t k, const double *__restrict__ cent,
                                                  float *__restrict__ ema) {
#pragma clang fp contract(off)
    __shared__ double cnt[QAT_KMAX];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int j = wave; j < k; j += 4) {
        const int64_t t = 4 * (int64_t)j + 3;
        double acc = 0.0;
        for (int64_t b = lane; b < blocks; b += 64) acc += part[t * blocks + b];
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
        if (lane == 0) cnt[j] = acc;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < k; j += blockDim.x) {
        const double c = cnt[j];
        ema[4 * j] = (float)c;
        for (int ch = 0; ch < 3; ++ch)
            ema[4 * j + 1 + ch] = (float)(c * (double)(float)cent[3 * j + ch]);
    }
}

// codebook stage m (float32) from the centroids, and the residuals for the next stage
__global__ __launch_bounds__(QB) void k_kmeans_finish(double *__restrict__ resid, int64_t n,
                                                      int32_t k, const double *__restrict__ cent,
                                                      float *__restrict__ book) {
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * QB + threadIdx.x;
    if (blockIdx.x == 0)
        for (int t = threadIdx.x; t < 3 * k; t += QB) book[t] = (float)cent[t];
    if (i >= n) return;
    const double r0 = resid[3 * i], r1 = resid[3 * i + 1], r2 = resid[3 * i + 2];
    const int j = nearest(cent, k, r0, r1, r2);
    resid[3 * i] = r0 - cent[3 * j];
    resid[3 * i + 1] = r1 - cent[3 * j + 1];
    resid[3 * i + 2] = r2 - cent[3 * j + 2];
}

__global__ __launch_bounds__(QB) void k_qat_encode(const float4 *__restrict__ params, int64_t n,
                                                   QatArgs qa, uint32_t *__restrict__ mu,
                                                   uint8_t *__restrict__ codes,
                                                   uint8_t *__restrict__ index) {
    const int64_t i = (int64_t)blockIdx.x * QB + threadIdx.x;
    if (i >= n) return;
    const float4 a = params[2 * i], b = params[2 * i + 1];
    float q[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
    QuantFacts f;
    qat_fake_quant(q, qa, &f);
    const uint32_t hx = __builtin_bit_cast(uint16_t, (_Float16)a.x);
    const uint32_t hy = __builtin_bit_cast(uint16_t, (_Float16)a.y);
    mu[i] = hx | (hy << 16);
    for (int k = 0; k < 3; ++k) codes[3 * i + k] = (uint8_t)f.code[k];
    for (int m = 0; m < qa.stages; ++m) index[i * qa.stages + m] = (uint8_t)f.idx[m];
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + QB - 1) / QB); }

}  // namespace

size_t qat_init_scratch_bytes(int64_t n, int size) {
    const int64_t blocks = (n + QB - 1) / QB;
    // resid [n][3] f64, centroids [size][3] f64, partials [blocks][size][4] f64, range [blocks][6]
    return sizeof(double) * (3 * (size_t)n + 3 * (size_t)size + 4 * (size_t)blocks * size) +
           sizeof(float) * 6 * (size_t)blocks + 256;
}

hipError_t launch_qat_init(const float *params, int64_t n, const QatArgs &qa, int kmeans_iters,
                           float *ema, void *scratch, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + QB - 1) / QB;
    const float4 *p4 = reinterpret_cast<const float4 *>(params);
    double *resid = reinterpret_cast<double *>(scratch);
    double *cent = resid + 3 * n;
    double *part = cent + 3 * qa.size;
    float *range = reinterpret_cast<float *>(part + 4 * blocks * qa.size);
    float *quant = const_cast<float *>(qa.quant);
    hipLaunchKernelGGL(k_slot_range, dim3(blocks_for(n)), dim3(QB), 0, s, p4, n, range);
    hipLaunchKernelGGL(k_lsq_init, dim3(1), dim3(64), 0, s, range, blocks, qa.bits, quant);
    hipLaunchKernelGGL(k_resid_init, dim3(blocks_for(n)), dim3(QB), 0, s, p4, n, resid);
    for (int m = 0; m < qa.stages; ++m) {
        hipLaunchKernelGGL(k_kmeans_seed, dim3(1), dim3(QAT_KMAX), 0, s, resid, n, qa.size, cent);
        for (int it = 0; it < kmeans_iters; ++it) {
            hipLaunchKernelGGL(k_kmeans_assign, dim3(blocks_for(n)), dim3(QB), 0, s, resid, n,
                               qa.size, cent, part);
            hipLaunchKernelGGL(k_kmeans_update, dim3(1), dim3(256), 0, s, part, blocks, qa.size,
                               cent);
        }
        hipLaunchKernelGGL(k_kmeans_assign, dim3(blocks_for(n)), dim3(QB), 0, s, resid, n, qa.size,
                           cent, part);
        hipLaunchKernelGGL(k_ema_init, dim3(1), dim3(256), 0, s, part, blocks, qa.size, cent,
                           ema + (int64_t)m * qa.size * 4);
        hipLaunchKernelGGL(k_kmeans_finish, dim3(blocks_for(n)), dim3(QB), 0, s, resid, n,
                           qa.size, cent, quant + 6 + (int64_t)m * qa.size * 3);
    }
    return hipGetLastError();
}

hipError_t launch_qat_encode(const float *params, int64_t n, const QatArgs &qa, uint16_t *mu,
                             uint8_t *codes, uint8_t *index, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_qat_encode, dim3(blocks_for(n)), dim3(QB), 0, s,
                       reinterpret_cast<const float4 *>(params), n, qa,
                       reinterpret_cast<uint32_t *>(mu), codes, index);
    return hipGetLastError();
}

}  // namespace gi
