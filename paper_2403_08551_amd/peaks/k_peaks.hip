// Microbenchmarks behind the roofline denominators: the FP32 FMA issue rate, the rate of the
// base-2 exponential (v_exp_f32) alone and interleaved with FMAs, and the device-memory copy
// bandwidth, each timed with HIP events on the caller's stream.  Built as a library of its own
// (libgi_peaks.so): measurement tooling, not part of the renderer's ABI.
//
// Kernels are sized to fill the chip: 256 CUs x 8 workgroups of 256 threads, eight independent
// chains per thread (enough independent work to hide every latency), loop counts as arguments
// so that nothing folds at compile time, results stored so that nothing is dropped.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int CHAINS = 8;
constexpr int THREADS = 256;

// CHAINS dependent FMA chains per thread, a[c] += x[c] y[c] with every operand in a VGPR (the
// v_fmac_f32 form the raster kernels' sums take; an FMA that reads two scalar operands issues
// at half this rate): iters * 8 * CHAINS lane FMAs per thread.
__global__ __launch_bounds__(THREADS) void k_fma(float *out, float x, float y, int iters) {
    float a[CHAINS], xs[CHAINS], ys[CHAINS];
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) {
        a[c] = (float)(threadIdx.x + c);
        xs[c] = x + 0.001f * (float)(c * threadIdx.x);
        ys[c] = y - 0.002f * (float)c;
    }
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
#pragma unroll
            for (int c = 0; c < CHAINS; ++c) a[c] = fmaf(xs[c], ys[c], a[c]);
        }
    }
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) s += a[c];
    out[blockIdx.x * THREADS + threadIdx.x] = s;
}

// CHAINS dependent exp2 chains per thread (a <- 2^-a stays in (0, 1]): iters * 8 * CHAINS
// lane exponentials per thread.
__global__ __launch_bounds__(THREADS) void k_exp(float *out, int iters) {
    float a[CHAINS];
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) a[c] = 0.01f * (float)(threadIdx.x + c);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
#pragma unroll
            for (int c = 0; c < CHAINS; ++c) a[c] = __builtin_amdgcn_exp2f(-a[c]);
        }
    }
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) s += a[c];
    out[blockIdx.x * THREADS + threadIdx.x] = s;
}

// The marginal cost of an exp2 among other VALU work: per step and chain an add, an exp2 of its
// result and an add of that into a sum (WITH_EXP), or the same without the exp2; the difference
// of the two times is the exp2's.  iters * 8 * CHAINS steps per thread.
template <bool WITH_EXP>
__global__ __launch_bounds__(THREADS) void k_mixed(float *out, float x, float y, int iters) {
    float a[CHAINS], e[CHAINS];
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) {
        a[c] = -0.01f * (float)(threadIdx.x + c);
        e[c] = 0.f;
    }
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
#pragma unroll
            for (int c = 0; c < CHAINS; ++c) {
                a[c] = a[c] - y;
                e[c] += WITH_EXP ? __builtin_amdgcn_exp2f(a[c]) : a[c];
            }
        }
        if (!WITH_EXP) x += 0.f;
    }
    float s = x;
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) s += a[c] + e[c];
    out[blockIdx.x * THREADS + threadIdx.x] = s;
}

// The smallest per-pair instruction sequences of the raster kernels, in loops: a forward pair
// (u2 by one FMA, the exponent by one FMA, exp2, three colour FMAs: 5 VALU + 1 exp2) and an
// adjoint pair (u2, exponent, exp2, three colour sums, <g, c'> by a multiply and two FMAs,
// w u2 by two multiplies, the u2 and u2^2 sums: 12 VALU + 1 exp2).  Four independent pairs per
// step (four rows, as a forward lane owns them); the offsets move every step so nothing folds.
// iters * 8 * 4 pairs per thread.
__global__ __launch_bounds__(THREADS) void k_fwd_pairs(float *out, float b, float u1s, int iters) {
    float acc[4][3];
    float u2b = 0.001f * (float)threadIdx.x - 2.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j][0] = acc[j][1] = acc[j][2] = 0.f;
    const float c0 = 0.3f, c1 = 0.5f, c2 = 0.7f;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float u2 = fmaf((float)j, b, u2b);
                const float e = __builtin_amdgcn_exp2f(-fmaf(u2, u2, u1s));
                acc[j][0] = fmaf(c0, e, acc[j][0]);
                acc[j][1] = fmaf(c1, e, acc[j][1]);
                acc[j][2] = fmaf(c2, e, acc[j][2]);
            }
            u2b += 0.0625f;
        }
        u2b -= 0.5f;
    }
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) s += acc[j][0] + acc[j][1] + acc[j][2];
    out[blockIdx.x * THREADS + threadIdx.x] = s;
}

__global__ __launch_bounds__(THREADS) void k_bwd_pairs(float *out, float b, float u1s, int iters) {
    // dL/dC of 16 pixels in LDS, read per pair as the adjoint reads its tile's values
    __shared__ float4 sg[16];
    if (threadIdx.x < 16)
        sg[threadIdx.x] = make_float4(0.01f * (float)threadIdx.x - 0.07f, 0.2f - 0.013f * (float)threadIdx.x,
                                      0.05f + 0.007f * (float)threadIdx.x, 0.f);
    __syncthreads();
    float D[3] = {0.f, 0.f, 0.f}, WU2 = 0.f, WU22 = 0.f;
    float t = 0.001f * (float)threadIdx.x;
    const float c0 = 0.3f, c1 = 0.5f, c2 = 0.7f;
    for (int i = 0; i < iters; ++i) {
        const int rot = i & 15;  // the pixels' order moves every trip: nothing is hoisted
#pragma unroll
        for (int k = 0; k < 8; ++k) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float4 g = sg[(rot + 4 * k + j) & 15];
                const float u2 = fmaf((float)j, b, -t);
                const float e = __builtin_amdgcn_exp2f(-fmaf(u2, u2, u1s));
                D[0] = fmaf(g.x, e, D[0]);
                D[1] = fmaf(g.y, e, D[1]);
                D[2] = fmaf(g.z, e, D[2]);
                const float gc = fmaf(g.z, c2, fmaf(g.y, c1, g.x * c0));
                const float wu2 = (e * gc) * u2;
                WU2 += wu2;
                WU22 = fmaf(wu2, u2, WU22);
            }
            t += 0.0625f;
        }
        t -= 0.375f;
    }
    out[blockIdx.x * THREADS + threadIdx.x] = D[0] + D[1] + D[2] + WU2 + WU22;
}

// Grid-stride copy, four independent 16-byte loads in flight per thread before the stores.
__global__ __launch_bounds__(THREADS) void k_copy(const float4 *__restrict__ src,
                                                  float4 *__restrict__ dst, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * THREADS;
    int64_t i = (int64_t)blockIdx.x * THREADS + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const float4 a = src[i], b = src[i + stride], c = src[i + 2 * stride],
                     d = src[i + 3 * stride];
        dst[i] = a;
        dst[i + stride] = b;
        dst[i + 2 * stride] = c;
        dst[i + 3 * stride] = d;
    }
    for (; i < n; i += stride) dst[i] = src[i];
}

int cu_count() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return cus;
}

}  // namespace

extern "C" {

// kind 0: lane FMAs per second (v_fmac_f32); 1: lane exp2 per second (exp2 alone); 2: lane exp2
// per second from the marginal cost of an exp2 among adds (also writes the rate of the adds-only
// steps to *rate2); 3: copy bandwidth, bytes read plus bytes written per second, of n_bytes
// copied device to device; 4, 5: forward and adjoint pixel-Gaussian pairs per second of the
// smallest per-pair sequences.
// iters sizes the arithmetic kernels (loop trips; 8 x 8 operations per trip and chain set).
// One untimed run, then the fastest of three timed runs.  Returns 0 on success, -1 on a bad argument, -3 on a HIP error.  Allocates (kind 3 and the
// result buffer) and synchronises.
int peaks_run(int kind, int64_t iters_or_bytes, double *rate, double *rate2) {
    if (!rate || kind < 0 || kind > 5 || iters_or_bytes <= 0) return -1;
    const int cus = cu_count();
    if (cus <= 0) return -3;
    const int blocks = cus * 8;
    hipEvent_t a = nullptr, b = nullptr;
    float *out = nullptr;
    float4 *src = nullptr, *dst = nullptr;
    int rc = 0;
    auto ok = [&](hipError_t e) {
        if (e != hipSuccess && rc == 0) rc = -3;
        return rc == 0;
    };
    if (ok(hipEventCreate(&a)) && ok(hipEventCreate(&b)) &&
        ok(hipMalloc((void **)&out, sizeof(float) * (size_t)blocks * THREADS))) {
        const int iters = (int)(kind == 3 ? 1 : iters_or_bytes);
        const int64_t n4 = kind == 3 ? iters_or_bytes / 16 : 0;
        if (kind == 3 && ok(hipMalloc((void **)&src, 16 * (size_t)n4)))
            ok(hipMalloc((void **)&dst, 16 * (size_t)n4));
        if (kind == 3 && rc == 0) ok(hipMemset(src, 0, 16 * (size_t)n4));
        // one untimed run, then the fastest of three timed runs; kind 2 alternates its two
        // kernels (adds only on even runs) and keeps the fastest of each
        float best[2] = {0.f, 0.f};
        const int runs = kind == 2 ? 8 : 4;
        for (int rep = 0; rep < runs && rc == 0; ++rep) {
            const int which = kind == 2 ? rep % 2 : 0;
            ok(hipEventRecord(a, nullptr));
            if (kind == 0)
                hipLaunchKernelGGL(k_fma, dim3(blocks), dim3(THREADS), 0, nullptr, out, 0.999f,
                                   0.001f, iters);
            else if (kind == 1)
                hipLaunchKernelGGL(k_exp, dim3(blocks), dim3(THREADS), 0, nullptr, out, iters);
            else if (kind == 2 && which == 0)
                hipLaunchKernelGGL(k_mixed<false>, dim3(blocks), dim3(THREADS), 0, nullptr, out,
                                   0.999f, 0.0001f, iters);
            else if (kind == 2)
                hipLaunchKernelGGL(k_mixed<true>, dim3(blocks), dim3(THREADS), 0, nullptr, out,
                                   0.999f, 0.0001f, iters);
            else if (kind == 4)
                hipLaunchKernelGGL(k_fwd_pairs, dim3(blocks), dim3(THREADS), 0, nullptr, out,
                                   0.37f, 0.25f, iters);
            else if (kind == 5)
                hipLaunchKernelGGL(k_bwd_pairs, dim3(blocks), dim3(THREADS), 0, nullptr, out,
                                   0.37f, 0.25f, iters);
            else
                hipLaunchKernelGGL(k_copy, dim3(blocks * 4), dim3(THREADS), 0, nullptr, src,
                                   dst, n4);
            ok(hipGetLastError());
            ok(hipEventRecord(b, nullptr));
            ok(hipEventSynchronize(b));
            float t = 0.f;
            if (rc == 0 && rep >= (kind == 2 ? 2 : 1) && ok(hipEventElapsedTime(&t, a, b)) &&
                t > 0.f)
                best[which] = best[which] > 0.f ? (t < best[which] ? t : best[which]) : t;
        }
        const float ms = best[kind == 2 ? 1 : 0];
        if (rc == 0 && ms > 0.f) {
            const double sec = 1e-3 * ms;
            const double lanes = (double)blocks * THREADS;
            const double per_lane = (double)iters * 8 * CHAINS;
            if (kind == 0 || kind == 1) *rate = lanes * per_lane / sec;
            if (kind == 2) {
                // exp2s per second from the time the exp2s add to the same steps
                const double extra = sec - 1e-3 * best[0];
                *rate = extra > 0.0 ? lanes * per_lane / extra : 0.0;
                if (rate2) *rate2 = lanes * per_lane / (1e-3 * best[0]);
            }
            if (kind == 3) *rate = 2.0 * 16.0 * (double)n4 / sec;
            if (kind == 4 || kind == 5) *rate = lanes * (double)iters * 8 * 4 / sec;
        }
    }
    if (out) (void)hipFree(out);
    if (src) (void)hipFree(src);
    if (dst) (void)hipFree(dst);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    return rc;
}

}  // extern "C"
