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

// CHAINS dependent FMA chains per thread: iters * CHAINS lane FMAs per thread.
__global__ __launch_bounds__(THREADS) void k_fma(float *out, float x, float y, int iters) {
    float a[CHAINS];
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) a[c] = (float)(threadIdx.x + c);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
#pragma unroll
            for (int c = 0; c < CHAINS; ++c) a[c] = fmaf(a[c], x, y);
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

// Per step and chain: one exp2 chain and four FMA chains advance once each (4 FMAs per exp,
// the ratio of the raster kernels' inner loops is near 5 to 6): iters * 8 * CHAINS exps and
// four times as many FMAs per thread.
__global__ __launch_bounds__(THREADS) void k_mixed(float *out, float x, float y, int iters) {
    float e[CHAINS], f[CHAINS][4];
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) {
        e[c] = 0.01f * (float)(threadIdx.x + c);
#pragma unroll
        for (int j = 0; j < 4; ++j) f[c][j] = (float)(threadIdx.x + c + j);
    }
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
#pragma unroll
            for (int c = 0; c < CHAINS; ++c) {
                e[c] = __builtin_amdgcn_exp2f(-e[c]);
#pragma unroll
                for (int j = 0; j < 4; ++j) f[c][j] = fmaf(f[c][j], x, y);
            }
        }
    }
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) s += e[c] + f[c][0] + f[c][1] + f[c][2] + f[c][3];
    out[blockIdx.x * THREADS + threadIdx.x] = s;
}

__global__ __launch_bounds__(THREADS) void k_copy(const float4 *__restrict__ src,
                                                  float4 *__restrict__ dst, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * THREADS;
    for (int64_t i = (int64_t)blockIdx.x * THREADS + threadIdx.x; i < n; i += stride)
        dst[i] = src[i];
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

// kind 0: lane FMAs per second; 1: lane exp2 per second; 2: lane exp2 per second with four FMAs
// issued beside each one (also writes the FMAs per second of that run to *rate2); 3: copy
// bandwidth, bytes read plus bytes written per second, of n_bytes copied device to device.
// iters sizes the arithmetic kernels (loop trips; 8 x 8 operations per trip and chain set).
// Returns 0 on success, -1 on a bad argument, -3 on a HIP error.  Allocates (kind 3 and the
// result buffer) and synchronises.
int peaks_run(int kind, int64_t iters_or_bytes, double *rate, double *rate2) {
    if (!rate || kind < 0 || kind > 3 || iters_or_bytes <= 0) return -1;
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
        for (int rep = 0; rep < 2 && rc == 0; ++rep) {  // the first run warms up
            ok(hipEventRecord(a, nullptr));
            if (kind == 0)
                hipLaunchKernelGGL(k_fma, dim3(blocks), dim3(THREADS), 0, nullptr, out, 0.999f,
                                   0.001f, iters);
            else if (kind == 1)
                hipLaunchKernelGGL(k_exp, dim3(blocks), dim3(THREADS), 0, nullptr, out, iters);
            else if (kind == 2)
                hipLaunchKernelGGL(k_mixed, dim3(blocks), dim3(THREADS), 0, nullptr, out, 0.999f,
                                   0.001f, iters);
            else
                hipLaunchKernelGGL(k_copy, dim3(blocks * 4), dim3(THREADS), 0, nullptr, src,
                                   dst, n4);
            ok(hipGetLastError());
            ok(hipEventRecord(b, nullptr));
            ok(hipEventSynchronize(b));
        }
        float ms = 0.f;
        if (rc == 0 && ok(hipEventElapsedTime(&ms, a, b)) && ms > 0.f) {
            const double s = 1e-3 * ms;
            const double lanes = (double)blocks * THREADS;
            const double per_lane = (double)iters * 8 * CHAINS;
            if (kind == 0) *rate = lanes * per_lane / s;
            if (kind == 1) *rate = lanes * per_lane / s;
            if (kind == 2) {
                *rate = lanes * per_lane / s;
                if (rate2) *rate2 = 4.0 * lanes * per_lane / s;
            }
            if (kind == 3) *rate = 2.0 * 16.0 * (double)n4 / s;
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
