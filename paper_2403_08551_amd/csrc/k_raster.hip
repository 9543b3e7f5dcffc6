// Rasterisation kernels for gfx950: the per-tile forward (Eq. rasterization4), the per-tile
// adjoint (App. A.1), the fused fit kernel (forward, L2 loss gradient, adjoint) and the
// per-Gaussian kernels that finish the gradient (App. A.2) and apply the Adam update.
//
// Evaluation of sigma.  With L^{-1} d = (u1, u2), u1 = dx / l1 and u2 = (dy - l2 u1) / l3,
// sigma = |L^{-1} d|^2 / 2 (Eq. rasterization2 with Sigma = L L^T).  The projection kernel
// stores a = s/l1, b = s/l3, k = s l2 / (l1 l3) with s = sqrt(log2(e)/2), so that per pixel
//     u1 = a dx,  u2 = b dy - k dx,  exp(-sigma) = exp2(-(u1^2 + u2^2)).
// A sum of squares does not cancel, unlike the quadratic form with the inverse covariance, so
// float32 keeps sigma to a few ulp even for elongated, correlated Gaussians.
//
// Work mapping.  Forward: one workgroup per 16x16 tile, one pixel column segment per lane
// (PX pixels of one column), the tile's records read in sorted order through the scalar unit
// (every lane uses the same Gaussian at once), colour accumulated in float32 registers with a
// two-level sum (partial sums per chunk of 32 Gaussians).  Adjoint: one Gaussian per lane, the
// tile's 256 dL/dC values staged in LDS and read as broadcasts, so each lane reduces its own
// Gaussian over the tile's pixels in registers: no cross-lane reduction and no atomics.  The
// eight partial sums of each (tile, Gaussian) pair are stored at that pair's key position and
// the per-Gaussian kernel adds them in a fixed order, which keeps gradients deterministic.
#include "gi_common.h"

namespace gi {

namespace {

constexpr int CHUNK = 32;
constexpr int BWD_T = 256;

__device__ inline float ex2(float x) { return __builtin_amdgcn_exp2f(x); }

// One Gaussian's contribution to the PX pixels of this lane (A = mu_x, mu_y, a, b;
// B = k, c0, c1, c2).
template <int PX>
__device__ inline void fwd_eval(const float4 A, const float4 B, float px, const float (&py)[PX],
                                float (&part)[PX][3]) {
    const float dx = px - A.x;
    const float u1 = A.z * dx;
    const float u1s = u1 * u1;
    const float t = B.x * dx;
#pragma unroll
    for (int j = 0; j < PX; ++j) {
        const float dy = py[j] - A.y;
        const float u2 = fmaf(dy, A.w, -t);
        const float e = ex2(-fmaf(u2, u2, u1s));
        part[j][0] = fmaf(B.y, e, part[j][0]);
        part[j][1] = fmaf(B.z, e, part[j][1]);
        part[j][2] = fmaf(B.w, e, part[j][2]);
    }
}

// Forward accumulation for the PX pixels (one column) of this thread.  Records are read in
// groups of four through the scalar unit; the next group is requested before the current one is
// evaluated, so its latency overlaps the arithmetic.  Partial sums are folded into the totals
// every 32 Gaussians.
template <int PX>
__device__ inline void fwd_tile(const float4 *__restrict__ rec, uint2 r, float px,
                                const float (&py)[PX], float (&acc)[PX][3]) {
    float part[PX][3];
#pragma unroll
    for (int j = 0; j < PX; ++j) {
        acc[j][0] = acc[j][1] = acc[j][2] = 0.f;
        part[j][0] = part[j][1] = part[j][2] = 0.f;
    }
    const uint32_t ng = (r.y - r.x) / 4;
    uint32_t i = r.x;
    float4 cur[8];
    if (ng) {
#pragma unroll
        for (int k = 0; k < 8; ++k) cur[k] = rec[2 * (int64_t)i + k];
        // scalar loads complete out of order and can only be awaited all together: wait here so
        // that inside the loop only the prefetched group is outstanding during the arithmetic
        __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
    }
    for (uint32_t g = 0; g < ng; ++g) {
        float4 nxt[8];
        const bool more = g + 1 < ng;
        if (more) {
#pragma unroll
            for (int k = 0; k < 8; ++k) nxt[k] = rec[2 * (int64_t)(i + 4) + k];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) fwd_eval<PX>(cur[2 * k], cur[2 * k + 1], px, py, part);
        i += 4;
        if (((i - r.x) & (CHUNK - 1)) == 0) {
#pragma unroll
            for (int j = 0; j < PX; ++j) {
                acc[j][0] += part[j][0];
                acc[j][1] += part[j][1];
                acc[j][2] += part[j][2];
                part[j][0] = part[j][1] = part[j][2] = 0.f;
            }
        }
        if (more) {
#pragma unroll
            for (int k = 0; k < 8; ++k) cur[k] = nxt[k];
        }
    }
    for (; i < r.y; ++i) fwd_eval<PX>(rec[2 * (int64_t)i], rec[2 * (int64_t)i + 1], px, py, part);
#pragma unroll
    for (int j = 0; j < PX; ++j) {
        acc[j][0] += part[j][0];
        acc[j][1] += part[j][1];
        acc[j][2] += part[j][2];
    }
}

// Adjoint of one tile: Gaussian-per-lane over the tile's list, dL/dC of the tile in LDS.
template <int NT>
__device__ inline void bwd_tile(const float4 *__restrict__ rec, const uint32_t *__restrict__ slot,
                                uint2 r, const TileInfo &ti, const float4 *sg,
                                float4 *__restrict__ part) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const float x0 = (float)(ti.tx * TILE) + 0.5f;
    const float y0 = (float)(ti.ty * TILE) + 0.5f;
    for (uint32_t c = r.x + (uint32_t)wave * 64u; c < r.y; c += NT) {
        const uint32_t i = c + (uint32_t)lane;
        const bool act = i < r.y;
        float4 A = make_float4(0.f, 0.f, 0.f, 0.f), B = A;
        uint32_t sl = 0;
        if (act) {
            A = rec[2 * i];
            B = rec[2 * i + 1];
            sl = slot[i];
        }
        float dy[TILE];
#pragma unroll
        for (int rr = 0; rr < TILE; ++rr) dy[rr] = (y0 + (float)rr) - A.y;
        float C0 = 0.f, C1 = 0.f, C2 = 0.f, P1 = 0.f, P2 = 0.f, Q11 = 0.f, Q12 = 0.f, Q22 = 0.f;
        for (int cc = 0; cc < TILE; ++cc) {
            const float dx = (x0 + (float)cc) - A.x;
            const float u1 = A.z * dx;
            const float u1s = u1 * u1;
            const float t = B.x * dx;
            float Wc = 0.f, WU2 = 0.f, WU22 = 0.f;
#pragma unroll
            for (int rr = 0; rr < TILE; ++rr) {
                const float4 g = sg[rr * TILE + cc];
                const float u2 = fmaf(dy[rr], A.w, -t);
                const float e = ex2(-fmaf(u2, u2, u1s));
                C0 = fmaf(g.x, e, C0);
                C1 = fmaf(g.y, e, C1);
                C2 = fmaf(g.z, e, C2);
                const float gc = fmaf(g.z, B.w, fmaf(g.y, B.z, g.x * B.y));
                const float w = e * gc;  // -dL/dsigma of this pixel
                Wc += w;
                const float wu2 = w * u2;
                WU2 += wu2;
                WU22 = fmaf(wu2, u2, WU22);
            }
            P1 = fmaf(u1, Wc, P1);
            Q11 = fmaf(u1s, Wc, Q11);
            Q12 = fmaf(u1, WU2, Q12);
            P2 += WU2;
            Q22 += WU22;
        }
        if (act) {
            part[2 * (int64_t)sl] = make_float4(C0, C1, C2, P1);
            part[2 * (int64_t)sl + 1] = make_float4(P2, Q11, Q12, Q22);
        }
    }
}

template <int PX>
__global__ __launch_bounds__(256 / PX) void k_raster_fwd(const float4 *__restrict__ rec,
                                                         const uint2 *__restrict__ ranges,
                                                         ImgTable tab, float *__restrict__ image) {
    constexpr int ROWS = TILE / PX;
    const uint32_t tile = blockIdx.x;
    const TileInfo ti = tile_info(tab, tile);
    const int col = threadIdx.x & 15, row = threadIdx.x >> 4;
    const int x = ti.tx * TILE + col;
    const float px = (float)x + 0.5f;
    float py[PX];
#pragma unroll
    for (int j = 0; j < PX; ++j) py[j] = (float)(ti.ty * TILE + row + j * ROWS) + 0.5f;
    float acc[PX][3];
    fwd_tile<PX>(rec, ranges[tile], px, py, acc);
#pragma unroll
    for (int j = 0; j < PX; ++j) {
        const int y = ti.ty * TILE + row + j * ROWS;
        if (x < ti.W && y < ti.H) {
            const unsigned long long idx = (ti.pix_base + (unsigned long long)y * ti.W + x) * 3ull;
            image[idx] = acc[j][0];
            image[idx + 1] = acc[j][1];
            image[idx + 2] = acc[j][2];
        }
    }
}

__global__ __launch_bounds__(BWD_T) void k_raster_bwd(const float4 *__restrict__ rec,
                                                      const uint32_t *__restrict__ slot,
                                                      const uint2 *__restrict__ ranges,
                                                      ImgTable tab, const float *__restrict__ G,
                                                      float4 *__restrict__ part) {
    __shared__ float4 sg[TILE_PX];
    const uint32_t tile = blockIdx.x;
    const TileInfo ti = tile_info(tab, tile);
    for (int p = threadIdx.x; p < TILE_PX; p += BWD_T) {
        const int x = ti.tx * TILE + (p & 15), y = ti.ty * TILE + (p >> 4);
        float4 g = make_float4(0.f, 0.f, 0.f, 0.f);
        if (x < ti.W && y < ti.H) {
            const unsigned long long idx = (ti.pix_base + (unsigned long long)y * ti.W + x) * 3ull;
            g = make_float4(G[idx], G[idx + 1], G[idx + 2], 0.f);
        }
        sg[p] = g;
    }
    __syncthreads();
    bwd_tile<BWD_T>(rec, slot, ranges[tile], ti, sg, part);
}

// Fit step for one tile: forward, residual and dL/dC = 2 (C - T) / (3 H W) into LDS, per-tile
// sum of squared residuals, then the adjoint.
template <int PX>
__global__ __launch_bounds__(256 / PX) void k_raster_fit(const float4 *__restrict__ rec,
                                                         const uint32_t *__restrict__ slot,
                                                         const uint2 *__restrict__ ranges,
                                                         ImgTable tab,
                                                         const float *__restrict__ target,
                                                         float4 *__restrict__ part,
                                                         float *__restrict__ image_out,
                                                         float *__restrict__ loss_part) {
    constexpr int NT = 256 / PX;
    constexpr int ROWS = TILE / PX;
    __shared__ float4 sg[TILE_PX];
    __shared__ float red[NT / 64];
    const uint32_t tile = blockIdx.x;
    const TileInfo ti = tile_info(tab, tile);
    const uint2 r = ranges[tile];
    const int col = threadIdx.x & 15, row = threadIdx.x >> 4;
    const int x = ti.tx * TILE + col;
    const float px = (float)x + 0.5f;
    float py[PX];
#pragma unroll
    for (int j = 0; j < PX; ++j) py[j] = (float)(ti.ty * TILE + row + j * ROWS) + 0.5f;
    float acc[PX][3];
    fwd_tile<PX>(rec, r, px, py, acc);
    const float scale = 2.0f / (3.0f * (float)ti.H * (float)ti.W);
    float sq = 0.f;
#pragma unroll
    for (int j = 0; j < PX; ++j) {
        const int y = ti.ty * TILE + row + j * ROWS;
        float4 g = make_float4(0.f, 0.f, 0.f, 0.f);
        if (x < ti.W && y < ti.H) {
            const unsigned long long idx = (ti.pix_base + (unsigned long long)y * ti.W + x) * 3ull;
            const float r0 = acc[j][0] - target[idx];
            const float r1 = acc[j][1] - target[idx + 1];
            const float r2 = acc[j][2] - target[idx + 2];
            sq = fmaf(r0, r0, fmaf(r1, r1, fmaf(r2, r2, sq)));
            g = make_float4(scale * r0, scale * r1, scale * r2, 0.f);
            if (image_out) {
                image_out[idx] = acc[j][0];
                image_out[idx + 1] = acc[j][1];
                image_out[idx + 2] = acc[j][2];
            }
        }
        sg[(row + j * ROWS) * TILE + col] = g;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) sq += __shfl_xor(sq, d, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sq;
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0.f;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) s += red[w];
        loss_part[tile] = s;
    }
    bwd_tile<NT>(rec, slot, r, ti, sg, part);
}

// Per-Gaussian reduction of the (tile, Gaussian) partial sums in key order, then the chain rule
// through the Cholesky factor (App. A.2; see the file header for u1, u2):
//   dL/dmu_x = (P1 - (l2/l3) P2) / (s l1),      dL/dmu_y = P2 / (s l3),
//   dL/dl1   = (Q11 - (l2/l3) Q12) / (s^2 l1),  dL/dl2   = Q12 / (s^2 l3),  dL/dl3 = Q22 / (s^2 l3),
//   dL/dc'_k = C_k,
// with P1 = sum w u1, P2 = sum w u2, Q11 = sum w u1^2, Q12 = sum w u1 u2, Q22 = sum w u2^2 over
// the Gaussian's pixels (u scaled by s), w = exp(-sigma) <dL/dC, c'> = -dL/dsigma.
__device__ inline void gauss_grad(const float4 *__restrict__ params, int64_t i,
                                  const uint32_t *__restrict__ count,
                                  const uint32_t *__restrict__ off,
                                  const float4 *__restrict__ part, unsigned long long keys,
                                  float (&g)[8], float4 &q0, float4 &q1) {
    q0 = params[2 * i];
    q1 = params[2 * i + 1];
    const uint32_t cnt = count[i];
    const uint32_t o = off[i];
    float S[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (cnt && (unsigned long long)o + cnt <= keys) {
        for (uint32_t j = o; j < o + cnt; ++j) {
            const float4 a = part[2 * (int64_t)j], b = part[2 * (int64_t)j + 1];
            S[0] += a.x; S[1] += a.y; S[2] += a.z; S[3] += a.w;
            S[4] += b.x; S[5] += b.y; S[6] += b.z; S[7] += b.w;
        }
    }
    if (cnt == 0) {
#pragma unroll
        for (int k = 0; k < 8; ++k) g[k] = 0.f;
        return;
    }
    const float l1 = q0.z, l2 = q0.w, l3 = q1.x;
    const float is = (float)(1.0 / U_SCALE);
    const float is2 = (float)(1.0 / (U_SCALE * U_SCALE));
    const float r23 = l2 / l3;
    g[0] = (S[3] - r23 * S[4]) * is / l1;
    g[1] = S[4] * is / l3;
    g[2] = (S[5] - r23 * S[6]) * is2 / l1;
    g[3] = S[6] * is2 / l3;
    g[4] = S[7] * is2 / l3;
    g[5] = S[0];
    g[6] = S[1];
    g[7] = S[2];
}

__global__ __launch_bounds__(256) void k_grad_out(const float4 *__restrict__ params, int64_t n,
                                                  const uint32_t *__restrict__ count,
                                                  const uint32_t *__restrict__ off,
                                                  const float4 *__restrict__ part,
                                                  const DevState *__restrict__ st, int64_t cap,
                                                  float4 *__restrict__ dparams) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    unsigned long long keys = st->keys_total;
    if (keys > (unsigned long long)cap) keys = (unsigned long long)cap;
    float g[8];
    float4 q0, q1;
    gauss_grad(params, i, count, off, part, keys, g, q0, q1);
    dparams[2 * i] = make_float4(g[0], g[1], g[2], g[3]);
    dparams[2 * i + 1] = make_float4(g[4], g[5], g[6], g[7]);
}

// Adam on every Gaussian.  Bias corrections are computed once per block in float64.
__global__ __launch_bounds__(256) void k_adam(float4 *__restrict__ params, int64_t n,
                                              const uint32_t *__restrict__ count,
                                              const uint32_t *__restrict__ off,
                                              const float4 *__restrict__ part, DevState *st,
                                              int64_t cap, float4 *__restrict__ m4,
                                              float4 *__restrict__ v4, int32_t *step,
                                              AdamArgs hp) {
    __shared__ float s_bc[2];
    if (threadIdx.x == 0) {
        const double t = (double)*step;
        s_bc[0] = (float)(1.0 - pow((double)hp.beta1, t));
        s_bc[1] = (float)(1.0 - pow((double)hp.beta2, t));
    }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    // gradients incomplete on key overflow: leave the state alone
    if (i < n && !(st->flags & FLAG_KEY_OVERFLOW)) {
        unsigned long long keys = st->keys_total;
        if (keys > (unsigned long long)cap) keys = (unsigned long long)cap;
        float g[8];
        float4 q0, q1;
        gauss_grad(params, i, count, off, part, keys, g, q0, q1);
        const float bc1 = s_bc[0], bc2 = s_bc[1];
        float p[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
        const float4 m0 = m4[2 * i], m1 = m4[2 * i + 1], v0 = v4[2 * i], v1 = v4[2 * i + 1];
        float m[8] = {m0.x, m0.y, m0.z, m0.w, m1.x, m1.y, m1.z, m1.w};
        float v[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const float lr = k < 2 ? hp.lr_mu : (k < 5 ? hp.lr_l : hp.lr_c);
            m[k] = hp.beta1 * m[k] + (1.f - hp.beta1) * g[k];
            v[k] = hp.beta2 * v[k] + (1.f - hp.beta2) * g[k] * g[k];
            const float mh = m[k] / bc1, vh = v[k] / bc2;
            p[k] -= lr * mh / (sqrtf(vh) + hp.eps);
        }
        if (hp.l_min > 0.f) {
            if (fabsf(p[2]) < hp.l_min) p[2] = copysignf(hp.l_min, p[2]);
            if (fabsf(p[4]) < hp.l_min) p[4] = copysignf(hp.l_min, p[4]);
        }
        params[2 * i] = make_float4(p[0], p[1], p[2], p[3]);
        params[2 * i + 1] = make_float4(p[4], p[5], p[6], p[7]);
        m4[2 * i] = make_float4(m[0], m[1], m[2], m[3]);
        m4[2 * i + 1] = make_float4(m[4], m[5], m[6], m[7]);
        v4[2 * i] = make_float4(v[0], v[1], v[2], v[3]);
        v4[2 * i + 1] = make_float4(v[4], v[5], v[6], v[7]);
    }
}

// Per-image mean of the squared residuals from the per-tile sums (float64 accumulation), and the
// step counter advance.  One block per image.
__global__ __launch_bounds__(256) void k_finish(const float *__restrict__ loss_part, ImgTable tab,
                                                int64_t n_tiles, float *__restrict__ loss_out,
                                                int32_t *__restrict__ step) {
    __shared__ double red[4];
    const int b = blockIdx.x;
    if (loss_out) {
        uint32_t t0 = 0, t1 = (uint32_t)n_tiles;
        double npx;
        if (tab.B == 1) {
            npx = (double)tab.H * tab.W;
        } else {
            t0 = tab.tile_base[b];
            t1 = tab.tile_base[b + 1];
            npx = (double)tab.dims[b].x * tab.dims[b].y;
        }
        double s = 0.0;
        for (uint32_t t = t0 + threadIdx.x; t < t1; t += 256) s += (double)loss_part[t];
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0) loss_out[b] = (float)((red[0] + red[1] + red[2] + red[3]) / (3.0 * npx));
    }
    if (step && b == 0 && threadIdx.x == 0) *step += 1;
}

}  // namespace

hipError_t launch_raster_fwd(const RasterArgs &a, float *image, int px, hipStream_t s) {
    if (a.n_tiles <= 0) return hipSuccess;
    const float4 *rec = reinterpret_cast<const float4 *>(a.rec);
    switch (px) {
        case 1: hipLaunchKernelGGL(k_raster_fwd<1>, dim3((unsigned)a.n_tiles), dim3(256), 0, s, rec, a.ranges, a.tab, image); break;
        case 4: hipLaunchKernelGGL(k_raster_fwd<4>, dim3((unsigned)a.n_tiles), dim3(64), 0, s, rec, a.ranges, a.tab, image); break;
        default: hipLaunchKernelGGL(k_raster_fwd<2>, dim3((unsigned)a.n_tiles), dim3(128), 0, s, rec, a.ranges, a.tab, image); break;
    }
    return hipGetLastError();
}

hipError_t launch_raster_bwd(const RasterArgs &a, const float *dl, float *part, hipStream_t s) {
    if (a.n_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_raster_bwd, dim3((unsigned)a.n_tiles), dim3(BWD_T), 0, s,
                       reinterpret_cast<const float4 *>(a.rec), a.slot, a.ranges, a.tab, dl,
                       reinterpret_cast<float4 *>(part));
    return hipGetLastError();
}

hipError_t launch_raster_fit(const RasterArgs &a, const float *target, float *part,
                             float *image_out, float *loss_part, int px, hipStream_t s) {
    if (a.n_tiles <= 0) return hipSuccess;
    const float4 *rec = reinterpret_cast<const float4 *>(a.rec);
    float4 *p4 = reinterpret_cast<float4 *>(part);
    switch (px) {
        case 1: hipLaunchKernelGGL(k_raster_fit<1>, dim3((unsigned)a.n_tiles), dim3(256), 0, s, rec, a.slot, a.ranges, a.tab, target, p4, image_out, loss_part); break;
        case 4: hipLaunchKernelGGL(k_raster_fit<4>, dim3((unsigned)a.n_tiles), dim3(64), 0, s, rec, a.slot, a.ranges, a.tab, target, p4, image_out, loss_part); break;
        default: hipLaunchKernelGGL(k_raster_fit<2>, dim3((unsigned)a.n_tiles), dim3(128), 0, s, rec, a.slot, a.ranges, a.tab, target, p4, image_out, loss_part); break;
    }
    return hipGetLastError();
}

hipError_t launch_grad_out(const UpdateArgs &u, float *dparams, hipStream_t s) {
    if (u.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_grad_out, dim3((unsigned)((u.n + 255) / 256)), dim3(256), 0, s,
                       reinterpret_cast<const float4 *>(u.params_in), u.n, u.count, u.off,
                       reinterpret_cast<const float4 *>(u.part), u.state, u.cap,
                       reinterpret_cast<float4 *>(dparams));
    return hipGetLastError();
}

hipError_t launch_adam(const UpdateArgs &u, float *params, float *m, float *v, int32_t *step,
                       const AdamArgs &hp, const float *loss_part, const ImgTable &tab,
                       int64_t n_tiles, float *loss_out, hipStream_t s) {
    if (u.n > 0) {
        hipLaunchKernelGGL(k_adam, dim3((unsigned)((u.n + 255) / 256)), dim3(256), 0, s,
                           reinterpret_cast<float4 *>(params), u.n, u.count, u.off,
                           reinterpret_cast<const float4 *>(u.part), u.state, u.cap,
                           reinterpret_cast<float4 *>(m), reinterpret_cast<float4 *>(v), step, hp);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return launch_finish(loss_part, tab, n_tiles, loss_out, step, s);
}

hipError_t launch_finish(const float *loss_part, const ImgTable &tab, int64_t n_tiles,
                         float *loss_out, int32_t *step, hipStream_t s) {
    hipLaunchKernelGGL(k_finish, dim3((unsigned)tab.B), dim3(256), 0, s, loss_part, tab, n_tiles,
                       loss_out, step);
    return hipGetLastError();
}

}  // namespace gi
