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
// groups of four through the scalar unit into two register sets used in turn: the next group is
// requested before the current one is evaluated, so its latency overlaps the arithmetic.
// Scalar loads complete out of order and can only be awaited together, so each half-step first
// waits for everything (only the group about to be used is outstanding then) and only then
// issues the next request.  Partial sums are folded into the totals every 32 Gaussians.
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
    float4 ga[8], gb[8];
    auto fold = [&]() {
        if (((i - r.x) & (CHUNK - 1)) == 0) {
#pragma unroll
            for (int j = 0; j < PX; ++j) {
                acc[j][0] += part[j][0];
                acc[j][1] += part[j][1];
                acc[j][2] += part[j][2];
                part[j][0] = part[j][1] = part[j][2] = 0.f;
            }
        }
    };
    if (ng) {
#pragma unroll
        for (int k = 0; k < 8; ++k) ga[k] = rec[2 * (int64_t)i + k];
    }
    for (uint32_t g = 0; g < ng;) {
        __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): group g is in ga
        if (g + 1 < ng) {
#pragma unroll
            for (int k = 0; k < 8; ++k) gb[k] = rec[2 * (int64_t)(i + 4) + k];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) fwd_eval<PX>(ga[2 * k], ga[2 * k + 1], px, py, part);
        i += 4;
        fold();
        if (++g >= ng) break;
        __builtin_amdgcn_s_waitcnt(0xc07f);  // group g is in gb
        if (g + 1 < ng) {
#pragma unroll
            for (int k = 0; k < 8; ++k) ga[k] = rec[2 * (int64_t)(i + 4) + k];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) fwd_eval<PX>(gb[2 * k], gb[2 * k + 1], px, py, part);
        i += 4;
        fold();
        ++g;
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

// ---- alpha blending (Eq. rasterization1 with Eq. rasterization2) -----------------------------
//
// Per pixel, in the tile's (ascending id) order: alpha = min(o exp(-sigma), ALPHA_MAX),
// C += c alpha T, T *= 1 - alpha, T starting at 1.  The adjoint walks the same order again with
// D = C - (colour accumulated so far including Gaussian k), which is T_{k+1} S_k for S_k the
// colour blended behind k, so dC/dalpha_k = T_k c_k - D / (1 - alpha_k) (no reverse pass and
// no division by a running T).  Pixel-per-lane: one wave per tile, four pixels of a column per
// lane; each (tile, Gaussian) pair's sums are reduced across the wave and stored at its key.

template <int PX>
__device__ inline void alpha_forward(const float4 *__restrict__ rec,
                                     const float *__restrict__ rec_o, uint2 r, float px,
                                     const float (&py)[PX], float (&acc)[PX][3],
                                     float (&T)[PX]) {
#pragma unroll
    for (int j = 0; j < PX; ++j) {
        acc[j][0] = acc[j][1] = acc[j][2] = 0.f;
        T[j] = 1.f;
    }
    for (uint32_t i = r.x; i < r.y; ++i) {
        const float4 A = rec[2 * (int64_t)i], B = rec[2 * (int64_t)i + 1];
        const float o = rec_o[i];
        const float dx = px - A.x;
        const float u1 = A.z * dx;
        const float u1s = u1 * u1;
        const float t = B.x * dx;
#pragma unroll
        for (int j = 0; j < PX; ++j) {
            const float u2 = fmaf(py[j] - A.y, A.w, -t);
            const float e = ex2(-fmaf(u2, u2, u1s));
            const float a = fminf(o * e, ALPHA_MAX);
            const float w = a * T[j];
            acc[j][0] = fmaf(B.y, w, acc[j][0]);
            acc[j][1] = fmaf(B.z, w, acc[j][1]);
            acc[j][2] = fmaf(B.w, w, acc[j][2]);
            T[j] *= 1.f - a;
        }
    }
}

template <int PX>
__global__ __launch_bounds__(256 / PX) void k_alpha_fwd(const float4 *__restrict__ rec,
                                                        const float *__restrict__ rec_o,
                                                        const uint2 *__restrict__ ranges,
                                                        ImgTable tab, float *__restrict__ image) {
    constexpr int ROWS = TILE / PX;
    const uint32_t tile = blockIdx.x;
    const TileInfo ti = tile_info(tab, tile);
    const int col = threadIdx.x & 15, row = threadIdx.x >> 4;
    const int x = ti.tx * TILE + col;
    const float px = (float)x + 0.5f;
    float py[PX], T[PX], acc[PX][3];
#pragma unroll
    for (int j = 0; j < PX; ++j) py[j] = (float)(ti.ty * TILE + row + j * ROWS) + 0.5f;
    alpha_forward<PX>(rec, rec_o, ranges[tile], px, py, acc, T);
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

__device__ inline float wave_sum(float v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// Adjoint walk of one tile (one wave, four pixels per lane): D holds the final colours on entry,
// g the pixels' dL/dC.
__device__ inline void alpha_adjoint(const float4 *__restrict__ rec,
                                     const float *__restrict__ rec_o,
                                     const uint32_t *__restrict__ slot, uint2 r, float px,
                                     const float (&py)[4], float (&D)[4][3],
                                     const float (&g)[4][3], float4 *__restrict__ part) {
    constexpr int PX = 4;
    float T[PX];
#pragma unroll
    for (int j = 0; j < PX; ++j) T[j] = 1.f;
    for (uint32_t i = r.x; i < r.y; ++i) {
        const float4 A = rec[2 * (int64_t)i], B = rec[2 * (int64_t)i + 1];
        const float o = rec_o[i];
        const float dx = px - A.x;
        const float u1 = A.z * dx;
        const float u1s = u1 * u1;
        const float t = B.x * dx;
        float C0 = 0.f, C1 = 0.f, C2 = 0.f, SO = 0.f, W = 0.f, WU2 = 0.f, WU22 = 0.f;
#pragma unroll
        for (int j = 0; j < PX; ++j) {
            const float u2 = fmaf(py[j] - A.y, A.w, -t);
            const float e = ex2(-fmaf(u2, u2, u1s));
            const float oe = o * e;
            const float a = fminf(oe, ALPHA_MAX);
            const float w = a * T[j];
            D[j][0] = fmaf(-B.y, w, D[j][0]);
            D[j][1] = fmaf(-B.z, w, D[j][1]);
            D[j][2] = fmaf(-B.w, w, D[j][2]);
            C0 = fmaf(g[j][0], w, C0);
            C1 = fmaf(g[j][1], w, C1);
            C2 = fmaf(g[j][2], w, C2);
            const float gc = fmaf(g[j][2], B.w, fmaf(g[j][1], B.z, g[j][0] * B.y));
            const float gd = fmaf(g[j][2], D[j][2], fmaf(g[j][1], D[j][1], g[j][0] * D[j][0]));
            const float ga = fmaf(T[j], gc, -gd * __builtin_amdgcn_rcpf(1.f - a));  // dL/dalpha
            const float gae = oe < ALPHA_MAX ? ga * e : 0.f;  // clamped: no dependence on o, sigma
            SO += gae;
            const float ws = o * gae;  // -dL/dsigma
            W += ws;
            const float wu2 = ws * u2;
            WU2 += wu2;
            WU22 = fmaf(wu2, u2, WU22);
            T[j] *= 1.f - a;
        }
        const float P1 = wave_sum(u1 * W), Q11 = wave_sum(u1s * W), Q12 = wave_sum(u1 * WU2);
        const float P2 = wave_sum(WU2), Q22 = wave_sum(WU22);
        C0 = wave_sum(C0);
        C1 = wave_sum(C1);
        C2 = wave_sum(C2);
        SO = wave_sum(SO);
        if (threadIdx.x == 0) {
            const int64_t sl = slot[i];
            part[3 * sl] = make_float4(C0, C1, C2, P1);
            part[3 * sl + 1] = make_float4(P2, Q11, Q12, Q22);
            part[3 * sl + 2] = make_float4(SO, 0.f, 0.f, 0.f);
        }
    }
}

// One wave per tile, 4 pixels per lane.
__global__ __launch_bounds__(64) void k_alpha_bwd(const float4 *__restrict__ rec,
                                                  const float *__restrict__ rec_o,
                                                  const uint32_t *__restrict__ slot,
                                                  const uint2 *__restrict__ ranges, ImgTable tab,
                                                  const float *__restrict__ G,
                                                  float4 *__restrict__ part) {
    constexpr int PX = 4, ROWS = TILE / PX;
    const uint32_t tile = blockIdx.x;
    const TileInfo ti = tile_info(tab, tile);
    const uint2 r = ranges[tile];
    const int col = threadIdx.x & 15, row = threadIdx.x >> 4;
    const int x = ti.tx * TILE + col;
    const float px = (float)x + 0.5f;
    float py[PX], T[PX], D[PX][3], g[PX][3];
#pragma unroll
    for (int j = 0; j < PX; ++j) {
        const int y = ti.ty * TILE + row + j * ROWS;
        py[j] = (float)y + 0.5f;
        g[j][0] = g[j][1] = g[j][2] = 0.f;
        if (x < ti.W && y < ti.H) {
            const unsigned long long idx = (ti.pix_base + (unsigned long long)y * ti.W + x) * 3ull;
            g[j][0] = G[idx];
            g[j][1] = G[idx + 1];
            g[j][2] = G[idx + 2];
        }
    }
    alpha_forward<PX>(rec, rec_o, r, px, py, D, T);
    alpha_adjoint(rec, rec_o, slot, r, px, py, D, g, part);
}

// Fit step of one tile with alpha blending: forward, residual, dL/dC = 2 (C - T) / (3 H W) in
// registers, per-tile sum of squared residuals, then the adjoint walk.
__global__ __launch_bounds__(64) void k_alpha_fit(const float4 *__restrict__ rec,
                                                  const float *__restrict__ rec_o,
                                                  const uint32_t *__restrict__ slot,
                                                  const uint2 *__restrict__ ranges, ImgTable tab,
                                                  const float *__restrict__ target,
                                                  float4 *__restrict__ part,
                                                  float *__restrict__ image_out,
                                                  float *__restrict__ loss_part) {
    constexpr int PX = 4, ROWS = TILE / PX;
    const uint32_t tile = blockIdx.x;
    const TileInfo ti = tile_info(tab, tile);
    const uint2 r = ranges[tile];
    const int col = threadIdx.x & 15, row = threadIdx.x >> 4;
    const int x = ti.tx * TILE + col;
    const float px = (float)x + 0.5f;
    float py[PX], T[PX], D[PX][3], g[PX][3];
#pragma unroll
    for (int j = 0; j < PX; ++j) py[j] = (float)(ti.ty * TILE + row + j * ROWS) + 0.5f;
    alpha_forward<PX>(rec, rec_o, r, px, py, D, T);
    const float scale = 2.0f / (3.0f * (float)ti.H * (float)ti.W);
    float sq = 0.f;
#pragma unroll
    for (int j = 0; j < PX; ++j) {
        const int y = ti.ty * TILE + row + j * ROWS;
        g[j][0] = g[j][1] = g[j][2] = 0.f;
        if (x < ti.W && y < ti.H) {
            const unsigned long long idx = (ti.pix_base + (unsigned long long)y * ti.W + x) * 3ull;
            const float r0 = D[j][0] - target[idx];
            const float r1 = D[j][1] - target[idx + 1];
            const float r2 = D[j][2] - target[idx + 2];
            sq = fmaf(r0, r0, fmaf(r1, r1, fmaf(r2, r2, sq)));
            g[j][0] = scale * r0;
            g[j][1] = scale * r1;
            g[j][2] = scale * r2;
            if (image_out) {
                image_out[idx] = D[j][0];
                image_out[idx + 1] = D[j][1];
                image_out[idx + 2] = D[j][2];
            }
        }
    }
    sq = wave_sum(sq);
    if (threadIdx.x == 0) loss_part[tile] = sq;
    alpha_adjoint(rec, rec_o, slot, r, px, py, D, g, part);
}

// Per-Gaussian gradient: the (tile, Gaussian) partial sums of Gaussian i, then the chain rule
// through the Cholesky factor (App. A.2; u1, u2 as in the file header, scaled by s):
//   dL/dmu_x = (P1 - (l2/l3) P2) / (s l1),      dL/dmu_y = P2 / (s l3),
//   dL/dl1   = (Q11 - (l2/l3) Q12) / (s^2 l1),  dL/dl2   = Q12 / (s^2 l3),  dL/dl3 = Q22 / (s^2 l3),
//   dL/dc'_k = C_k,
// with P1 = sum w u1, P2 = sum w u2, Q11 = sum w u1^2, Q12 = sum w u1 u2, Q22 = sum w u2^2 over
// the Gaussian's pixels, w = exp(-sigma) <dL/dC, c'> = -dL/dsigma.
//
// Rotation-scale records (s1, s2, theta), Sigma = R S^2 R^T (Eq. RSSR).  The same sums give
// dL/dSigma = (1/2) L^{-T} Q L^{-1} with Q = [[Q11, Q12], [Q12, Q22]] / s^2, L the Cholesky
// factor of Sigma.  With O = L^{-1} R S (orthogonal: both L^{-1} and S^{-1} R^T whiten d) and
// V = O^T Q O, the derivatives of Sigma along s1, s2 and theta, R diag(2 s1, 0) R^T,
// R diag(0, 2 s2) R^T and (s1^2 - s2^2)(r1 r2^T + r2 r1^T) (r1, r2 the columns of R), give
//   dL/ds1 = V11 / s1,  dL/ds2 = V22 / s2,  dL/dtheta = (s1^2 - s2^2) V12 / (s1 s2),
// and dL/dmu is the Cholesky expression with this L.  The factor is rebuilt in float64.
//
// Four lanes serve one Gaussian: lane q adds partials q, q + 4, ... of its key range, the quad
// combines the four sums (a fixed order, so results are reproducible), and lane q then owns
// parameters 2q and 2q + 1 for the output or the Adam update.
constexpr int UPD_T = 256;
constexpr int UPD_G = UPD_T / 4;  // Gaussians per block

template <int COV, int NV = 2>
__device__ inline void quad_grad(const float4 *__restrict__ params, int64_t i, int q,
                                 const uint32_t *__restrict__ count,
                                 const uint32_t *__restrict__ off,
                                 const float4 *__restrict__ part, unsigned long long keys,
                                 float (&g)[8], float4 &q0, float4 &q1, float *extra = nullptr) {
    constexpr int NS = NV == 3 ? 9 : 8;  // sums per key: 8, or 9 with the opacity sum
    q0 = params[2 * i];
    q1 = params[2 * i + 1];
    const uint32_t cnt = count[i];
    const uint32_t o = off[i];
    float S[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) S[k] = 0.f;
    if (cnt && (unsigned long long)o + cnt <= keys) {
        for (uint32_t j = o + (uint32_t)q; j < o + cnt; j += 4) {
            const float4 a = part[NV * (int64_t)j], b = part[NV * (int64_t)j + 1];
            S[0] += a.x; S[1] += a.y; S[2] += a.z; S[3] += a.w;
            S[4] += b.x; S[5] += b.y; S[6] += b.z; S[7] += b.w;
            if constexpr (NV == 3) S[8] += part[NV * (int64_t)j + 2].x;
        }
    }
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        S[k] += __shfl_xor(S[k], 1, 4);
        S[k] += __shfl_xor(S[k], 2, 4);
    }
    if (extra) *extra = cnt ? S[NS - 1] : 0.f;
    if (cnt == 0) {
#pragma unroll
        for (int k = 0; k < 8; ++k) g[k] = 0.f;
        return;
    }
    if (COV == COV_ROTATION_SCALE) {
        const double s1 = q0.z, s2 = q0.w;
        double sn, cs;
        sincos((double)q1.x, &sn, &cs);
        const double A = s1 * s1, B = s2 * s2;
        const double l1 = sqrt(cs * cs * A + sn * sn * B);
        const double l2 = cs * sn * (A - B) / l1;
        const double l3 = fabs(s1 * s2) / l1;
        const double is = 1.0 / U_SCALE, is2 = is * is;
        const double P1 = S[3] * is, P2 = S[4] * is;
        const double Q11 = S[5] * is2, Q12 = S[6] * is2, Q22 = S[7] * is2;
        // O = L^{-1} R S
        const double o11 = cs * s1 / l1, o12 = -sn * s2 / l1;
        const double o21 = s1 * (sn * l1 - cs * l2) / (l1 * l3);
        const double o22 = s2 * (sn * l2 + cs * l1) / (l1 * l3);
        const double V11 = o11 * o11 * Q11 + 2.0 * o11 * o21 * Q12 + o21 * o21 * Q22;
        const double V22 = o12 * o12 * Q11 + 2.0 * o12 * o22 * Q12 + o22 * o22 * Q22;
        const double V12 = o11 * o12 * Q11 + (o11 * o22 + o21 * o12) * Q12 + o21 * o22 * Q22;
        g[0] = (float)((P1 - (l2 / l3) * P2) / l1);
        g[1] = (float)(P2 / l3);
        g[2] = (float)(V11 / s1);
        g[3] = (float)(V22 / s2);
        g[4] = (float)((A - B) * V12 / (s1 * s2));
    } else {
        const float l1 = q0.z, l2 = q0.w, l3 = q1.x;
        const float is = (float)(1.0 / U_SCALE);
        const float is2 = (float)(1.0 / (U_SCALE * U_SCALE));
        const float r23 = l2 / l3;
        g[0] = (S[3] - r23 * S[4]) * is / l1;
        g[1] = S[4] * is / l3;
        g[2] = (S[5] - r23 * S[6]) * is2 / l1;
        g[3] = S[6] * is2 / l3;
        g[4] = S[7] * is2 / l3;
    }
    g[5] = S[0];
    g[6] = S[1];
    g[7] = S[2];
}

template <int COV>
__global__ __launch_bounds__(UPD_T) void k_grad_out(const float4 *__restrict__ params, int64_t n,
                                                    const uint32_t *__restrict__ count,
                                                    const uint32_t *__restrict__ off,
                                                    const float4 *__restrict__ part,
                                                    const DevState *__restrict__ st, int64_t cap,
                                                    float2 *__restrict__ dparams) {
    const int64_t i = (int64_t)blockIdx.x * UPD_G + (threadIdx.x >> 2);
    const int q = threadIdx.x & 3;
    if (i >= n) return;  // whole quads leave together
    unsigned long long keys = st->keys_total;
    if (keys > (unsigned long long)cap) keys = (unsigned long long)cap;
    float g[8];
    float4 q0, q1;
    quad_grad<COV>(params, i, q, count, off, part, keys, g, q0, q1);
    dparams[4 * i + q] = make_float2(g[2 * q], g[2 * q + 1]);
}

// Gradient of the opacity renderings.  BLEND_SUM: the records carried c' = o c, so
// dL/dc = o dL/dc' and dL/do = <c, dL/dc'>; BLEND_ALPHA: the sums already hold dL/dc and dL/do.
template <int COV, int BLEND>
__global__ __launch_bounds__(UPD_T) void k_grad_opacity(const float4 *__restrict__ params,
                                                        const float *__restrict__ opacity,
                                                        int64_t n,
                                                        const uint32_t *__restrict__ count,
                                                        const uint32_t *__restrict__ off,
                                                        const float4 *__restrict__ part,
                                                        const DevState *__restrict__ st,
                                                        int64_t cap, float2 *__restrict__ dparams,
                                                        float *__restrict__ dopacity) {
    const int64_t i = (int64_t)blockIdx.x * UPD_G + (threadIdx.x >> 2);
    const int q = threadIdx.x & 3;
    if (i >= n) return;
    unsigned long long keys = st->keys_total;
    if (keys > (unsigned long long)cap) keys = (unsigned long long)cap;
    float g[8], so = 0.f;
    float4 q0, q1;
    quad_grad<COV, BLEND == BLEND_ALPHA ? 3 : 2>(params, i, q, count, off, part, keys, g, q0, q1,
                                                 BLEND == BLEND_ALPHA ? &so : nullptr);
    if (BLEND == BLEND_SUM) {
        const float o = opacity[i];
        so = fmaf(q1.w, g[7], fmaf(q1.z, g[6], q1.y * g[5]));
        g[5] *= o;
        g[6] *= o;
        g[7] *= o;
    }
    dparams[4 * i + q] = make_float2(g[2 * q], g[2 * q + 1]);
    if (q == 0) dopacity[i] = so;
}

// Adam on every Gaussian.  Bias corrections are computed once per block in float64.
// With an opacity rendering (BLEND != BLEND_NONE) lane 0 of each quad also updates the
// Gaussian's opacity (moments m_op, v_op; colour learning rate), with the gradients of
// k_grad_opacity.
template <int COV, int BLEND = BLEND_NONE>
__global__ __launch_bounds__(UPD_T) void k_adam(float4 *__restrict__ params, int64_t n,
                                                const uint32_t *__restrict__ count,
                                                const uint32_t *__restrict__ off,
                                                const float4 *__restrict__ part, DevState *st,
                                                int64_t cap, float2 *__restrict__ m2,
                                                float2 *__restrict__ v2, int32_t *step,
                                                AdamArgs hp, float *__restrict__ opacity,
                                                float *__restrict__ m_op,
                                                float *__restrict__ v_op) {
    __shared__ float s_bc[2];
    if (threadIdx.x == 0) {
        const double t = (double)*step;
        s_bc[0] = (float)(1.0 - pow((double)hp.beta1, t));
        s_bc[1] = (float)(1.0 - pow((double)hp.beta2, t));
    }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * UPD_G + (threadIdx.x >> 2);
    const int q = threadIdx.x & 3;
    // gradients incomplete on key overflow: leave the state alone
    if (i >= n || (st->flags & FLAG_KEY_OVERFLOW)) return;
    unsigned long long keys = st->keys_total;
    if (keys > (unsigned long long)cap) keys = (unsigned long long)cap;
    float g[8], so = 0.f;
    float4 q0, q1;
    quad_grad<COV, BLEND == BLEND_ALPHA ? 3 : 2>(params, i, q, count, off, part, keys, g, q0, q1,
                                                 BLEND == BLEND_ALPHA ? &so : nullptr);
    float op = 0.f;
    if (BLEND != BLEND_NONE) op = opacity[i];
    if (BLEND == BLEND_SUM) {
        so = fmaf(q1.w, g[7], fmaf(q1.z, g[6], q1.y * g[5]));
        g[5] *= op;
        g[6] *= op;
        g[7] *= op;
    }
    const float pv[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
    const float bc1 = s_bc[0], bc2 = s_bc[1];
    const float2 mo = m2[4 * i + q], vo = v2[4 * i + q];
    float p[2] = {pv[2 * q], pv[2 * q + 1]};
    float m[2] = {mo.x, mo.y}, v[2] = {vo.x, vo.y};
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const int k = 2 * q + e;
        const float lr = k < 2 ? hp.lr_mu : (k < 5 ? hp.lr_l : hp.lr_c);
        m[e] = hp.beta1 * m[e] + (1.f - hp.beta1) * g[k];
        v[e] = hp.beta2 * v[e] + (1.f - hp.beta2) * g[k] * g[k];
        const float mh = m[e] / bc1, vh = v[e] / bc2;
        p[e] -= lr * mh / (sqrtf(vh) + hp.eps);
        const bool floor = COV == COV_ROTATION_SCALE ? (k == 2 || k == 3) : (k == 2 || k == 4);
        if (floor && hp.l_min > 0.f && fabsf(p[e]) < hp.l_min)
            p[e] = copysignf(hp.l_min, p[e]);
    }
    // every lane of the quad has read the parameters it needs before any lane writes
    __builtin_amdgcn_wave_barrier();
    reinterpret_cast<float2 *>(params)[4 * i + q] = make_float2(p[0], p[1]);
    m2[4 * i + q] = make_float2(m[0], m[1]);
    v2[4 * i + q] = make_float2(v[0], v[1]);
    if (BLEND != BLEND_NONE && q == 0) {
        const float mm = hp.beta1 * m_op[i] + (1.f - hp.beta1) * so;
        const float vv = hp.beta2 * v_op[i] + (1.f - hp.beta2) * so * so;
        opacity[i] = op - hp.lr_c * (mm / bc1) / (sqrtf(vv / bc2) + hp.eps);
        m_op[i] = mm;
        v_op[i] = vv;
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

hipError_t launch_alpha_fwd(const RasterArgs &a, const float *rec_o, float *image, hipStream_t s) {
    if (a.n_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_alpha_fwd<2>, dim3((unsigned)a.n_tiles), dim3(128), 0, s,
                       reinterpret_cast<const float4 *>(a.rec), rec_o, a.ranges, a.tab, image);
    return hipGetLastError();
}

hipError_t launch_alpha_bwd(const RasterArgs &a, const float *rec_o, const float *dl,
                            float *part12, hipStream_t s) {
    if (a.n_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_alpha_bwd, dim3((unsigned)a.n_tiles), dim3(64), 0, s,
                       reinterpret_cast<const float4 *>(a.rec), rec_o, a.slot, a.ranges, a.tab,
                       dl, reinterpret_cast<float4 *>(part12));
    return hipGetLastError();
}

hipError_t launch_grad_opacity(const UpdateArgs &u, const float *opacity, int32_t blend,
                               float *dparams, float *dopacity, hipStream_t s) {
    if (u.n <= 0) return hipSuccess;
    const dim3 grid((unsigned)((u.n + UPD_G - 1) / UPD_G));
    const float4 *pin = reinterpret_cast<const float4 *>(u.params_in);
    const float4 *part = reinterpret_cast<const float4 *>(u.part);
    float2 *out = reinterpret_cast<float2 *>(dparams);
    const bool rs = u.cov == COV_ROTATION_SCALE;
#define GI_LAUNCH_GO(C, BL)                                                                     \
    hipLaunchKernelGGL((k_grad_opacity<C, BL>), grid, dim3(UPD_T), 0, s, pin, opacity, u.n,     \
                       u.count, u.off, part, u.state, u.cap, out, dopacity)
    if (blend == BLEND_ALPHA) {
        if (rs) GI_LAUNCH_GO(COV_ROTATION_SCALE, BLEND_ALPHA);
        else GI_LAUNCH_GO(COV_CHOLESKY, BLEND_ALPHA);
    } else {
        if (rs) GI_LAUNCH_GO(COV_ROTATION_SCALE, BLEND_SUM);
        else GI_LAUNCH_GO(COV_CHOLESKY, BLEND_SUM);
    }
#undef GI_LAUNCH_GO
    return hipGetLastError();
}

hipError_t launch_grad_out(const UpdateArgs &u, float *dparams, hipStream_t s) {
    if (u.n <= 0) return hipSuccess;
    const dim3 grid((unsigned)((u.n + UPD_G - 1) / UPD_G));
    const float4 *pin = reinterpret_cast<const float4 *>(u.params_in);
    const float4 *part = reinterpret_cast<const float4 *>(u.part);
    float2 *out = reinterpret_cast<float2 *>(dparams);
    if (u.cov == COV_ROTATION_SCALE)
        hipLaunchKernelGGL(k_grad_out<COV_ROTATION_SCALE>, grid, dim3(UPD_T), 0, s, pin, u.n,
                           u.count, u.off, part, u.state, u.cap, out);
    else
        hipLaunchKernelGGL(k_grad_out<COV_CHOLESKY>, grid, dim3(UPD_T), 0, s, pin, u.n, u.count,
                           u.off, part, u.state, u.cap, out);
    return hipGetLastError();
}

hipError_t launch_adam(const UpdateArgs &u, float *params, float *m, float *v, int32_t *step,
                       const AdamArgs &hp, const float *loss_part, const ImgTable &tab,
                       int64_t n_tiles, float *loss_out, hipStream_t s) {
    if (u.n > 0) {
        const dim3 grid((unsigned)((u.n + UPD_G - 1) / UPD_G));
        float4 *p4 = reinterpret_cast<float4 *>(params);
        const float4 *part = reinterpret_cast<const float4 *>(u.part);
        float2 *m2 = reinterpret_cast<float2 *>(m), *v2 = reinterpret_cast<float2 *>(v);
        float *nf = nullptr;
        if (u.cov == COV_ROTATION_SCALE)
            hipLaunchKernelGGL((k_adam<COV_ROTATION_SCALE, BLEND_NONE>), grid, dim3(UPD_T), 0, s,
                               p4, u.n, u.count, u.off, part, u.state, u.cap, m2, v2, step, hp,
                               nf, nf, nf);
        else
            hipLaunchKernelGGL((k_adam<COV_CHOLESKY, BLEND_NONE>), grid, dim3(UPD_T), 0, s, p4,
                               u.n, u.count, u.off, part, u.state, u.cap, m2, v2, step, hp, nf,
                               nf, nf);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return launch_finish(loss_part, tab, n_tiles, loss_out, step, s);
}

hipError_t launch_alpha_fit(const RasterArgs &a, const float *rec_o, const float *target,
                            float *part12, float *image_out, float *loss_part, hipStream_t s) {
    if (a.n_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_alpha_fit, dim3((unsigned)a.n_tiles), dim3(64), 0, s,
                       reinterpret_cast<const float4 *>(a.rec), rec_o, a.slot, a.ranges, a.tab,
                       target, reinterpret_cast<float4 *>(part12), image_out, loss_part);
    return hipGetLastError();
}

hipError_t launch_adam_opacity(const UpdateArgs &u, float *params, float *opacity, float *m,
                               float *v, float *mo, float *vo, int32_t *step, const AdamArgs &hp,
                               int32_t blend, const float *loss_part, const ImgTable &tab,
                               int64_t n_tiles, float *loss_out, hipStream_t s) {
    if (u.n > 0) {
        const dim3 grid((unsigned)((u.n + UPD_G - 1) / UPD_G));
        float4 *p4 = reinterpret_cast<float4 *>(params);
        const float4 *part = reinterpret_cast<const float4 *>(u.part);
        float2 *m2 = reinterpret_cast<float2 *>(m), *v2 = reinterpret_cast<float2 *>(v);
        const bool rs = u.cov == COV_ROTATION_SCALE;
#define GI_LAUNCH_AO(C, BL)                                                                     \
    hipLaunchKernelGGL((k_adam<C, BL>), grid, dim3(UPD_T), 0, s, p4, u.n, u.count, u.off, part, \
                       u.state, u.cap, m2, v2, step, hp, opacity, mo, vo)
        if (blend == BLEND_ALPHA) {
            if (rs) GI_LAUNCH_AO(COV_ROTATION_SCALE, BLEND_ALPHA);
            else GI_LAUNCH_AO(COV_CHOLESKY, BLEND_ALPHA);
        } else {
            if (rs) GI_LAUNCH_AO(COV_ROTATION_SCALE, BLEND_SUM);
            else GI_LAUNCH_AO(COV_CHOLESKY, BLEND_SUM);
        }
#undef GI_LAUNCH_AO
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
