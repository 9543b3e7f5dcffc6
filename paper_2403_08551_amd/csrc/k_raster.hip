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
// Work mapping.  Forward: one workgroup of 256 threads per 16x16 tile.  The tile's list is cut
// into four equal parts; each part is summed by one group of 256 / PX threads, each lane owning
// PX pixels of one column (so per-column terms are shared by PX pixels), the part's records
// streamed in sorted order through the wave's own LDS and read as broadcasts (every lane uses the
// same Gaussian at once), colour accumulated in float32 registers with a two-level sum (partial
// sums of 8 Gaussians).  The four part sums meet in LDS and are added in part order, so every PX
// gives the same bits.
// Adjoint: each Gaussian of the tile's list is taken by a group of 2 lanes (4, 8 or 16 in a
// short last round), each lane covering every second (fourth, ...) column; the tile's 256 dL/dC
// values are staged in LDS and read as broadcasts, each lane reduces its share of the pixels in
// registers and the group adds its lanes' sums with DPP steps: no atomics.  The eight partial
// sums of each (tile, Gaussian) pair are stored at that pair's key position and the
// per-Gaussian kernel adds them in a fixed order, which keeps gradients deterministic.
#include "gi_common.h"

namespace gi {

namespace {

constexpr int PARTS = 4;  // parts of a tile's list summed separately in the forward
constexpr int BWD_T = 256;

// ---- begin: the fused fit kernel and the device functions it calls ----
__device__ inline float ex2(float x) { return __builtin_amdgcn_exp2f(x); }

// One Gaussian's contribution to the PX pixels of this lane (A = mu_x, mu_y, a, b;
// B = k, c0, c1, c2).  The lane's pixels lie in one column and in one group of four rows
// starting at row centre py0; pixel j sits of[j] rows below it.  Every pixel's u2 is taken from
// the group's first row as fl(o b + u2(py0)) (o b is exact in the FMA), whatever PX is, so the
// forward gives the same bits for every PX; with PX = 4 the four rows share dx, u1, u1^2, k dx
// and u2(py0).
template <int PX, bool INIT = false>
__device__ inline void fwd_eval(const float4 A, const float4 B, float px, float py0,
                                const float (&of)[PX], float (&part)[PX][3]) {
    const float dx = px - A.x;
    const float u1 = A.z * dx;
    const float u1s = u1 * u1;
    const float t = B.x * dx;
    const float u2b = fmaf(py0 - A.y, A.w, -t);
#pragma unroll
    for (int j = 0; j < PX; ++j) {
        const float u2 = PX == 4 ? (j == 0 ? u2b : fmaf((float)j, A.w, u2b))
                                 : fmaf(of[j], A.w, u2b);
        const float e = ex2(-fmaf(u2, u2, u1s));
        if (INIT) {  // the first record of a partial sum sets it
            part[j][0] = B.y * e;
            part[j][1] = B.z * e;
            part[j][2] = B.w * e;
        } else {
            part[j][0] = fmaf(B.y, e, part[j][0]);
            part[j][1] = fmaf(B.z, e, part[j][1]);
            part[j][2] = fmaf(B.w, e, part[j][2]);
        }
    }
}

// Forward accumulation for the PX pixels (one column) of this thread over the list range r, the
// records reaching the VALU through LDS rather than the scalar unit: a VALU instruction that
// reads a scalar register issues at half the rate of one that reads only vector registers
// (measured on gfx950: 38 against 60-72 T lane-op/s), and the per-record arithmetic reads the
// record in every instruction.  The wave streams its list range in chunks of 32 records: one
// 16-byte load per lane (coalesced), written to the wave's own 1 KB of LDS, then each record
// read back as two broadcast 16-byte LDS reads; the next chunk's load is in flight while the
// current one is evaluated.  LDS operations of one wave complete in order, so the wave needs no
// barrier.  Two-level sum: each group of 8 records forms a partial sum (set by its first record),
// added to the totals after the group; then one group of 4 and one of the rest, so the grouping
// depends on the list alone, not on PX.  With PRIO the wave lowers its issue priority from 3 to
// 0 as it passes a quarter, a half and three quarters of its records, so the waves sharing a
// SIMD progress together instead of oldest first (which leaves each CU's last workgroup running
// alone, without a second wave to pair VALU instructions with).
template <int PX, bool PRIO = false>
__device__ __forceinline__ void fwd_tile_lds(const float4 *__restrict__ rec, uint2 r, float px,
                                             float py0, const float (&of)[PX],
                                             float (&acc)[PX][3], float4 *lbuf) {
    constexpr uint32_t CH = 32;  // records per chunk (64 lanes x 16 bytes)
    const int lane = threadIdx.x & 63;
    float part[PX][3];
#pragma unroll
    for (int j = 0; j < PX; ++j) acc[j][0] = acc[j][1] = acc[j][2] = 0.f;
    auto fold = [&]() {
#pragma unroll
        for (int j = 0; j < PX; ++j) {
            acc[j][0] += part[j][0];
            acc[j][1] += part[j][1];
            acc[j][2] += part[j][2];
        }
    };
    const uint32_t L = r.y - r.x;
    if (L == 0) return;
    // The 16-byte words of records [first, first + cnt), cnt >= 1: lane l reads word l and lanes
    // past the end read the last word again (in bounds; their LDS words are never read).  The
    // load is unconditional on purpose: a load under a lane condition had been compiled into a
    // flat load through a pointer select (a zero kept in private memory), and a flat load counts
    // against the LDS wait counter too, so every LDS wait of a chunk waited for the prefetch.
    auto chunk_word = [&](uint32_t first, uint32_t cnt) {
        const uint32_t last = 2 * cnt - 1;
        return rec[2 * (int64_t)first + ((uint32_t)lane < last ? (uint32_t)lane : last)];
    };
    float4 stage = chunk_word(r.x, L < CH ? L : CH);
    const uint32_t q1 = L >> 2, q2 = L >> 1, q3 = (L >> 2) + (L >> 1);
    if (PRIO) __builtin_amdgcn_s_setprio(3);
    for (uint32_t c0 = 0; c0 < L; c0 += CH) {
        const uint32_t n = L - c0 < CH ? L - c0 : CH;
        if (PRIO) {  // the chunk that crosses a quarter mark lowers the priority
            if (c0 >= q1 && c0 < q1 + CH) __builtin_amdgcn_s_setprio(2);
            if (c0 >= q2 && c0 < q2 + CH) __builtin_amdgcn_s_setprio(1);
            if (c0 >= q3 && c0 < q3 + CH) __builtin_amdgcn_s_setprio(0);
        }
        lbuf[lane] = stage;
        if (c0 + CH < L) stage = chunk_word(r.x + c0 + CH, L - c0 - CH < CH ? L - c0 - CH : CH);
        uint32_t k = 0;
        for (; k + 8 <= n; k += 8) {
            fwd_eval<PX, true>(lbuf[2 * k], lbuf[2 * k + 1], px, py0, of, part);
#pragma unroll
            for (uint32_t e = 1; e < 8; ++e) {
                // scheduling fence between the two halves of the group (same arithmetic): left
                // free, the compiler issues all 16 LDS reads first and clusters the exp2s, which
                // measured 1.5% slower in the fit kernel
                if (e == 4) __builtin_amdgcn_sched_barrier(0);
                fwd_eval<PX>(lbuf[2 * (k + e)], lbuf[2 * (k + e) + 1], px, py0, of, part);
            }
            fold();
        }
        if (k + 4 <= n) {
            fwd_eval<PX, true>(lbuf[2 * k], lbuf[2 * k + 1], px, py0, of, part);
#pragma unroll
            for (uint32_t e = 1; e < 4; ++e)
                fwd_eval<PX>(lbuf[2 * (k + e)], lbuf[2 * (k + e) + 1], px, py0, of, part);
            fold();
            k += 4;
        }
        if (k < n) {
            fwd_eval<PX, true>(lbuf[2 * k], lbuf[2 * k + 1], px, py0, of, part);
            for (++k; k < n; ++k) fwd_eval<PX>(lbuf[2 * k], lbuf[2 * k + 1], px, py0, of, part);
            fold();
        }
    }
}

// The LPG lanes sharing a Gaussian in the adjoint add their values: DPP quad_perm [1, 0, 3, 2]
// then [2, 3, 0, 1] (every lane of a quad then holds the quad's sum), row_half_mirror (every lane
// of a group of 8 then holds its sum), row_mirror (every lane of a row of 16 then holds its
// sum).  The order of the additions is fixed: ((v0 + v1) + (v2 + v3)) + ((v4 + v5) + (v6 + v7)),
// and so on.
template <int CTRL>
__device__ inline float dpp_mov(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
                                         0, __builtin_bit_cast(int, x), CTRL, 0xf, 0xf, false));
}

template <int LPG>
__device__ inline float group_add(float v) {
    v += dpp_mov<0xb1>(v);                 // quad_perm [1, 0, 3, 2]
    if (LPG >= 4) v += dpp_mov<0x4e>(v);   // quad_perm [2, 3, 0, 1]
    if (LPG >= 8) v += dpp_mov<0x141>(v);  // row_half_mirror
    if (LPG >= 16) v += dpp_mov<0x140>(v); // row_mirror
    return v;
}

// One round of the adjoint for this lane: Gaussian i (if act) over the tile's columns
// LPG k + par (k < 16 / LPG), all 16 rows, dL/dC of the tile in LDS.  The LPG lanes of a
// Gaussian (lanes LPG j ... LPG j + LPG - 1, neighbouring LDS words, so the broadcast reads hit
// different banks) add their sums at the end and the group's first lane stores them.
// Per pixel, with w = exp(-sigma) <dL/dC, c'>: the colour sums D += e g, then w, sum w u2 and
// sum w u2^2, each product formed per pixel (no difference of larger sums, which would lose
// the relative accuracy of a single term).  The column's sum of w is <D, c'> (the colour sums
// are needed anyway), not a per-pixel sum.
template <int LPG>
__device__ __forceinline__ void bwd_round(const float4 *__restrict__ rec,
                                          const uint32_t *__restrict__ slot, uint32_t i, bool act,
                                          int par, const TileInfo &ti, const float4 *sg,
                                          float4 *__restrict__ part) {
    const float x0 = (float)(ti.tx * TILE + par) + 0.5f;
    const float y0 = (float)(ti.ty * TILE) + 0.5f;
    float4 A = make_float4(0.f, 0.f, 0.f, 0.f), B = A;
    if (act) {
        A = rec[2 * i];
        B = rec[2 * i + 1];
    }
    float dy[TILE];
#pragma unroll
    for (int rr = 0; rr < TILE; ++rr) dy[rr] = (y0 + (float)rr) - A.y;
    float C0 = 0.f, C1 = 0.f, C2 = 0.f, P1 = 0.f, P2 = 0.f, Q11 = 0.f, Q12 = 0.f, Q22 = 0.f;
    float dx = x0 - A.x;  // this lane's column LPG k + par: dx advances by LPG per column
    for (int k = 0; k < TILE / LPG; ++k) {
        const int cc = LPG * k + par;
        const float u1 = A.z * dx;
        const float u1s = u1 * u1;
        const float t = B.x * dx;
        float D0 = 0.f, D1 = 0.f, D2 = 0.f, WU2 = 0.f, WU22 = 0.f;
#pragma unroll
        for (int rr = 0; rr < TILE; ++rr) {
            const float4 g = sg[rr * TILE + cc];
            const float u2 = fmaf(dy[rr], A.w, -t);
            const float e = ex2(-fmaf(u2, u2, u1s));
            D0 = fmaf(g.x, e, D0);
            D1 = fmaf(g.y, e, D1);
            D2 = fmaf(g.z, e, D2);
            const float gc = fmaf(g.z, B.w, fmaf(g.y, B.z, g.x * B.y));
            const float wu2 = (e * gc) * u2;  // -dL/dsigma of this pixel times u2
            WU2 += wu2;
            WU22 = fmaf(wu2, u2, WU22);
        }
        // the column's sum of w from its colour sums: sum_r e <g, c'> = <sum_r e g, c'>
        const float Wc = fmaf(B.w, D2, fmaf(B.z, D1, B.y * D0));
        C0 += D0;
        C1 += D1;
        C2 += D2;
        P1 = fmaf(u1, Wc, P1);
        Q11 = fmaf(u1s, Wc, Q11);
        Q12 = fmaf(u1, WU2, Q12);
        P2 += WU2;
        Q22 += WU22;
        dx += (float)LPG;
    }
    C0 = group_add<LPG>(C0);
    C1 = group_add<LPG>(C1);
    C2 = group_add<LPG>(C2);
    P1 = group_add<LPG>(P1);
    P2 = group_add<LPG>(P2);
    Q11 = group_add<LPG>(Q11);
    Q12 = group_add<LPG>(Q12);
    Q22 = group_add<LPG>(Q22);
    if (act && par == 0) {
        const int64_t sl = slot[i];
        part[2 * sl] = make_float4(C0, C1, C2, P1);
        part[2 * sl + 1] = make_float4(P2, Q11, Q12, Q22);
    }
}

// Adjoint of one tile by NT threads.  Rounds of NT / 2 Gaussians, two lanes per Gaussian (even
// and odd columns), wave w taking Gaussians w 32 ... w 32 + 31 of each round.  A remainder of at
// most NT / 4 Gaussians after the whole rounds takes one round with 4, 8 or 16 lanes per
// Gaussian (the fewest that keep every Gaussian in it: 4 up to NT / 4 Gaussians, 8 up to NT / 8,
// 16 up to NT / 16), each lane then covering 4, 2 or 1 columns: that round costs a half, a
// quarter or an eighth of a full one, where a full round mostly of idle lanes would cost it all
// (a list of L Gaussians otherwise pays ceil(L / (NT / 2)) full rounds).
template <int NT>
__device__ __forceinline__ void bwd_tile(const float4 *__restrict__ rec, const uint32_t *__restrict__ slot,
                                uint2 r, const TileInfo &ti, const float4 *sg,
                                float4 *__restrict__ part) {
    constexpr uint32_t FULL = NT / 2, WAVES = NT / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t L = r.y - r.x;
    const uint32_t rem = L % FULL;
    // rounds of two lanes per Gaussian: the whole ones, and the remainder when it is large
    const uint32_t end2 = r.x + (L - rem) + (rem > FULL / 2 ? rem : 0u);
    for (uint32_t c = r.x + (uint32_t)wave * 32u; c < end2; c += FULL) {
        const uint32_t i = c + (uint32_t)(lane >> 1);
        bwd_round<2>(rec, slot, i, i < end2, lane & 1, ti, sg, part);
    }
    const uint32_t left = r.y - end2;  // 0, or the remainder of at most FULL / 2
    if (left == 0) return;
    if (left > FULL / 4) {
        const uint32_t i = end2 + (uint32_t)wave * (64u / 4u) + (uint32_t)(lane >> 2);
        bwd_round<4>(rec, slot, i, i < r.y, lane & 3, ti, sg, part);
    } else if (left > FULL / 8) {
        const uint32_t i = end2 + (uint32_t)wave * (64u / 8u) + (uint32_t)(lane >> 3);
        bwd_round<8>(rec, slot, i, i < r.y, lane & 7, ti, sg, part);
    } else {
        const uint32_t i = end2 + (uint32_t)wave * (64u / 16u) + (uint32_t)(lane >> 4);
        bwd_round<16>(rec, slot, i, i < r.y, lane & 15, ti, sg, part);
    }
    static_assert(WAVES * (64 / 4) == FULL / 2 && WAVES * (64 / 16) == FULL / 8,
                  "a tail round holds the remainder it is chosen for");
}

// Part q of a tile's list: [r.x + floor(q L / PARTS), r.x + floor((q + 1) L / PARTS)).
__device__ inline uint2 list_part(uint2 r, int q) {
    const uint64_t L = r.y - r.x;
    return make_uint2(r.x + (uint32_t)(L * (uint64_t)q / PARTS),
                      r.x + (uint32_t)(L * (uint64_t)(q + 1) / PARTS));
}

// Part sums of the tile's pixels into qs[PARTS][3][TILE_PX].  PX groups of 256 / PX threads
// (whole waves) each take PARTS / PX parts in turn; lane l of a group owns the PX consecutive
// rows from (l >> 4) PX on of column l & 15.
template <int PX, bool PRIO = false>
__device__ __forceinline__ void fwd_parts(const float4 *__restrict__ rec, uint2 r,
                                          const TileInfo &ti, float *qs, float4 *lrec) {
    constexpr int GROUP = 256 / PX, PER = PARTS / PX;
    static_assert(GROUP % 64 == 0 && PARTS % PX == 0 && PX <= 4, "groups are whole waves");
    const int grp = __builtin_amdgcn_readfirstlane((int)threadIdx.x / GROUP);
    const int lt = (int)threadIdx.x % GROUP;
    const int col = lt & 15, first = (lt >> 4) * PX;
    const float px = (float)(ti.tx * TILE + col) + 0.5f;
    const float py0 = (float)(ti.ty * TILE + (first & ~3)) + 0.5f;
    float of[PX];
#pragma unroll
    for (int j = 0; j < PX; ++j) of[j] = (float)((first & 3) + j);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int q = grp * PER + k;
        float acc[PX][3];
        fwd_tile_lds<PX, PRIO>(rec, list_part(r, q), px, py0, of, acc,
                         lrec + 64 * (threadIdx.x >> 6));
#pragma unroll
        for (int j = 0; j < PX; ++j) {
            const int p = (first + j) * TILE + col;
            qs[(q * 3) * TILE_PX + p] = acc[j][0];
            qs[(q * 3 + 1) * TILE_PX + p] = acc[j][1];
            qs[(q * 3 + 2) * TILE_PX + p] = acc[j][2];
        }
    }
}

// Colour of pixel p from the part sums (after a barrier), added in part order.
__device__ inline float3 fwd_colour(const float *qs, int p) {
    float c[3];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        float v = qs[ch * TILE_PX + p];
#pragma unroll
        for (int q = 1; q < PARTS; ++q) v += qs[(q * 3 + ch) * TILE_PX + p];
        c[ch] = v;
    }
    return make_float3(c[0], c[1], c[2]);
}

template <int PX>
__global__ __launch_bounds__(256) void k_raster_fwd(const float4 *__restrict__ rec,
                                                         const uint2 *__restrict__ ranges,
                                                         ImgTable tab, float *__restrict__ image,
    const uint32_t *__restrict__ order, DevState *flag_state, uint32_t *flags_out) {
    __shared__ float qs[PARTS * 3 * TILE_PX];
    __shared__ float4 lrec[4 * 64];
    // the render's flags are final once the binning has run (this kernel raises none): one
    // thread hands them to the caller and clears them, where the caller asks for that
    if (flag_state && blockIdx.x == 0 && threadIdx.x == 0) {
        const uint32_t f = flag_state->flags;
        if (flags_out) *flags_out = f;
        flag_state->flags = 0u;
    }
    const uint32_t tile = order ? order[blockIdx.x] : blockIdx.x;
    const TileInfo ti = tile_info(tab, tile);
    fwd_parts<PX, true>(rec, ranges[tile], ti, qs, lrec);
    __syncthreads();
    const int p = threadIdx.x;
    const int x = ti.tx * TILE + (p & 15), y = ti.ty * TILE + (p >> 4);
    if (x < ti.W && y < ti.H) {
        const float3 c = fwd_colour(qs, p);
        const unsigned long long idx = (ti.pix_base + (unsigned long long)y * ti.W + x) * 3ull;
        image[idx] = c.x;
        image[idx + 1] = c.y;
        image[idx + 2] = c.z;
    }
}

__global__ __launch_bounds__(BWD_T) void k_raster_bwd(const float4 *__restrict__ rec,
                                                      const uint32_t *__restrict__ slot,
                                                      const uint2 *__restrict__ ranges,
                                                      ImgTable tab, const float *__restrict__ G,
                                                      float4 *__restrict__ part,
    const uint32_t *__restrict__ order) {
    __shared__ float4 sg[TILE_PX];
    const uint32_t tile = order ? order[blockIdx.x] : blockIdx.x;
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
// The second bound is waves per SIMD, WAVES of them.  With four (four workgroups per CU, which
// is what a timeline of the launch shows resident at the 124 VGPRs the compiler takes: 1024 of
// the 1536 tiles of 768x512 start at once) the compiler may take up to 128 VGPRs; bounded at
// five it took 94 and measured 7% slower at 768x512 / 70k (111.5 against 104 us): there the
// registers buy scheduling more than a fifth workgroup buys latency hiding.  With six (80 VGPRs)
// more tiles are in flight, which pays when the lists are short (a batch of small images), so
// both builds exist and the autotuner picks one per size class.
template <int PX, int WAVES>
__global__ __launch_bounds__(256, WAVES) void k_raster_fit(const float4 *__restrict__ rec,
                                                         const uint32_t *__restrict__ slot,
                                                         const uint2 *__restrict__ ranges,
                                                         ImgTable tab,
                                                         const float *__restrict__ target,
                                                         float4 *__restrict__ part,
                                                         float *__restrict__ image_out,
                                                         float *__restrict__ loss_part,
                                                         int32_t *__restrict__ step_inc,
    const uint32_t *__restrict__ order) {
    constexpr int NT = 256;
    __shared__ float qs[PARTS * 3 * TILE_PX];
    __shared__ float4 sg[TILE_PX];
    __shared__ float red[NT / 64];
    __shared__ float4 lrec[4 * 64];
    // Wave priority: the forward at the highest level, the adjoint at the lowest.  The arbiter
    // otherwise issues from the oldest waves first, so a workgroup that starts when another
    // finishes waited behind the older ones and then ran alone at the end of the kernel; this
    // way its forward takes the issue slots from the adjoints around it.  Same arithmetic.
    __builtin_amdgcn_s_setprio(3);
    const uint32_t tile = order ? order[blockIdx.x] : blockIdx.x;
    const TileInfo ti = tile_info(tab, tile);
    const uint2 r = ranges[tile];
    fwd_parts<PX>(rec, r, ti, qs, lrec);
    __syncthreads();
    const float scale = 2.0f / (3.0f * (float)ti.H * (float)ti.W);
    float sq = 0.f;
    {
        const int p = threadIdx.x;
        const int x = ti.tx * TILE + (p & 15), y = ti.ty * TILE + (p >> 4);
        float4 g = make_float4(0.f, 0.f, 0.f, 0.f);
        if (x < ti.W && y < ti.H) {
            const float3 c = fwd_colour(qs, p);
            const unsigned long long idx = (ti.pix_base + (unsigned long long)y * ti.W + x) * 3ull;
            const float r0 = c.x - target[idx];
            const float r1 = c.y - target[idx + 1];
            const float r2 = c.z - target[idx + 2];
            sq = fmaf(r0, r0, fmaf(r1, r1, fmaf(r2, r2, sq)));
            g = make_float4(scale * r0, scale * r1, scale * r2, 0.f);
            if (image_out) {
                image_out[idx] = c.x;
                image_out[idx + 1] = c.y;
                image_out[idx + 2] = c.z;
            }
        }
        sg[p] = g;
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
        // the step counter advances here; the update kernel that follows uses *step - 1
        if (step_inc && tile == 0) *step_inc += 1;
    }
    __builtin_amdgcn_s_setprio(0);
    bwd_tile<NT>(rec, slot, r, ti, sg, part);
}

// ---- end: the fused fit kernel and the device functions it calls ----

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

// Four parts per tile, one wave each (four pixels per lane: column lane & 15, rows
// (lane >> 4) + 4 j): each part composites its share of the list alone, from T = 1, into
// (colour, transmittance), and the parts compose in order:
// C = C_0 + T_0 (C_1 + T_1 (C_2 + T_2 C_3)).
constexpr int ALPHA_PARTS = 4;

__device__ inline int alpha_pix(int lane, int j) { return ((lane >> 4) + 4 * j) * TILE + (lane & 15); }

// Transmittance and colour in front of part q (Tb, Cb) and the total colour C of one pixel, from
// the parts' (colour, transmittance) in xs[part * TILE_PX + pixel].
__device__ inline void alpha_compose(const float4 *xs, int q, int pix, float &Tb, float (&Cb)[3],
                                     float (&C)[3]) {
    float T = 1.f, c0 = 0.f, c1 = 0.f, c2 = 0.f;
    Tb = 1.f;
    Cb[0] = Cb[1] = Cb[2] = 0.f;
#pragma unroll
    for (int p = 0; p < ALPHA_PARTS; ++p) {
        if (p == q) {
            Tb = T;
            Cb[0] = c0;
            Cb[1] = c1;
            Cb[2] = c2;
        }
        const float4 v = xs[p * TILE_PX + pix];
        c0 = fmaf(T, v.x, c0);
        c1 = fmaf(T, v.y, c1);
        c2 = fmaf(T, v.z, c2);
        T *= v.w;
    }
    C[0] = c0;
    C[1] = c1;
    C[2] = c2;
}

__global__ __launch_bounds__(256) void k_alpha_fwd(const float4 *__restrict__ rec,
                                                   const float *__restrict__ rec_o,
                                                   const uint2 *__restrict__ ranges, ImgTable tab,
                                                   float *__restrict__ image,
    const uint32_t *__restrict__ order) {
    constexpr int PX = 4;
    __shared__ float4 xs[ALPHA_PARTS * TILE_PX];
    const uint32_t tile = order ? order[blockIdx.x] : blockIdx.x;
    const TileInfo ti = tile_info(tab, tile);
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int col = lane & 15, row = lane >> 4;
    const float px = (float)(ti.tx * TILE + col) + 0.5f;
    float py[PX], T[PX], acc[PX][3];
#pragma unroll
    for (int j = 0; j < PX; ++j) py[j] = (float)(ti.ty * TILE + row + 4 * j) + 0.5f;
    alpha_forward<PX>(rec, rec_o, list_part(ranges[tile], q), px, py, acc, T);
#pragma unroll
    for (int j = 0; j < PX; ++j)
        xs[q * TILE_PX + alpha_pix(lane, j)] = make_float4(acc[j][0], acc[j][1], acc[j][2], T[j]);
    __syncthreads();
    if (q != 0) return;
    const int x = ti.tx * TILE + col;
#pragma unroll
    for (int j = 0; j < PX; ++j) {
        const int y = ti.ty * TILE + row + 4 * j;
        float Tb, Cb[3], C[3];
        alpha_compose(xs, 0, alpha_pix(lane, j), Tb, Cb, C);
        if (x < ti.W && y < ti.H) {
            const unsigned long long idx = (ti.pix_base + (unsigned long long)y * ti.W + x) * 3ull;
            image[idx] = C[0];
            image[idx + 1] = C[1];
            image[idx + 2] = C[2];
        }
    }
}

// Sum over the 64 lanes with DPP adds (no LDS traffic); the total is valid in lane 63.
template <int CTRL, int ROW_MASK = 0xf>
__device__ inline float dpp_add(float v) {
    return v + __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
                                             0, __builtin_bit_cast(int, v), CTRL, ROW_MASK, 0xf,
                                             false));
}

__device__ inline float wave_sum_to_last(float v) {
    v = dpp_add<0xb1>(v);         // quad_perm [1, 0, 3, 2]: pairs
    v = dpp_add<0x4e>(v);         // quad_perm [2, 3, 0, 1]: quads
    v = dpp_add<0x141>(v);        // row_half_mirror: eights
    v = dpp_add<0x140>(v);        // row_mirror: rows of 16
    v = dpp_add<0x142, 0xa>(v);   // row_bcast15 into rows 1 and 3
    v = dpp_add<0x143, 0xc>(v);   // row_bcast31 into rows 2 and 3: lane 63 holds the total
    return v;
}

__device__ inline float wave_sum(float v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// Adjoint walk of one part of a tile's list (one wave, four pixels per lane): T0 holds the
// transmittance and D the colour behind the part's first Gaussian on entry, g the pixels' dL/dC.
// Each Gaussian's nine sums are reduced over the wave in groups of ALPHA_GRP Gaussians: the
// lanes store their partial sums as rows of LDS (`red`, this wave's ALPHA_GRP * 9 rows of
// ALPHA_STR floats), then each lane adds up one row in lane order and stores it.  Every wave of
// the workgroup runs maxlen / ALPHA_GRP rounds (maxlen: the longest part), so the barriers are
// reached by all.
constexpr int ALPHA_GRP = 4;
constexpr int ALPHA_NV = 9;
constexpr int ALPHA_STR = 68;  // row stride: 16-byte aligned rows; lanes l, l+16, .. share banks
constexpr int ALPHA_RED = ALPHA_GRP * ALPHA_NV * ALPHA_STR;
__device__ inline void alpha_adjoint(const float4 *__restrict__ rec,
                                     const float *__restrict__ rec_o,
                                     const uint32_t *__restrict__ slot, uint2 r, uint32_t maxlen,
                                     float px, const float (&py)[4], const float (&T0)[4],
                                     float (&D)[4][3], const float (&g)[4][3],
                                     float4 *__restrict__ part, float *red) {
    constexpr int PX = 4;
    const int lane = threadIdx.x & 63;
    float T[PX];
#pragma unroll
    for (int j = 0; j < PX; ++j) T[j] = T0[j];
    const uint32_t len = r.y - r.x;
    for (uint32_t o = 0; o < maxlen; o += ALPHA_GRP) {
        const uint32_t i0 = r.x + o;
        const uint32_t ng = o >= len ? 0u : (len - o < (uint32_t)ALPHA_GRP ? len - o : (uint32_t)ALPHA_GRP);
        for (uint32_t k = 0; k < ng; ++k) {
            const uint32_t i = i0 + k;
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
            // rows in the order of the stored sums: C0 C1 C2 P1 | P2 Q11 Q12 Q22 | SO
            float *row = red + (int)k * ALPHA_NV * ALPHA_STR + lane;
            row[0 * ALPHA_STR] = C0;
            row[1 * ALPHA_STR] = C1;
            row[2 * ALPHA_STR] = C2;
            row[3 * ALPHA_STR] = u1 * W;
            row[4 * ALPHA_STR] = WU2;
            row[5 * ALPHA_STR] = u1s * W;
            row[6 * ALPHA_STR] = u1 * WU2;
            row[7 * ALPHA_STR] = WU22;
            row[8 * ALPHA_STR] = SO;
        }
        __syncthreads();  // one wave: the rows are in LDS
        for (uint32_t rw = lane; rw < ng * ALPHA_NV; rw += 64) {
            const float4 *q = reinterpret_cast<const float4 *>(red + rw * ALPHA_STR);
            float acc = 0.f;
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                const float4 v = q[c];
                acc += v.x;
                acc += v.y;
                acc += v.z;
                acc += v.w;
            }
            const uint32_t k = rw / ALPHA_NV, v = rw - k * ALPHA_NV;
            const int64_t sl = slot[i0 + k];
            reinterpret_cast<float *>(part)[12 * sl + v] = acc;
        }
        __syncthreads();  // the rows are read before the next group writes them
    }
}

// Four waves per tile (parts of the list), 4 pixels per lane.  The parts' (colour,
// transmittance) meet in LDS (`red` holds them first, then each wave's reduction rows).
__global__ __launch_bounds__(256) void k_alpha_bwd(const float4 *__restrict__ rec,
                                                   const float *__restrict__ rec_o,
                                                   const uint32_t *__restrict__ slot,
                                                   const uint2 *__restrict__ ranges, ImgTable tab,
                                                   const float *__restrict__ G,
                                                   float4 *__restrict__ part,
    const uint32_t *__restrict__ order) {
    constexpr int PX = 4;
    __shared__ __align__(16) float red[ALPHA_PARTS * ALPHA_RED];
    static_assert(ALPHA_PARTS * ALPHA_RED >= 4 * ALPHA_PARTS * TILE_PX, "the part sums fit");
    float4 *xs = reinterpret_cast<float4 *>(red);
    // forward at wave priority 3, adjoint at 0 (as in k_raster_fit)
    __builtin_amdgcn_s_setprio(3);
    const uint32_t tile = order ? order[blockIdx.x] : blockIdx.x;
    const TileInfo ti = tile_info(tab, tile);
    const uint2 r = ranges[tile];
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int col = lane & 15, row = lane >> 4;
    const int x = ti.tx * TILE + col;
    const float px = (float)x + 0.5f;
    const uint2 rq = list_part(r, q);
    float py[PX], T[PX], D[PX][3], g[PX][3];
#pragma unroll
    for (int j = 0; j < PX; ++j) {
        const int y = ti.ty * TILE + row + 4 * j;
        py[j] = (float)y + 0.5f;
        g[j][0] = g[j][1] = g[j][2] = 0.f;
        if (x < ti.W && y < ti.H) {
            const unsigned long long idx = (ti.pix_base + (unsigned long long)y * ti.W + x) * 3ull;
            g[j][0] = G[idx];
            g[j][1] = G[idx + 1];
            g[j][2] = G[idx + 2];
        }
    }
    alpha_forward<PX>(rec, rec_o, rq, px, py, D, T);
#pragma unroll
    for (int j = 0; j < PX; ++j)
        xs[q * TILE_PX + alpha_pix(lane, j)] = make_float4(D[j][0], D[j][1], D[j][2], T[j]);
    __syncthreads();
    float Tb[PX];
#pragma unroll
    for (int j = 0; j < PX; ++j) {
        float Cb[3], C[3];
        alpha_compose(xs, q, alpha_pix(lane, j), Tb[j], Cb, C);
#pragma unroll
        for (int c = 0; c < 3; ++c) D[j][c] = C[c] - Cb[c];  // colour behind the part's start
    }
    __syncthreads();  // xs is read before the reduction rows overwrite it
    __builtin_amdgcn_s_setprio(0);
    alpha_adjoint(rec, rec_o, slot, rq, (r.y - r.x + ALPHA_PARTS - 1) / ALPHA_PARTS, px, py, Tb,
                  D, g, part, red + q * ALPHA_RED);
}

// Fit step of one tile with alpha blending: the parts' forward, their composition, residual,
// dL/dC = 2 (C - T) / (3 H W) in registers, per-tile sum of squared residuals (first wave), then
// each part's adjoint walk.
__global__ __launch_bounds__(256) void k_alpha_fit(const float4 *__restrict__ rec,
                                                   const float *__restrict__ rec_o,
                                                   const uint32_t *__restrict__ slot,
                                                   const uint2 *__restrict__ ranges, ImgTable tab,
                                                   const float *__restrict__ target,
                                                   float4 *__restrict__ part,
                                                   float *__restrict__ image_out,
                                                   float *__restrict__ loss_part,
                                                   int32_t *__restrict__ step_inc,
    const uint32_t *__restrict__ order) {
    constexpr int PX = 4;
    __shared__ __align__(16) float red[ALPHA_PARTS * ALPHA_RED];
    static_assert(ALPHA_PARTS * ALPHA_RED >= 4 * ALPHA_PARTS * TILE_PX, "the part sums fit");
    float4 *xs = reinterpret_cast<float4 *>(red);
    // forward at wave priority 3, adjoint at 0 (as in k_raster_fit)
    __builtin_amdgcn_s_setprio(3);
    const uint32_t tile = order ? order[blockIdx.x] : blockIdx.x;
    const TileInfo ti = tile_info(tab, tile);
    const uint2 r = ranges[tile];
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int col = lane & 15, row = lane >> 4;
    const int x = ti.tx * TILE + col;
    const float px = (float)x + 0.5f;
    const uint2 rq = list_part(r, q);
    float py[PX], T[PX], D[PX][3], g[PX][3];
#pragma unroll
    for (int j = 0; j < PX; ++j) py[j] = (float)(ti.ty * TILE + row + 4 * j) + 0.5f;
    alpha_forward<PX>(rec, rec_o, rq, px, py, D, T);
#pragma unroll
    for (int j = 0; j < PX; ++j)
        xs[q * TILE_PX + alpha_pix(lane, j)] = make_float4(D[j][0], D[j][1], D[j][2], T[j]);
    __syncthreads();
    const float scale = 2.0f / (3.0f * (float)ti.H * (float)ti.W);
    float sq = 0.f, Tb[PX];
#pragma unroll
    for (int j = 0; j < PX; ++j) {
        float Cb[3], C[3];
        alpha_compose(xs, q, alpha_pix(lane, j), Tb[j], Cb, C);
        const int y = ti.ty * TILE + row + 4 * j;
        g[j][0] = g[j][1] = g[j][2] = 0.f;
        if (x < ti.W && y < ti.H) {
            const unsigned long long idx = (ti.pix_base + (unsigned long long)y * ti.W + x) * 3ull;
            const float r0 = C[0] - target[idx];
            const float r1 = C[1] - target[idx + 1];
            const float r2 = C[2] - target[idx + 2];
            sq = fmaf(r0, r0, fmaf(r1, r1, fmaf(r2, r2, sq)));
            g[j][0] = scale * r0;
            g[j][1] = scale * r1;
            g[j][2] = scale * r2;
            if (image_out && q == 0) {
                image_out[idx] = C[0];
                image_out[idx + 1] = C[1];
                image_out[idx + 2] = C[2];
            }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) D[j][c] = C[c] - Cb[c];  // colour behind the part's start
    }
    if (q == 0) {
        sq = wave_sum(sq);
        if (lane == 0) {
            loss_part[tile] = sq;
            if (step_inc && tile == 0) *step_inc += 1;
        }
    }
    __syncthreads();  // xs is read before the reduction rows overwrite it
    __builtin_amdgcn_s_setprio(0);
    alpha_adjoint(rec, rec_o, slot, rq, (r.y - r.x + ALPHA_PARTS - 1) / ALPHA_PARTS, px, py, Tb,
                  D, g, part, red + q * ALPHA_RED);
}

// Per-image mean of the squared residuals from the per-tile sums (float64 accumulation): blocks
// take images blockIdx.x, blockIdx.x + gridDim.x, ...  256 threads; call from all of them.
__device__ inline void block_image_losses(const float *__restrict__ loss_part, const ImgTable &tab,
                                          int64_t n_tiles, float *__restrict__ loss_out,
                                          double *red, int first = -1, int stride = -1) {
    if (first < 0) first = blockIdx.x;
    if (stride < 0) stride = gridDim.x;
    for (int b = first; b < tab.B; b += stride) {
        uint32_t t0 = 0, t1 = (uint32_t)n_tiles;
        double npx;
        if (tab.B == 1) {
            npx = (double)tab.H * tab.W;
        } else {
            t0 = tab.tile_base[b];
            t1 = tab.tile_base[b + 1];
            npx = (double)tab.dims[b].x * tab.dims[b].y;
        }
        // eight reads issued before any is added (the additions keep the order of a plain
        // strided loop; lanes past the end read the last entry and drop it)
        double s = 0.0;
        for (uint32_t t = t0 + threadIdx.x; t < t1; t += 256 * 8) {
            float v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const uint32_t u = t + 256u * k;
                v[k] = loss_part[u < t1 ? u : t1 - 1];
            }
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (t + 256u * k < t1) s += (double)v[k];
        }
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
        __syncthreads();  // red is free
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0)
            loss_out[b] = (float)((red[0] + red[1] + red[2] + red[3]) / (3.0 * npx));
    }
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

template <int COV, int NV = 2, bool RECIPE = false>
__device__ inline void quad_grad(const float4 *__restrict__ params, int64_t i, int q,
                                 const uint32_t *__restrict__ count,
                                 const uint32_t *__restrict__ off,
                                 const float4 *__restrict__ part, unsigned long long keys,
                                 float (&g)[8], float4 &q0, float4 &q1, float *extra = nullptr,
                                 const float *at = nullptr) {
    constexpr int NS = NV == 3 ? 9 : 8;  // sums per key: 8, or 9 with the opacity sum
    q0 = params[2 * i];
    q1 = params[2 * i + 1];
    const uint32_t cnt = count[i];
    const uint32_t o = off[i];
    float S[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) S[k] = 0.f;
    if (cnt && (unsigned long long)o + cnt <= keys) {
        // two keys per step, both read before either is added (same order of additions)
        const uint32_t end = o + cnt;
        for (uint32_t j = o + (uint32_t)q; j < end; j += 8) {
            const bool two = j + 4 < end;
            const int64_t j2 = two ? j + 4 : j;
            const float4 a = part[NV * (int64_t)j], b = part[NV * (int64_t)j + 1];
            const float4 a2 = part[NV * j2], b2 = part[NV * j2 + 1];
            float x = 0.f, x2 = 0.f;
            if constexpr (NV == 3) {
                x = part[NV * (int64_t)j + 2].x;
                x2 = part[NV * j2 + 2].x;
            }
            S[0] += a.x; S[1] += a.y; S[2] += a.z; S[3] += a.w;
            S[4] += b.x; S[5] += b.y; S[6] += b.z; S[7] += b.w;
            if constexpr (NV == 3) S[8] += x;
            // the second key by a multiply with 1 or 0 (exact either way), not a branch that the
            // compiler would sink the reads into
            const float w2 = two ? 1.f : 0.f;
            S[0] = fmaf(a2.x, w2, S[0]); S[1] = fmaf(a2.y, w2, S[1]);
            S[2] = fmaf(a2.z, w2, S[2]); S[3] = fmaf(a2.w, w2, S[3]);
            S[4] = fmaf(b2.x, w2, S[4]); S[5] = fmaf(b2.y, w2, S[5]);
            S[6] = fmaf(b2.z, w2, S[6]); S[7] = fmaf(b2.w, w2, S[7]);
            if constexpr (NV == 3) S[8] = fmaf(x2, w2, S[8]);
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
    // the chain rule runs at the record that was rendered: the effective record of the recipe
    // (raw + 0.5 on the diagonal / scales), or the slots given in `at` (fake-quantised values)
    const float e2 = at ? at[0] : (RECIPE ? q0.z + 0.5f : q0.z);
    const float e3 = at ? at[1] : (RECIPE && COV == COV_ROTATION_SCALE ? q0.w + 0.5f : q0.w);
    const float e4 = at ? at[2] : (RECIPE && COV != COV_ROTATION_SCALE ? q1.x + 0.5f : q1.x);
    if (COV == COV_ROTATION_SCALE) {
        const double s1 = e2, s2 = e3;
        double sn, cs;
        sincos((double)e4, &sn, &cs);
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
        const float l1 = e2, l2 = e3, l3 = e4;
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
// Longest list first: each tile goes to the bin of its list length (descending), the bins'
// starts come from one exclusive scan in LDS, and each tile takes the next place of its bin
// (an LDS atomic: within a bin the order is arbitrary, which only changes the dispatch order).
template <int NTH>
__device__ inline void tile_order_block(const uint2 *__restrict__ ranges, int64_t T,
                                        uint32_t *__restrict__ order, uint32_t *bin,
                                        uint32_t *wsum) {
    static_assert(TILE_ORDER_BINS % NTH == 0 && NTH % 64 == 0, "bins split evenly over waves");
    for (int b = threadIdx.x; b < TILE_ORDER_BINS; b += NTH) bin[b] = 0u;
    __syncthreads();
    auto key = [&](int64_t t) {
        const uint2 r = ranges[t];
        const uint32_t len = r.y - r.x;
        return (uint32_t)(TILE_ORDER_BINS - 1) - (len < (uint32_t)(TILE_ORDER_BINS - 1)
                                                      ? len : (uint32_t)(TILE_ORDER_BINS - 1));
    };
    for (int64_t t = threadIdx.x; t < T; t += NTH) atomicAdd(&bin[key(t)], 1u);
    __syncthreads();
    // exclusive scan of the bins: each thread owns TILE_ORDER_BINS / NTH consecutive bins
    constexpr int PER = TILE_ORDER_BINS / NTH;
    uint32_t v[PER], run = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        v[j] = bin[threadIdx.x * PER + j];
        run += v[j];
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t inc = run;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_up(inc, d, 64);
        if (lane >= d) inc += o;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    uint32_t base = 0;
    for (int w = 0; w < wave; ++w) base += wsum[w];
    uint32_t at = base + inc - run;
    __syncthreads();  // every bin has been read
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        bin[threadIdx.x * PER + j] = at;
        at += v[j];
    }
    __syncthreads();
    for (int64_t t = threadIdx.x; t < T; t += NTH)
        order[atomicAdd(&bin[key(t)], 1u)] = (uint32_t)t;
}

// With ORDER, block 0 writes the longest-first tile order of this step's lists into `order`
// (for the next step's raster kernels, which any permutation of the tiles serves equally) and
// the update runs in blocks 1, 2, ...; the order block starts with the first and ends long
// before the last, so the order costs no launch and no time on the critical path.
template <int COV, int BLEND = BLEND_NONE, bool ORDER = false>
__global__ __launch_bounds__(UPD_T) void k_adam(float4 *__restrict__ params, int64_t n,
                                                const uint32_t *__restrict__ count,
                                                const uint32_t *__restrict__ off,
                                                const float4 *__restrict__ part, DevState *st,
                                                int64_t cap, float2 *__restrict__ m2,
                                                float2 *__restrict__ v2, int32_t *step,
                                                AdamArgs hp, float *__restrict__ opacity,
                                                float *__restrict__ m_op,
                                                float *__restrict__ v_op,
                                                const float *__restrict__ loss_part,
                                                ImgTable tab, int64_t n_tiles,
                                                float *__restrict__ loss_out,
                                                const uint2 *__restrict__ ranges = nullptr,
                                                uint32_t *__restrict__ order = nullptr) {
    __shared__ float s_bc[2];
    __shared__ double red[4];
    if constexpr (ORDER) {
        __shared__ uint32_t obin[TILE_ORDER_BINS];
        __shared__ uint32_t owsum[UPD_T / 64];
        if (blockIdx.x == 0) {
            tile_order_block<UPD_T>(ranges, n_tiles, order, obin, owsum);
            return;
        }
    }
    const int bx = (int)blockIdx.x - (ORDER ? 1 : 0), nbx = (int)gridDim.x - (ORDER ? 1 : 0);
    if (loss_out) block_image_losses(loss_part, tab, n_tiles, loss_out, red, bx, nbx);
    if (threadIdx.x == 0) {
        const double t = (double)(*step - 1);  // the fit kernel has advanced the counter
        s_bc[0] = (float)(1.0 - pow((double)hp.beta1, t));
        s_bc[1] = (float)(1.0 - pow((double)hp.beta2, t));
    }
    // The sums do not need the bias corrections: they are read while thread 0 forms them, and
    // the barrier comes only before the update.
    const int64_t i = (int64_t)bx * UPD_G + (threadIdx.x >> 2);
    const int q = threadIdx.x & 3;
    // the moments and the overflow flag are read along with the sums (the reads stay within
    // the key buffers either way); gradients incomplete on key overflow: the state is left alone
    bool overflow = true;
    float2 mo, vo;
    float g[8], so = 0.f;
    float4 q0, q1;
    if (i < n) {
        overflow = (st->flags & FLAG_KEY_OVERFLOW) != 0;
        mo = m2[4 * i + q];
        vo = v2[4 * i + q];
        unsigned long long keys = st->keys_total;
        if (keys > (unsigned long long)cap) keys = (unsigned long long)cap;
        quad_grad<COV, BLEND == BLEND_ALPHA ? 3 : 2>(params, i, q, count, off, part, keys, g, q0,
                                                     q1, BLEND == BLEND_ALPHA ? &so : nullptr);
    }
    __syncthreads();  // s_bc
    if (i >= n || overflow) return;
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

// The fitting recipe's step on the raw records (App. C, Sec. 4.1): gradients at the effective
// record, the position chain factor extent / 2 (1 - tanh(rho)^2), then Adan with the learning
// rate halved every `halve_every` steps; on the first step the previous gradient is the current
// one.  Bias corrections and the rate are formed once per block in float64.
template <int COV>
__global__ __launch_bounds__(UPD_T) void k_adan(float4 *__restrict__ raw, int64_t n,
                                                const uint32_t *__restrict__ count,
                                                const uint32_t *__restrict__ off,
                                                const float4 *__restrict__ part, DevState *st,
                                                int64_t cap, float2 *__restrict__ state,
                                                const int32_t *__restrict__ step, AdanArgs hp,
                                                ImgTable tab, const float *__restrict__ loss_part,
                                                int64_t n_tiles, float *__restrict__ loss_out) {
    __shared__ float s_c[4];
    __shared__ double red[4];
    if (loss_out) block_image_losses(loss_part, tab, n_tiles, loss_out, red);
    const int32_t k = *step - 1;  // the fit kernel has advanced the counter
    if (threadIdx.x == 0) {
        const double lr = hp.halve_every > 0
                              ? (double)hp.lr * exp2(-(double)((k - 1) / hp.halve_every))
                              : (double)hp.lr;
        s_c[0] = (float)(1.0 - pow((double)hp.beta1, (double)k));
        s_c[1] = (float)(1.0 - pow((double)hp.beta2, (double)k));
        s_c[2] = (float)(1.0 - pow((double)hp.beta3, (double)k));
        s_c[3] = (float)lr;
    }
    // the sums and the state are read while thread 0 forms the constants (as in k_adam)
    const int64_t i = (int64_t)blockIdx.x * UPD_G + (threadIdx.x >> 2);
    const int q = threadIdx.x & 3;
    const int64_t stride = 4 * n;  // float2 entries per state array
    float2 *m2 = state, *v2 = state + stride, *n2 = state + 2 * stride, *p2 = state + 3 * stride;
    bool overflow = true;
    float g[8];
    float4 q0, q1;
    float2 mo, vo, no, go;
    if (i < n) {
        overflow = (st->flags & FLAG_KEY_OVERFLOW) != 0;
        mo = m2[4 * i + q];
        vo = v2[4 * i + q];
        no = n2[4 * i + q];
        go = p2[4 * i + q];
        unsigned long long keys = st->keys_total;
        if (keys > (unsigned long long)cap) keys = (unsigned long long)cap;
        quad_grad<COV, 2, true>(raw, i, q, count, off, part, keys, g, q0, q1);
    }
    __syncthreads();  // s_c
    if (i >= n || overflow) return;
    int32_t H = tab.H, W = tab.W;
    if (tab.B > 1) {
        const int4 d = tab.dims[upper_index(tab.gauss_off, tab.B, (uint32_t)i)];
        H = d.x;
        W = d.y;
    }
    const float tx = tanhf(q0.x), ty = tanhf(q0.y);
    g[0] *= 0.5f * (float)W * (1.f - tx * tx);
    g[1] *= 0.5f * (float)H * (1.f - ty * ty);
    const float pv[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
    const float bc1 = s_c[0], bc2 = s_c[1], bc3 = s_c[2], lr = s_c[3];
    float p[2] = {pv[2 * q], pv[2 * q + 1]};
    float m[2] = {mo.x, mo.y}, v[2] = {vo.x, vo.y}, nn[2] = {no.x, no.y};
    const float gprev[2] = {go.x, go.y};
    float gk[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        gk[e] = g[2 * q + e];
        const float diff = k == 1 ? 0.f : gk[e] - gprev[e];
        m[e] = hp.beta1 * m[e] + (1.f - hp.beta1) * gk[e];
        v[e] = hp.beta2 * v[e] + (1.f - hp.beta2) * diff;
        const float t = fmaf(hp.beta2, diff, gk[e]);
        nn[e] = hp.beta3 * nn[e] + (1.f - hp.beta3) * t * t;
        const float upd = (m[e] / bc1 + hp.beta2 * v[e] / bc2) / (sqrtf(nn[e] / bc3) + hp.eps);
        p[e] = (p[e] - lr * upd) / (1.f + lr * hp.weight_decay);
    }
    // every lane of the quad has read the record before any lane writes
    __builtin_amdgcn_wave_barrier();
    reinterpret_cast<float2 *>(raw)[4 * i + q] = make_float2(p[0], p[1]);
    m2[4 * i + q] = make_float2(m[0], m[1]);
    v2[4 * i + q] = make_float2(v[0], v[1]);
    n2[4 * i + q] = make_float2(nn[0], nn[1]);
    p2[4 * i + q] = make_float2(gk[0], gk[1]);
}

// Quantisation-aware fine-tuning (Sec. 3.3, Sec. 3.4): the Gaussians' Adam step with
// straight-through gradients of the fake-quantised record, and per-block sums for the
// quantiser: the LSQ+ terms of gamma and beta and the commitment sum |C[i] - r|^2 (float), and
// per codebook entry the number of Gaussians that chose it and the sum of their residuals
// before its stage (float64), for the moving average.  Per-Gaussian terms go through LDS and
// are added in Gaussian order, so the sums do not depend on scheduling.  qpart: float sums
// [QAT_FSUMS][gridDim.x], then (8-byte aligned) float64 sums [4 M B][gridDim.x], entry-major
// so that the quantiser kernel reads each entry's block sums contiguously.
constexpr int QAT_FSUMS = 7;  // 6 LSQ terms, the commitment sum

__host__ __device__ constexpr int64_t qat_dsum_offset(int64_t blocks) {
    return (QAT_FSUMS * blocks + 1) & ~(int64_t)1;  // in floats, rounded up to a double
}

template <int COV>
__global__ __launch_bounds__(UPD_T) void k_qat_adam(float4 *__restrict__ params, int64_t n,
                                                    const uint32_t *__restrict__ count,
                                                    const uint32_t *__restrict__ off,
                                                    const float4 *__restrict__ part,
                                                    DevState *st, int64_t cap,
                                                    float2 *__restrict__ m2,
                                                    float2 *__restrict__ v2,
                                                    const int32_t *__restrict__ step, AdamArgs hp,
                                                    QatArgs qa, float *__restrict__ qpart,
                                                    const float *__restrict__ loss_part,
                                                    ImgTable tab, int64_t n_tiles,
                                                    float *__restrict__ loss_out) {
#pragma clang fp contract(off)
    __shared__ float s_bc[2];
    __shared__ double red[4];
    __shared__ float rows[UPD_G][QAT_FSUMS];
    __shared__ double res[UPD_G][QAT_MAX_STAGES][3];
    __shared__ int32_t sidx[UPD_G][QAT_MAX_STAGES];
    __shared__ float s_quant[6 + 3 * QAT_MAX_ENTRIES];  // gamma, beta and the codebooks
    if (loss_out) block_image_losses(loss_part, tab, n_tiles, loss_out, red);
    // the quantiser is read from LDS by every Gaussian's search (one global read each here)
    const int nq = 6 + 3 * qa.stages * qa.size;
    for (int t = threadIdx.x; t < nq; t += UPD_T) s_quant[t] = qa.quant[t];
    QatArgs ql = qa;
    ql.quant = s_quant;
    if (threadIdx.x == 0) {
        const double t = (double)(*step - 1);  // the fit kernel has advanced the counter
        s_bc[0] = (float)(1.0 - pow((double)hp.beta1, t));
        s_bc[1] = (float)(1.0 - pow((double)hp.beta2, t));
    }
    const int gl = threadIdx.x >> 2;  // Gaussian of this quad within the block
    const int64_t i = (int64_t)blockIdx.x * UPD_G + gl;
    const int q = threadIdx.x & 3;
    const bool live = i < n && !(st->flags & FLAG_KEY_OVERFLOW);
    if (q == 0) {
        for (int k = 0; k < QAT_FSUMS; ++k) rows[gl][k] = 0.f;
        for (int m = 0; m < QAT_MAX_STAGES; ++m) sidx[gl][m] = -1;
    }
    __syncthreads();
    if (live) {
        unsigned long long keys = st->keys_total;
        if (keys > (unsigned long long)cap) keys = (unsigned long long)cap;
        const float4 a = params[2 * i], b = params[2 * i + 1];
        float rq[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
        QuantFacts f;
        qat_fake_quant(rq, ql, &f);
        float g[8];
        float4 q0, q1;
        quad_grad<COV>(params, i, q, count, off, part, keys, g, q0, q1, nullptr, rq + 2);
        const double top = (double)((1 << qa.bits) - 1);
        bool inside[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) inside[k] = f.x[k] >= 0.0 && f.x[k] <= top;
        if (q == 0) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double dg = inside[k] ? f.code[k] - f.x[k] : (f.x[k] > top ? top : 0.0);
                rows[gl][k] = (float)((double)g[2 + k] * dg);
                rows[gl][3 + k] = inside[k] ? 0.f : g[2 + k];
            }
            // the residual before each stage and the chosen entry
            double r0 = b.y, r1 = b.z, r2 = b.w;  // the float colour
            double lc = 0.0;
            const float *books = ql.quant + 6;
#pragma unroll
            for (int m = 0; m < QAT_MAX_STAGES; ++m) {
                if (m >= qa.stages) break;
                const float *e = books + ((int64_t)m * qa.size + f.idx[m]) * 3;
                res[gl][m][0] = r0;
                res[gl][m][1] = r1;
                res[gl][m][2] = r2;
                sidx[gl][m] = f.idx[m];
                const double d0 = (double)e[0] - r0, d1 = (double)e[1] - r1;
                const double d2 = (double)e[2] - r2;
                lc += (d0 * d0 + d1 * d1) + d2 * d2;
                r0 -= (double)e[0];
                r1 -= (double)e[1];
                r2 -= (double)e[2];
            }
            rows[gl][6] = (float)lc;
        }
        // straight-through: covariance slots pass the gradient only inside the code range
#pragma unroll
        for (int k = 0; k < 3; ++k)
            if (!inside[k]) g[2 + k] = 0.f;
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
            p[e] -= lr * (m[e] / bc1) / (sqrtf(v[e] / bc2) + hp.eps);
            const bool floor = COV == COV_ROTATION_SCALE ? (k == 2 || k == 3) : (k == 2 || k == 4);
            if (floor && hp.l_min > 0.f && fabsf(p[e]) < hp.l_min)
                p[e] = copysignf(hp.l_min, p[e]);
        }
        __builtin_amdgcn_wave_barrier();
        reinterpret_cast<float2 *>(params)[4 * i + q] = make_float2(p[0], p[1]);
        m2[4 * i + q] = make_float2(m[0], m[1]);
        v2[4 * i + q] = make_float2(v[0], v[1]);
    }
    __syncthreads();
    // block sums in Gaussian order: LSQ terms and the commitment sum (float), then per codebook
    // entry the count and the residual sum (float64)
    const int64_t blocks = gridDim.x;
    double *dpart = reinterpret_cast<double *>(qpart + qat_dsum_offset(blocks));
    const int nd = 4 * qa.stages * qa.size;
    for (int t = threadIdx.x; t < QAT_FSUMS + nd; t += UPD_T) {
        if (t < QAT_FSUMS) {
            float acc = 0.f;
            for (int j = 0; j < UPD_G; ++j) acc += rows[j][t];
            qpart[(int64_t)t * blocks + blockIdx.x] = acc;
        } else {
            const int e = (t - QAT_FSUMS) >> 2, ch = (t - QAT_FSUMS) & 3;
            const int m = e / qa.size, k = e % qa.size, chr = ch < 3 ? ch : 0;
            // every term is read (no load waits on a comparison) and a Gaussian that chose
            // another entry adds -0.0, which leaves any sum unchanged
            double acc = 0.0;
#pragma unroll 16
            for (int j = 0; j < UPD_G; ++j) {
                const double r = ch < 3 ? res[j][m][chr] : 1.0;
                acc += sidx[j][m] == k ? r : -0.0;
            }
            dpart[(int64_t)(t - QAT_FSUMS) * blocks + blockIdx.x] = acc;
        }
    }
}

// The quantiser's step.  Block t < 6 takes gamma or beta (t) and its Adam step with rate lr_q;
// block 6 + e takes codebook entry e = m B + j and its moving average: count <- d count +
// (1 - d) n_j, sum <- d sum + (1 - d) s_j, entry = sum / count while the count is positive
// (float64 arithmetic, each result rounded once to float32); the last block adds lambda L_c
// to the loss.  Threads add the block sums in a fixed strided order (float64) and a fixed tree
// joins them, so the result does not depend on scheduling.
__global__ __launch_bounds__(256) void k_qat_quant_update(float *__restrict__ quant,
                                                          float *__restrict__ qm,
                                                          float *__restrict__ qv,
                                                          float *__restrict__ ema, float decay,
                                                          const float *__restrict__ qpart,
                                                          int64_t blocks, int64_t n, QatArgs qa,
                                                          float lambda, float lr_q, AdamArgs hp,
                                                          const int32_t *__restrict__ step,
                                                          const DevState *__restrict__ st,
                                                          float *__restrict__ loss_out) {
#pragma clang fp contract(off)
    if (st->flags & FLAG_KEY_OVERFLOW) return;  // the Gaussians were not updated either
    const int entries = qa.stages * qa.size;
    const int t = blockIdx.x;  // 0 .. 6 + entries
    const double *dpart = reinterpret_cast<const double *>(qpart + qat_dsum_offset(blocks));
    __shared__ double red[4][4];
    const int nv = (t >= 6 && t < 6 + entries) ? 4 : 1;
    // each value's strided thread sums and shuffle tree; an entry's four values side by side,
    // so that their reads are in flight together
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    if (nv == 4) {
        const double *src = dpart + (int64_t)(4 * (t - 6)) * blocks;
        for (int64_t b = threadIdx.x; b < blocks; b += 256) {
#pragma unroll
            for (int c = 0; c < 4; ++c) s[c] += src[c * blocks + b];
        }
    } else {
        const int row = t < 6 ? t : 6;  // the commitment sum after the six LSQ terms
        const float *src = qpart + (int64_t)row * blocks;
        for (int64_t b = threadIdx.x; b < blocks; b += 256) s[0] += (double)src[b];
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
#pragma unroll
        for (int c = 0; c < 4; ++c) s[c] += __shfl_xor(s[c], d, 64);
    }
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int c = 0; c < 4; ++c) red[c][threadIdx.x >> 6] = s[c];
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double tot[4];
    for (int c = 0; c < nv; ++c) tot[c] = (red[c][0] + red[c][1]) + (red[c][2] + red[c][3]);
    if (t < 6) {
        const double t_step = (double)(*step - 1);
        const float g = (float)tot[0];
        const float bc1 = (float)(1.0 - pow((double)hp.beta1, t_step));
        const float bc2 = (float)(1.0 - pow((double)hp.beta2, t_step));
        const float m = hp.beta1 * qm[t] + (1.f - hp.beta1) * g;
        const float v = hp.beta2 * qv[t] + (1.f - hp.beta2) * g * g;
        quant[t] -= lr_q * (m / bc1) / (sqrtf(v / bc2) + hp.eps);
        qm[t] = m;
        qv[t] = v;
    } else if (t < 6 + entries) {
        const int e = t - 6;
        const double d = (double)decay;
        float *es = ema + 4 * (int64_t)e;
        const float cnt = (float)(d * (double)es[0] + (1.0 - d) * tot[3]);
        float sum[3];
        for (int c = 0; c < 3; ++c) sum[c] = (float)(d * (double)es[1 + c] + (1.0 - d) * tot[c]);
        es[0] = cnt;
        for (int c = 0; c < 3; ++c) es[1 + c] = sum[c];
        if (cnt > 0.f)
            for (int c = 0; c < 3; ++c)
                quant[6 + 3 * (int64_t)e + c] = (float)((double)sum[c] / (double)cnt);
    } else if (loss_out) {
        loss_out[0] += (float)(lambda * tot[0] / ((double)n * (double)qa.size));
    }
}

__global__ __launch_bounds__(256) void k_recipe_effective(const float4 *__restrict__ raw,
                                                          int64_t n, ImgTable tab, int32_t cov,
                                                          float4 *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float4 a = raw[2 * i], b = raw[2 * i + 1];
    float q[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
    int32_t H = tab.H, W = tab.W;
    if (tab.B > 1) {
        const int4 d = tab.dims[upper_index(tab.gauss_off, tab.B, (uint32_t)i)];
        H = d.x;
        W = d.y;
    }
    recipe_effective(q, H, W, cov == COV_ROTATION_SCALE);
    out[2 * i] = make_float4(q[0], q[1], q[2], q[3]);
    out[2 * i + 1] = make_float4(q[4], q[5], q[6], q[7]);
}

// Per-image mean of the squared residuals from the per-tile sums (float64 accumulation), and the
// step counter advance.  One block per image.
__global__ __launch_bounds__(256) void k_finish(const float *__restrict__ loss_part, ImgTable tab,
                                                int64_t n_tiles, float *__restrict__ loss_out) {
    __shared__ double red[4];
    block_image_losses(loss_part, tab, n_tiles, loss_out, red);
}

}  // namespace

__global__ __launch_bounds__(1024) void k_tile_order(const uint2 *__restrict__ ranges,
                                                     int64_t T, uint32_t *__restrict__ order) {
    __shared__ uint32_t bin[TILE_ORDER_BINS];
    __shared__ uint32_t wsum[1024 / 64];
    tile_order_block<1024>(ranges, T, order, bin, wsum);
}

hipError_t launch_tile_order(const uint2 *ranges, int64_t n_tiles, uint32_t *order,
                             hipStream_t s) {
    if (n_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(1024), 0, s, ranges, n_tiles, order);
    return hipGetLastError();
}

hipError_t launch_raster_fwd(const RasterArgs &a, float *image, int px, hipStream_t s,
                             DevState *flag_state, uint32_t *flags_out) {
    if (a.n_tiles <= 0) return hipSuccess;
    const float4 *rec = reinterpret_cast<const float4 *>(a.rec);
    switch (px) {
        case 1: hipLaunchKernelGGL(k_raster_fwd<1>, dim3((unsigned)a.n_tiles), dim3(256), 0, s, rec, a.ranges, a.tab, image, a.order, flag_state, flags_out); break;
        case 4: hipLaunchKernelGGL(k_raster_fwd<4>, dim3((unsigned)a.n_tiles), dim3(256), 0, s, rec, a.ranges, a.tab, image, a.order, flag_state, flags_out); break;
        default: hipLaunchKernelGGL(k_raster_fwd<2>, dim3((unsigned)a.n_tiles), dim3(256), 0, s, rec, a.ranges, a.tab, image, a.order, flag_state, flags_out); break;
    }
    return hipGetLastError();
}

hipError_t launch_raster_bwd(const RasterArgs &a, const float *dl, float *part, hipStream_t s) {
    if (a.n_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_raster_bwd, dim3((unsigned)a.n_tiles), dim3(BWD_T), 0, s,
                       reinterpret_cast<const float4 *>(a.rec), a.slot, a.ranges, a.tab, dl,
                       reinterpret_cast<float4 *>(part), a.order);
    return hipGetLastError();
}

hipError_t launch_raster_fit(const RasterArgs &a, const float *target, float *part,
                             float *image_out, float *loss_part, int px, int waves,
                             int32_t *step_inc, hipStream_t s) {
    if (a.n_tiles <= 0) return hipSuccess;
    const float4 *rec = reinterpret_cast<const float4 *>(a.rec);
    float4 *p4 = reinterpret_cast<float4 *>(part);
#define GI_LAUNCH_FIT(PX, WV)                                                                   \
    hipLaunchKernelGGL((k_raster_fit<PX, WV>), dim3((unsigned)a.n_tiles), dim3(256), 0, s, rec, \
                       a.slot, a.ranges, a.tab, target, p4, image_out, loss_part, step_inc,     \
                       a.order)
    if (waves == 6) {
        switch (px) {
            case 1: GI_LAUNCH_FIT(1, 6); break;
            case 4: GI_LAUNCH_FIT(4, 6); break;
            default: GI_LAUNCH_FIT(2, 6); break;
        }
    } else {
        switch (px) {
            case 1: GI_LAUNCH_FIT(1, 4); break;
            case 4: GI_LAUNCH_FIT(4, 4); break;
            default: GI_LAUNCH_FIT(2, 4); break;
        }
    }
#undef GI_LAUNCH_FIT
    return hipGetLastError();
}

hipError_t launch_alpha_fwd(const RasterArgs &a, const float *rec_o, float *image, hipStream_t s) {
    if (a.n_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_alpha_fwd, dim3((unsigned)a.n_tiles), dim3(256), 0, s,
                       reinterpret_cast<const float4 *>(a.rec), rec_o, a.ranges, a.tab, image, a.order);
    return hipGetLastError();
}

hipError_t launch_alpha_bwd(const RasterArgs &a, const float *rec_o, const float *dl,
                            float *part12, hipStream_t s) {
    if (a.n_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_alpha_bwd, dim3((unsigned)a.n_tiles), dim3(256), 0, s,
                       reinterpret_cast<const float4 *>(a.rec), rec_o, a.slot, a.ranges, a.tab,
                       dl, reinterpret_cast<float4 *>(part12), a.order);
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
                       int64_t n_tiles, float *loss_out, hipStream_t s, const uint2 *ranges,
                       uint32_t *order_out) {
    if (u.n > 0) {
        const bool ord = order_out && ranges && n_tiles > 0;
        const dim3 grid((unsigned)((u.n + UPD_G - 1) / UPD_G + (ord ? 1 : 0)));
        float4 *p4 = reinterpret_cast<float4 *>(params);
        const float4 *part = reinterpret_cast<const float4 *>(u.part);
        float2 *m2 = reinterpret_cast<float2 *>(m), *v2 = reinterpret_cast<float2 *>(v);
        float *nf = nullptr;
#define GI_LAUNCH_ADAM(C, O)                                                                    \
    hipLaunchKernelGGL((k_adam<C, BLEND_NONE, O>), grid, dim3(UPD_T), 0, s, p4, u.n, u.count,  \
                       u.off, part, u.state, u.cap, m2, v2, step, hp, nf, nf, nf, loss_part,   \
                       tab, n_tiles, loss_out, ranges, order_out)
        if (u.cov == COV_ROTATION_SCALE) {
            if (ord) GI_LAUNCH_ADAM(COV_ROTATION_SCALE, true);
            else GI_LAUNCH_ADAM(COV_ROTATION_SCALE, false);
        } else {
            if (ord) GI_LAUNCH_ADAM(COV_CHOLESKY, true);
            else GI_LAUNCH_ADAM(COV_CHOLESKY, false);
        }
#undef GI_LAUNCH_ADAM
        return hipGetLastError();
    }
    if (order_out && ranges && n_tiles > 0) {
        const hipError_t e = launch_tile_order(ranges, n_tiles, order_out, s);
        if (e != hipSuccess) return e;
    }
    return launch_finish(loss_part, tab, n_tiles, loss_out, s);
}

hipError_t launch_alpha_fit(const RasterArgs &a, const float *rec_o, const float *target,
                            float *part12, float *image_out, float *loss_part, int32_t *step_inc,
                            hipStream_t s) {
    if (a.n_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_alpha_fit, dim3((unsigned)a.n_tiles), dim3(256), 0, s,
                       reinterpret_cast<const float4 *>(a.rec), rec_o, a.slot, a.ranges, a.tab,
                       target, reinterpret_cast<float4 *>(part12), image_out, loss_part,
                       step_inc, a.order);
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
                       u.state, u.cap, m2, v2, step, hp, opacity, mo, vo, loss_part, tab,       \
                       n_tiles, loss_out)
        if (blend == BLEND_ALPHA) {
            if (rs) GI_LAUNCH_AO(COV_ROTATION_SCALE, BLEND_ALPHA);
            else GI_LAUNCH_AO(COV_CHOLESKY, BLEND_ALPHA);
        } else {
            if (rs) GI_LAUNCH_AO(COV_ROTATION_SCALE, BLEND_SUM);
            else GI_LAUNCH_AO(COV_CHOLESKY, BLEND_SUM);
        }
#undef GI_LAUNCH_AO
        return hipGetLastError();
    }
    return launch_finish(loss_part, tab, n_tiles, loss_out, s);
}

hipError_t launch_adan(const UpdateArgs &u, float *raw, float *state, int32_t *step,
                       const AdanArgs &hp, const ImgTable &tab, const float *loss_part,
                       int64_t n_tiles, float *loss_out, hipStream_t s) {
    if (u.n > 0) {
        const dim3 grid((unsigned)((u.n + UPD_G - 1) / UPD_G));
        float4 *r4 = reinterpret_cast<float4 *>(raw);
        const float4 *part = reinterpret_cast<const float4 *>(u.part);
        float2 *st2 = reinterpret_cast<float2 *>(state);
        if (u.cov == COV_ROTATION_SCALE)
            hipLaunchKernelGGL(k_adan<COV_ROTATION_SCALE>, grid, dim3(UPD_T), 0, s, r4, u.n,
                               u.count, u.off, part, u.state, u.cap, st2, step, hp, tab,
                               loss_part, n_tiles, loss_out);
        else
            hipLaunchKernelGGL(k_adan<COV_CHOLESKY>, grid, dim3(UPD_T), 0, s, r4, u.n, u.count,
                               u.off, part, u.state, u.cap, st2, step, hp, tab, loss_part,
                               n_tiles, loss_out);
        return hipGetLastError();
    }
    return launch_finish(loss_part, tab, n_tiles, loss_out, s);
}

hipError_t launch_qat_update(const UpdateArgs &u, float *params, float *m, float *v,
                             int32_t *step, const AdamArgs &hp, const QatArgs &qa, float lambda,
                             float lr_q, float *quant_m, float *quant_v, float *ema, float decay,
                             float *qpart, const float *loss_part, const ImgTable &tab,
                             int64_t n_tiles, float *loss_out, hipStream_t s) {
    if (u.n <= 0) return launch_finish(loss_part, tab, n_tiles, loss_out, s);
    const int64_t blocks = (u.n + UPD_G - 1) / UPD_G;
    const dim3 grid((unsigned)blocks);
    float4 *p4 = reinterpret_cast<float4 *>(params);
    const float4 *part = reinterpret_cast<const float4 *>(u.part);
    float2 *m2 = reinterpret_cast<float2 *>(m), *v2 = reinterpret_cast<float2 *>(v);
    if (u.cov == COV_ROTATION_SCALE)
        hipLaunchKernelGGL(k_qat_adam<COV_ROTATION_SCALE>, grid, dim3(UPD_T), 0, s, p4, u.n,
                           u.count, u.off, part, u.state, u.cap, m2, v2, step, hp, qa, qpart,
                           loss_part, tab, n_tiles, loss_out);
    else
        hipLaunchKernelGGL(k_qat_adam<COV_CHOLESKY>, grid, dim3(UPD_T), 0, s, p4, u.n, u.count,
                           u.off, part, u.state, u.cap, m2, v2, step, hp, qa, qpart, loss_part,
                           tab, n_tiles, loss_out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_qat_quant_update, dim3((unsigned)(6 + qa.stages * qa.size + 1)),
                       dim3(256), 0, s, const_cast<float *>(qa.quant), quant_m, quant_v, ema,
                       decay, qpart, blocks, u.n, qa, lambda, lr_q, hp, step, u.state, loss_out);
    return hipGetLastError();
}

int64_t qat_part_floats(int64_t n, int stages, int size) {
    const int64_t blocks = (n + UPD_G - 1) / UPD_G;
    return qat_dsum_offset(blocks) + 2 * 4 * (int64_t)stages * size * blocks;
}

hipError_t launch_recipe_effective(const float *raw, int64_t n, const ImgTable &tab, int32_t cov,
                                   float *params, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_recipe_effective, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       reinterpret_cast<const float4 *>(raw), n, tab, cov,
                       reinterpret_cast<float4 *>(params));
    return hipGetLastError();
}

hipError_t launch_finish(const float *loss_part, const ImgTable &tab, int64_t n_tiles,
                         float *loss_out, hipStream_t s) {
    if (!loss_out) return hipSuccess;
    hipLaunchKernelGGL(k_finish, dim3((unsigned)tab.B), dim3(256), 0, s, loss_part, tab, n_tiles,
                       loss_out);
    return hipGetLastError();
}

}  // namespace gi
