// Binning kernels for gfx950: projection and 3-sigma tile culling, prefix scans, and three
// ways to put every (tile, Gaussian) key into tile order with its record, slot and the tile
// ranges: a one-pass counting sort (up to 2048 tiles), row binning (a counting sort in two
// levels, for more tiles), and key duplication with a stable LSD radix sort and a gather (any
// size).  All three give the same order.
//
// The paper renders tile by tile (Sec. 4.1 builds on the tile-based rasteriser of 3D-GS) and
// removes the depth sort because the accumulated sum does not depend on order (Sec. 3.2, after
// Eq. rasterization3).  What remains is grouping Gaussians by tile: each Gaussian emits one
// (tile id, Gaussian id) key per covered tile, in row-major order within its rectangle, and a
// stable sort by tile id yields per-tile lists in ascending Gaussian order.
#include <cstring>
#include <type_traits>

#include "gi_common.h"

namespace gi {

namespace {

constexpr int BLK = 256;           // threads per block for per-Gaussian and per-key kernels
constexpr uint32_t DUP_OWN_CAP = 16384;  // keys of a duplication block held in its owner table
constexpr int SORT_T = 256;        // threads per sort block
constexpr int SORT_IPT = 16;       // keys per thread
constexpr int SORT_TILE = SORT_T * SORT_IPT;
constexpr int SORT_WAVES = SORT_T / 64;
constexpr int XCDS = 8;

// Workgroup i runs on XCD i mod 8.  Give each XCD a contiguous range of chunks, so that the
// chunks writing neighbouring positions of a tile's list share one L2 and their partial-line
// writes combine there before reaching memory.
__device__ inline uint32_t xcd_chunk(uint32_t i, uint32_t nchunk) {
    const uint32_t q = nchunk / XCDS, rem = nchunk % XCDS;
    const uint32_t x = i % XCDS, k = i / XCDS;
    return x * q + (x < rem ? x : rem) + k;
}
constexpr int SCAN_T = 256;
constexpr int SCAN_IPT = 16;
constexpr int SCAN_TILE = SCAN_T * SCAN_IPT;

// LDS staging index with one pad word per 32: both the coalesced (j * 256 + t) and the
// thread-contiguous (16 t + j) access patterns then hit 32 distinct banks.
__device__ inline int spad(int i) { return i + (i >> 5); }

// ---- small block-level helpers --------------------------------------------------------------

// in[idx] for idx < n, else 0, read without a branch (the index is clamped into [0, n) and the
// value dropped): guarded reads in an unrolled loop are otherwise awaited one by one.
__device__ inline uint32_t read_or_zero(const uint32_t *__restrict__ in, int64_t idx, int64_t n) {
    const uint32_t v = in[idx < n ? idx : (n > 0 ? n - 1 : 0)];
    return idx < n ? v : 0u;
}

template <typename T>
__device__ inline T wave_inclusive_scan(T v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        T o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

// Exclusive scan over the block; returns this thread's exclusive prefix, *total the sum.
// `tmp` holds one entry per wave.  Contains __syncthreads.
template <typename T, int NT>
__device__ inline T block_exclusive_scan(T v, T *tmp, T *total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    T inc = wave_inclusive_scan(v);
    if (lane == 63) tmp[wave] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        T run = 0;
        for (int w = 0; w < NT / 64; ++w) {
            T x = tmp[w];
            tmp[w] = run;
            run += x;
        }
        tmp[NT / 64] = run;
    }
    __syncthreads();
    T res = inc - v + tmp[wave];
    *total = tmp[NT / 64];
    __syncthreads();
    return res;
}

// ---- K1: projection and tile culling ---------------------------------------------------------

// r^2 >= 9 lambda_max(Sigma), decided by the characteristic polynomial of Sigma at R/9 with
// R = r^2: p = R - 9 s00, q = R - 9 s11, p + q >= 0 and p q >= 81 s01^2.  Every step is a
// separately rounded IEEE float64 operation (no contraction) so that the decision is
// reproducible on any IEEE machine that evaluates the same expression.
__device__ inline bool covers(double r, double s00, double s01, double s11) {
#pragma clang fp contract(off)
    double R = r * r;
    double p = R - 9.0 * s00;
    double q = R - 9.0 * s11;
    return ((p + q) >= 0.0) && ((p * q) >= 81.0 * (s01 * s01));
}

constexpr double R_MAX = 33554432.0;  // 2^25: covers any image once |mu| <= 2^24

// Record of Gaussian i from the source.  A compressed record is decoded as in Sec. 3.3: the
// binary16 positions exactly, each covariance code as code * gamma + beta and the colour as the
// sum of the stage codebook entries in stage order, all in float64 (the products are exact)
// and rounded once to float32.  Returns false when a code or an index is out of range.
__device__ inline bool load_record(const RecordSrc &src, int64_t i, float (&q)[8]) {
#pragma clang fp contract(off)
    if (!src.codec.mu) {
        const float4 q0 = src.params[2 * i], q1 = src.params[2 * i + 1];
        q[0] = q0.x; q[1] = q0.y; q[2] = q0.z; q[3] = q0.w;
        q[4] = q1.x; q[5] = q1.y; q[6] = q1.z; q[7] = q1.w;
        return true;
    }
    const CodecArgs &c = src.codec;
    const uint32_t mu = reinterpret_cast<const uint32_t *>(c.mu)[i];
    q[0] = (float)__builtin_bit_cast(_Float16, (uint16_t)(mu & 0xffffu));
    q[1] = (float)__builtin_bit_cast(_Float16, (uint16_t)(mu >> 16));
    const uint32_t lim = (1u << c.bits) - 1u;
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const uint32_t code = c.codes[3 * i + k];
        ok = ok && code <= lim;
        q[2 + k] = (float)((double)code * (double)c.gamma[k] + (double)c.beta[k]);
    }
    double col0 = 0.0, col1 = 0.0, col2 = 0.0;
    for (int m = 0; m < c.stages; ++m) {
        uint32_t ix = c.index[i * c.stages + m];
        if (ix >= (uint32_t)c.size) {
            ok = false;
            ix = 0;
        }
        const float *e = c.book + ((int64_t)m * c.size + ix) * 3;
        col0 += (double)e[0];
        col1 += (double)e[1];
        col2 += (double)e[2];
    }
    q[5] = (float)col0;
    q[6] = (float)col1;
    q[7] = (float)col2;
    return ok;
}

// Projection and tile rectangle of Gaussian i (see the file header of k_raster.hip for the
// stored record).  Writes proj, rect, tinfo and count; returns the count.  FACTS (radix path):
// one 64-byte line per Gaussian with the slot facts that the gather after the sort reads; else
// (one-pass path) the 32-byte record alone, at a stride of 32 bytes.
template <bool FACTS>
__device__ inline uint32_t project_one(const RecordSrc &src, int64_t i,
                                       const ImgTable &tab, float4 *__restrict__ proj,
                                       int4 *__restrict__ rect, uint2 *__restrict__ tinfo,
                                       uint32_t *__restrict__ count, bool *nonfinite,
                                       bool *bad_code, int4 *rc_out, uint2 *inf_out,
                                       int32_t *img_out = nullptr) {
#pragma clang fp contract(off)
    uint32_t cnt = 0;
    float q[8];
    const bool code_ok = load_record(src, i, q);
    *bad_code = !code_ok;
    float o = 1.f;
    if (src.opacity) o = src.opacity[i];
    int32_t TW, TH, IH, IW;
    uint32_t tb, rb = 0;
    if (tab.B == 1) {
        // taken through readfirstlane so that they are values, not loads: the compiler had
        // merged this branch and the table read below into one flat load through a pointer
        // select (the kernel argument copied to private memory)
        TW = __builtin_amdgcn_readfirstlane(tab.TW);
        IH = __builtin_amdgcn_readfirstlane(tab.H);
        IW = __builtin_amdgcn_readfirstlane(tab.W);
        TH = (IH + TILE - 1) / TILE; tb = 0;
    } else {
        int32_t b = upper_index(tab.gauss_off, tab.B, (uint32_t)i);
        if (img_out) *img_out = b;
        int4 d = tab.dims[b];
        TW = d.z; TH = d.w; tb = tab.tile_base[b];
        if (FACTS) rb = tab.row_base[b];
        IH = d.x; IW = d.y;
    }
    if (src.recipe) recipe_effective(q, IH, IW, tab.cov == COV_ROTATION_SCALE);
    if (src.qat.quant) qat_fake_quant(q, src.qat, nullptr);
    bool finite = true;
#pragma unroll
    for (int k = 0; k < 8; ++k) finite = finite && isfinite(q[k]);
    finite = finite && isfinite(o);
    *nonfinite = !finite;
    const double mx = q[0], my = q[1];
    const bool rs = tab.cov == COV_ROTATION_SCALE;
    // (q2, q3, q4) = (l1, l2, l3), or (s1, s2, theta) in the rotation-scale form
    bool act = code_ok && finite && fabs(mx) <= 0x1p24 && fabs(my) <= 0x1p24 &&
               (rs ? fabs(q[2]) >= 0x1p-24 && fabs(q[3]) >= 0x1p-24 && fabs(q[4]) <= 0x1p24
                   : fabs(q[2]) >= 0x1p-24 && fabs(q[4]) >= 0x1p-24 && fabs(q[3]) <= 0x1p24);
    int4 rc = make_int4(0, 0, -1, -1);
    float4 p0 = make_float4(0.f, 0.f, 0.f, 0.f), p1 = p0;
    if (act) {
        double l1, l2, l3, r;
        if (rs) {
            // Sigma = R diag(s1^2, s2^2) R^T (Eq. RSSR) and its Cholesky factor: l1 = sqrt(s00),
            // l2 = s01 / l1, l3 = |s1 s2| / l1 (det Sigma = (l1 l3)^2 = (s1 s2)^2).  The
            // eigenvalues are s1^2 and s2^2, so r is the least integer with
            // r^2 >= 9 max(s1^2, s2^2); 3|s| and the squares are exact in float64.
            const double s1 = q[2], s2 = q[3];
            double sn, cs;
            sincos((double)q[4], &sn, &cs);
            const double A = s1 * s1, B = s2 * s2;
            const double s00 = cs * cs * A + sn * sn * B, s01 = cs * sn * (A - B);
            l1 = sqrt(s00);
            l2 = s01 / l1;
            l3 = fabs(s1 * s2) / l1;
            const double m = A > B ? A : B;
            r = ceil(3.0 * sqrt(m));
            if (r > R_MAX) r = R_MAX;
            while (r > 0.0 && (r - 1.0) * (r - 1.0) >= 9.0 * m) r -= 1.0;
            while (r < R_MAX && r * r < 9.0 * m) r += 1.0;
        } else {
            l1 = q[2]; l2 = q[3]; l3 = q[4];
            const double s00 = l1 * l1, s01 = l1 * l2, s11 = l2 * l2 + l3 * l3;
            // starting guess from the eigenvalue formula, then the least r that covers
            const double lam =
                0.5 * (s00 + s11) + sqrt(0.25 * (s00 - s11) * (s00 - s11) + s01 * s01);
            r = ceil(3.0 * sqrt(lam));
            if (!(r >= 0.0)) r = 0.0;
            if (r > R_MAX) r = R_MAX;
            while (r > 0.0 && covers(r - 1.0, s00, s01, s11)) r -= 1.0;
            while (r < R_MAX && !covers(r, s00, s01, s11)) r += 1.0;
        }
        double fx0 = floor((mx - r) / 16.0), fx1 = floor((mx + r) / 16.0);
        double fy0 = floor((my - r) / 16.0), fy1 = floor((my + r) / 16.0);
        if (fx0 < 0.0) fx0 = 0.0;
        if (fy0 < 0.0) fy0 = 0.0;
        if (fx1 > TW - 1.0) fx1 = TW - 1.0;
        if (fy1 > TH - 1.0) fy1 = TH - 1.0;
        if (fx0 <= fx1 && fy0 <= fy1) {
            rc = make_int4((int)fx0, (int)fy0, (int)fx1, (int)fy1);
            cnt = (uint32_t)(rc.z - rc.x + 1) * (uint32_t)(rc.w - rc.y + 1);
        }
        p0 = make_float4(q[0], q[1], (float)(U_SCALE / l1), (float)(U_SCALE / l3));
        if (src.blend == BLEND_SUM) {  // Eq. rasterization3: the record colour is o c
            q[5] *= o;
            q[6] *= o;
            q[7] *= o;
        }
        p1 = make_float4((float)(U_SCALE * l2 / (l1 * l3)), q[5], q[6], q[7]);
    }
    constexpr int STRIDE = FACTS ? PROJ_F4 : 2;
    proj[STRIDE * i] = p0;
    proj[STRIDE * i + 1] = p1;
    // the facts that turn a (tile, Gaussian) key into its slot: the key offset (written once the
    // counts are scanned), the image's first tile and tiles per row, the rectangle's width and
    // corner (all tile counts < 2^16); then the global tile row of the rectangle's first row and
    // its row count (row binning)
    if (FACTS) {
        proj[PROJ_F4 * i + 2] = __builtin_bit_cast(
            float4, make_uint4(0u, tb, (uint32_t)TW | ((uint32_t)(rc.z - rc.x + 1) << 16),
                               (uint32_t)rc.x | ((uint32_t)rc.y << 16)));
        proj[PROJ_F4 * i + 3] = __builtin_bit_cast(
            float4, make_uint4(rb + (uint32_t)rc.y, cnt ? (uint32_t)(rc.w - rc.y + 1) : 0u, 0u, 0u));
    }
    rect[i] = rc;
    const uint2 inf = make_uint2(tb, (uint32_t)TW);
    tinfo[i] = inf;
    count[i] = cnt;
    *rc_out = rc;
    *inf_out = inf;
    return cnt;
}

// Row binning's per-block row counts (see ImgTable): scan == null when not wanted.
struct RowHistArgs {
    uint32_t *scan;  // [len + 1]
    int64_t len;
    uint4 *bwin;     // [blocks] (first global row, rows) of the images the block spans
};

__device__ inline unsigned long long row_seg_of(const ImgTable &t, uint32_t row, uint32_t blocks) {
    return t.B == 1 ? (unsigned long long)row * blocks : t.row_seg[row];
}
__device__ inline uint32_t row_fb_of(const ImgTable &t, uint32_t row) {
    return t.B == 1 ? 0u : t.row_fb[row];
}

__global__ __launch_bounds__(BLK) void k_project(const RecordSrc src, int64_t n,
                                                 ImgTable tab, float4 *__restrict__ proj,
                                                 int4 *__restrict__ rect,
                                                 uint2 *__restrict__ tinfo,
                                                 uint32_t *__restrict__ count,
                                                 unsigned long long *__restrict__ blocksum,
                                                 RowHistArgs rh, DevState *state) {
    __shared__ unsigned long long tmp[BLK / 64 + 1];
    __shared__ uint32_t rhc[ROW_WIN_MAX];
    __shared__ int32_t img_lo, img_hi;
    const int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x;
    uint32_t cnt = 0, rows = 0, row0 = 0;
    int32_t img = 0;
    bool nonfinite = false, bad = false;
    if (rh.scan && threadIdx.x == 0) {
        img_lo = 0x7fffffff;
        img_hi = -1;
        // a new epoch for the chained scan of the row counts that follows
        if (blockIdx.x == 0) state->scan_epoch += 1u;
    }
    if (i < n) {
        int4 rc;
        uint2 inf;
        cnt = project_one<true>(src, i, tab, proj, rect, tinfo, count, &nonfinite, &bad, &rc,
                                &inf, &img);
        rows = cnt ? (uint32_t)(rc.w - rc.y + 1) : 0u;
        if (rh.scan) row0 = (tab.B == 1 ? 0u : tab.row_base[img]) + (uint32_t)rc.y;
    }
    if (__ballot(nonfinite) && (threadIdx.x & 63) == 0) atomicOr(&state->flags, FLAG_NONFINITE);
    if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(&state->flags, FLAG_BAD_CODE);
    unsigned long long tot;
    block_exclusive_scan<unsigned long long, BLK>((unsigned long long)cnt, tmp, &tot);
    if (threadIdx.x == 0) blocksum[blockIdx.x] = tot;
    if (!rh.scan) return;
    // row binning: this block's count of (row, Gaussian) pairs per tile row of the images its
    // Gaussians belong to (a window of consecutive global rows)
    if (i < n) {
        atomicMin(&img_lo, img);
        atomicMax(&img_hi, img);
    }
    for (int r = threadIdx.x; r < ROW_WIN_MAX; r += BLK) rhc[r] = 0u;
    __syncthreads();
    uint32_t w0, W;
    if (tab.B == 1) {
        w0 = 0;
        W = (uint32_t)tab.rows;
    } else {
        w0 = tab.row_base[img_lo];
        W = tab.row_base[img_hi + 1] - w0;
    }
    for (uint32_t k = 0; k < rows; ++k) atomicAdd(&rhc[row0 - w0 + k], 1u);
    __syncthreads();
    const uint32_t blocks = (uint32_t)gridDim.x;
    for (uint32_t r = threadIdx.x; r < W; r += BLK) {
        const uint32_t row = w0 + r, fb = row_fb_of(tab, row);
        if (fb != 0xffffffffu) rh.scan[row_seg_of(tab, row, blocks) + (blockIdx.x - fb)] = rhc[r];
    }
    if (threadIdx.x == 0) {
        rh.bwin[blockIdx.x] = make_uint4(w0, W, 0u, 0u);
        if (blockIdx.x == 0) rh.scan[rh.len] = 0u;  // the closing zero: its prefix is the total
    }
}

// Exclusive scan of the per-block totals by one 1024-thread block; also the grand total.  A
// second block, when launched, does the same for bs2 / total2.
__global__ __launch_bounds__(1024) void k_scan_top(unsigned long long *__restrict__ bs, int64_t nb,
                                                   unsigned long long *__restrict__ total,
                                                   unsigned long long *__restrict__ bs2,
                                                   unsigned long long *__restrict__ total2) {
    __shared__ unsigned long long tmp[1024 / 64 + 1];
    if (blockIdx.x == 1) {
        bs = bs2;
        total = total2;
    }
    const int64_t per = (nb + 1023) / 1024;
    const int64_t beg = threadIdx.x * per;
    const int64_t end = beg + per < nb ? beg + per : nb;
    unsigned long long s = 0;
    for (int64_t j = beg; j < end; ++j) s += bs[j];
    unsigned long long tot;
    unsigned long long run = block_exclusive_scan<unsigned long long, 1024>(s, tmp, &tot);
    for (int64_t j = beg; j < end; ++j) {
        unsigned long long x = bs[j];
        bs[j] = run;
        run += x;
    }
    if (threadIdx.x == 0 && total) *total = tot;
}

// ---- K2: key duplication --------------------------------------------------------------------

// Block b handles Gaussians [256 b, 256 b + 256): it rebuilds their offsets from the scanned
// block totals, then its threads stride over the block's keys so that writes are coalesced.  A
// key finds its Gaussian in an LDS table (one byte per key) when the block's keys fit, else by
// binary search over the offsets.
__global__ __launch_bounds__(BLK) void k_duplicate(const uint32_t *__restrict__ count,
                                                   const int4 *__restrict__ rect,
                                                   const uint2 *__restrict__ tinfo,
                                                   const unsigned long long *__restrict__ bs,
                                                   int64_t n, int64_t cap,
                                                   uint32_t *__restrict__ off,
                                                   uint32_t *__restrict__ keys,
                                                   uint32_t *__restrict__ vals,
                                                   float4 *__restrict__ proj,
                                                   DevState *state) {
    __shared__ unsigned long long tmp[BLK / 64 + 1];
    __shared__ unsigned long long pre[BLK];
    __shared__ int4 srect[BLK];
    __shared__ uint2 sinfo[BLK];
    __shared__ uint8_t owner[DUP_OWN_CAP];  // block-local key -> its Gaussian, when the keys fit
    const int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x;
    const uint32_t c = i < n ? count[i] : 0u;
    unsigned long long tot;
    const unsigned long long loc = block_exclusive_scan<unsigned long long, BLK>(c, tmp, &tot);
    const bool table = tot <= DUP_OWN_CAP;  // the same for the whole block
    if (table)
        for (uint32_t k = 0; k < c; ++k) owner[loc + k] = (uint8_t)threadIdx.x;
    const unsigned long long base = bs[blockIdx.x];
    pre[threadIdx.x] = loc;
    if (i < n) {
        off[i] = (uint32_t)(base + loc);
        reinterpret_cast<uint32_t *>(proj)[4 * (PROJ_F4 * i + 2)] = (uint32_t)(base + loc);
        srect[threadIdx.x] = rect[i];
        sinfo[threadIdx.x] = tinfo[i];
    }
    __syncthreads();
    unsigned long long limit = tot;
    if (base >= (unsigned long long)cap) limit = 0;
    else if (base + tot > (unsigned long long)cap) limit = (unsigned long long)cap - base;
    if (limit < tot && threadIdx.x == 0) atomicOr(&state->flags, FLAG_KEY_OVERFLOW);
    for (unsigned long long j = threadIdx.x; j < limit; j += BLK) {
        int lo = 0;  // owner: largest g with pre[g] <= j
        if (table) {
            lo = owner[j];
        } else {
            int hi = BLK - 1;
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if (pre[mid] <= j) lo = mid; else hi = mid - 1;
            }
        }
        const int4 r = srect[lo];
        const uint2 inf = sinfo[lo];
        const uint32_t li = (uint32_t)(j - pre[lo]);
        const uint32_t w = (uint32_t)(r.z - r.x + 1);
        const uint32_t tx = (uint32_t)r.x + li % w, ty = (uint32_t)r.y + li / w;
        // the sort carries the Gaussian; its position in Gaussian-major order (the slot) is
        // formed again after the sort from the projected record
        keys[base + j] = inf.x + ty * inf.y + tx;
        vals[base + j] = (uint32_t)((int64_t)blockIdx.x * BLK + lo);
    }
}

// ---- generic exclusive scan of uint32 --------------------------------------------------------

__global__ __launch_bounds__(SCAN_T) void k_scan_reduce(const uint32_t *__restrict__ in, int64_t n,
                                                        unsigned long long *__restrict__ bs) {
    __shared__ unsigned long long tmp[SCAN_T / 64 + 1];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    unsigned long long s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_IPT; ++j) s += read_or_zero(in, base + j * SCAN_T + threadIdx.x, n);
    unsigned long long tot;
    block_exclusive_scan<unsigned long long, SCAN_T>(s, tmp, &tot);
    if (threadIdx.x == 0) bs[blockIdx.x] = tot;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_down(const uint32_t *__restrict__ in,
                                                      uint32_t *__restrict__ out, int64_t n,
                                                      const unsigned long long *__restrict__ bs) {
    __shared__ unsigned long long tmp[SCAN_T / 64 + 1];
    __shared__ uint32_t stage[SCAN_TILE + SCAN_TILE / 32];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    // coalesced load into LDS, then each thread scans 16 consecutive values
    {
        uint32_t x[SCAN_IPT];
#pragma unroll
        for (int j = 0; j < SCAN_IPT; ++j) x[j] = read_or_zero(in, base + j * SCAN_T + threadIdx.x, n);
#pragma unroll
        for (int j = 0; j < SCAN_IPT; ++j) stage[spad(j * SCAN_T + threadIdx.x)] = x[j];
    }
    __syncthreads();
    uint32_t v[SCAN_IPT];
    unsigned long long s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_IPT; ++j) {
        v[j] = stage[spad(threadIdx.x * SCAN_IPT + j)];
        s += v[j];
    }
    unsigned long long tot;
    unsigned long long run = block_exclusive_scan<unsigned long long, SCAN_T>(s, tmp, &tot) +
                             bs[blockIdx.x];
#pragma unroll
    for (int j = 0; j < SCAN_IPT; ++j) {
        stage[spad(threadIdx.x * SCAN_IPT + j)] = (uint32_t)run;
        run += v[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < SCAN_IPT; ++j) {
        int64_t idx = base + j * SCAN_T + threadIdx.x;
        if (idx < n) out[idx] = stage[spad(j * SCAN_T + threadIdx.x)];
    }
}

// Small arrays (n <= 1024 * 16): one block does the whole exclusive scan.
__global__ __launch_bounds__(1024) void k_scan_single(const uint32_t *__restrict__ in,
                                                      uint32_t *__restrict__ out, int64_t n,
                                                      unsigned long long *__restrict__ total) {
    __shared__ unsigned long long tmp[1024 / 64 + 1];
    uint32_t v[16];
    unsigned long long s = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = read_or_zero(in, (int64_t)threadIdx.x * 16 + j, n);
#pragma unroll
    for (int j = 0; j < 16; ++j) s += v[j];
    unsigned long long tot;
    unsigned long long run = block_exclusive_scan<unsigned long long, 1024>(s, tmp, &tot);
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        int64_t idx = (int64_t)threadIdx.x * 16 + j;
        if (idx < n) out[idx] = (uint32_t)run;
        run += v[j];
    }
    if (threadIdx.x == 0 && total) *total = tot;
}

// ---- K3: stable LSD radix sort ---------------------------------------------------------------

__device__ inline int64_t sort_count(const unsigned long long *n_dev, int64_t n_max) {
    if (!n_dev) return n_max;
    unsigned long long t = *n_dev;
    return t < (unsigned long long)n_max ? (int64_t)t : n_max;
}

// Lanes of the wave whose digit equals this lane's (BITS ballots); `valid` lanes only.
template <int BITS>
__device__ inline unsigned long long match_digit(uint32_t d, bool valid) {
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
        const bool bit = (d >> b) & 1u;
        const unsigned long long bal = __ballot(bit);
        peers &= bit ? bal : ~bal;
    }
    return peers;
}

// Per-block digit histogram, written digit-major: hist[d * nblk + block].
// epoch (if not null): advanced for the chained scan of the histogram that follows.
template <int BITS>
__global__ __launch_bounds__(SORT_T) void k_radix_hist(const uint32_t *__restrict__ keys,
                                                       const unsigned long long *n_dev,
                                                       int64_t n_max, int shift,
                                                       uint32_t *__restrict__ hist,
                                                       int64_t nblk, DevState *epoch) {
    constexpr int BINS = 1 << BITS;
    __shared__ uint32_t h[SORT_WAVES][BINS];
    if (epoch && blockIdx.x == 0 && threadIdx.x == 0) epoch->scan_epoch += 1u;
    const int64_t n = sort_count(n_dev, n_max);
    const uint32_t nbu = (uint32_t)((n + SORT_TILE - 1) / SORT_TILE);
    const uint32_t blk = blockIdx.x < nbu ? xcd_chunk(blockIdx.x, nbu) : blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int d = threadIdx.x; d < SORT_WAVES * BINS; d += SORT_T) (&h[0][0])[d] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blk * SORT_TILE + (int64_t)wave * (SORT_TILE / SORT_WAVES);
    constexpr int ROUNDS = SORT_TILE / SORT_WAVES / 64;
    // all reads first (lanes past the end read the last key and drop it): a read under the
    // validity test would be awaited before the next one is issued
    const int64_t last = n > 0 ? n - 1 : 0;
    uint32_t kr[ROUNDS];
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) kr[r] = keys[min(base + r * 64 + lane, last)];
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        const bool valid = base + r * 64 + lane < n;
        const uint32_t d = valid ? (kr[r] >> shift) & (BINS - 1) : 0u;
        const unsigned long long peers = match_digit<BITS>(d, valid);
        if (valid && lane == __ffsll((long long)peers) - 1) h[wave][d] += __popcll(peers);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < BINS; d += SORT_T) {
        uint32_t s = 0;
#pragma unroll
        for (int w = 0; w < SORT_WAVES; ++w) s += h[w][d];
        hist[(int64_t)d * nblk + blk] = s;
    }
}

// Scatter with stable in-block ranks.  `hist` holds the exclusive scan of the digit-major
// histogram: the output position of the first key with digit d from block b.
template <int BITS>
__global__ __launch_bounds__(SORT_T) void k_radix_scatter(const uint32_t *__restrict__ kin,
                                                          const uint32_t *__restrict__ vin,
                                                          uint32_t *__restrict__ kout,
                                                          uint32_t *__restrict__ vout,
                                                          const unsigned long long *n_dev,
                                                          int64_t n_max, int shift,
                                                          const uint32_t *__restrict__ hist,
                                                          int64_t nblk) {
    constexpr int BINS = 1 << BITS;
    constexpr int ROUNDS = SORT_TILE / SORT_WAVES / 64;
    __shared__ uint32_t wh[SORT_WAVES][BINS];   // per-wave digit counts, then wave offsets
    __shared__ uint32_t dstart[BINS];            // first in-block position of each digit
    __shared__ uint32_t gofs[BINS];              // output position minus in-block position
    __shared__ uint32_t sk[SORT_TILE];
    __shared__ uint32_t sv[SORT_TILE];
    __shared__ uint32_t tmp[SORT_T / 64 + 1];
    const int64_t n = sort_count(n_dev, n_max);
    const uint32_t nbu = (uint32_t)((n + SORT_TILE - 1) / SORT_TILE);
    if (blockIdx.x >= nbu) return;
    const uint32_t blk = xcd_chunk(blockIdx.x, nbu);
    const int64_t blk_base = (int64_t)blk * SORT_TILE;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // this block's output base of every digit: read now, used after the ranking
    constexpr int DPT = (BINS + SORT_T - 1) / SORT_T;
    uint32_t hb[DPT];
#pragma unroll
    for (int k = 0; k < DPT; ++k) {
        const int d = (int)threadIdx.x + k * SORT_T;
        hb[k] = hist[(int64_t)(d < BINS ? d : BINS - 1) * nblk + blk];
    }
    for (int d = threadIdx.x; d < SORT_WAVES * BINS; d += SORT_T) (&wh[0][0])[d] = 0;
    __syncthreads();
    const int64_t base = blk_base + (int64_t)wave * (SORT_TILE / SORT_WAVES);
    uint32_t key[ROUNDS], val[ROUNDS], rank[ROUNDS];
    // all reads first (lanes past the end read the last pair and drop it), then the ranking
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        const int64_t idx = min(base + r * 64 + lane, n - 1);
        key[r] = kin[idx];
        val[r] = vin[idx];
    }
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        const int64_t idx = base + r * 64 + lane;
        const bool valid = idx < n;
        if (!valid) key[r] = val[r] = 0u;
        const uint32_t d = (key[r] >> shift) & (BINS - 1);
        const unsigned long long peers = match_digit<BITS>(d, valid);
        const unsigned long long lt = (1ull << lane) - 1ull;
        const uint32_t old = valid ? wh[wave][d] : 0u;  // every peer reads before the leader writes
        if (valid && lane == __ffsll((long long)peers) - 1) wh[wave][d] = old + __popcll(peers);
        rank[r] = old + __popcll(peers & lt);
    }
    __syncthreads();
    // wave offsets within each digit, and digit totals of the block
    uint32_t my_total = 0;
    for (int d = threadIdx.x; d < BINS; d += SORT_T) {
        uint32_t run = 0;
#pragma unroll
        for (int w = 0; w < SORT_WAVES; ++w) {
            uint32_t x = wh[w][d];
            wh[w][d] = run;
            run += x;
        }
        dstart[d] = run;  // total for now
    }
    __syncthreads();
    // exclusive scan of the digit totals (BINS entries, SORT_T threads, contiguous chunks)
    {
        constexpr int PER = (BINS + SORT_T - 1) / SORT_T;
        uint32_t loc[PER];
        uint32_t s = 0;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int d = threadIdx.x * PER + j;
            loc[j] = d < BINS ? dstart[d] : 0u;
            s += loc[j];
        }
        uint32_t tot;
        uint32_t run = block_exclusive_scan<uint32_t, SORT_T>(s, tmp, &tot);
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int d = threadIdx.x * PER + j;
            if (d < BINS) dstart[d] = run;
            run += loc[j];
        }
        (void)my_total;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < DPT; ++k) {
        const int d = (int)threadIdx.x + k * SORT_T;
        if (d < BINS) gofs[d] = hb[k] - dstart[d];
    }
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        const int64_t idx = base + r * 64 + lane;
        if (idx < n) {
            const uint32_t d = (key[r] >> shift) & (BINS - 1);
            const uint32_t pos = dstart[d] + wh[wave][d] + rank[r];
            sk[pos] = key[r];
            sv[pos] = val[r];
        }
    }
    __syncthreads();
    const int64_t cnt = n - blk_base < SORT_TILE ? n - blk_base : SORT_TILE;
    for (int j = threadIdx.x; j < cnt; j += SORT_T) {
        const uint32_t k = sk[j];
        const uint32_t d = (k >> shift) & (BINS - 1);
        const uint32_t dst = gofs[d] + (uint32_t)j;
        kout[dst] = k;
        vout[dst] = sv[j];
    }
}

// ---- K3: tile ranges and the gather into tile order -----------------------------------------

__global__ __launch_bounds__(BLK) void k_ranges_gather(const uint32_t *__restrict__ keys,
                                                       const uint32_t *__restrict__ vals,
                                                       const unsigned long long *n_dev,
                                                       int64_t n_max,
                                                       const float4 *__restrict__ proj,
                                                       uint2 *__restrict__ ranges,
                                                       float4 *__restrict__ rec,
                                                       uint32_t *__restrict__ slot,
                                                       const float *__restrict__ opac,
                                                       float *__restrict__ rec_o,
                                                       uint32_t *__restrict__ ids) {
    const int64_t n = sort_count(n_dev, n_max);
    const uint32_t nb = (uint32_t)((n + BLK - 1) / BLK);
    if (blockIdx.x >= nb) return;
    const int64_t i = (int64_t)xcd_chunk(blockIdx.x, nb) * BLK + threadIdx.x;
    if (i >= n) return;
    // the key, its neighbours and the Gaussian are read together (clamped, not guarded)
    const uint32_t key = keys[i];
    const uint32_t kp = keys[i > 0 ? i - 1 : 0], kn = keys[i + 1 < n ? i + 1 : i];
    const uint32_t g = vals[i];
    // one 64-byte projected record per key: the rasteriser record and the slot facts
    const float4 a = proj[PROJ_F4 * (int64_t)g], b = proj[PROJ_F4 * (int64_t)g + 1];
    const uint4 f = __builtin_bit_cast(uint4, proj[PROJ_F4 * (int64_t)g + 2]);
    if (i == 0 || kp != key) ranges[key].x = (uint32_t)i;
    if (i == n - 1 || kn != key) ranges[key].y = (uint32_t)(i + 1);
    const uint32_t tw = f.z & 0xffffu, w = f.z >> 16;
    const uint32_t local = key - f.y;  // ty * TW + tx within the Gaussian's image
    const uint32_t ty = local / tw, tx = local - ty * tw;
    rec[2 * i] = a;
    rec[2 * i + 1] = b;
    if (slot) slot[i] = f.x + (ty - (f.w >> 16)) * w + (tx - (f.w & 0xffffu));
    if (rec_o) rec_o[i] = opac[g];
    if (ids) ids[i] = g;
}

__global__ __launch_bounds__(BLK) void k_fill_u32(uint32_t *__restrict__ p, uint32_t v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---- one-pass binning for up to FUSED_MAX_TILES tiles --------------------------------------
//
// (A) k_project_hist: projection of a chunk of 256 Gaussians and the chunk's per-tile key
//     counts, written tile-major after the Gaussian counts: scan[n + t * nchunk + chunk].
// (B) k_chained_scan: exclusive scan of scan[0 .. n + T nchunk) in one pass (each block
//     publishes its sum and looks back over its predecessors).  The first n entries become the
//     key offsets of the Gaussians; entry n + t nchunk + c becomes K + the position of chunk c's
//     first key of tile t in tile order.
// (C) k_fused_scatter: each chunk enumerates its keys again in Gaussian-major order, ranks them
//     stably per tile, and writes the records, slots and Gaussian ids straight into tile order,
//     plus the tile ranges.  No key array is written or sorted: this is the counting sort by
//     tile id in one pass, and the result equals that of the stable radix sort.

constexpr int FB = 256;
// the scatter splits a chunk's keys over 4 or 8 waves (more waves per CU hide its latency;
// each needs T words of LDS counters), see scatter_waves
constexpr uint32_t OWN_CAP = 4096;
constexpr int CS_T = 256;
constexpr int CS_IPT = 16;
constexpr int CS_TILE = CS_T * CS_IPT;
// status word: epoch tag (29 bits) | flag (2 bits: 1 = block sum, 2 = inclusive prefix) |
// value (33 bits; every prefix is at most twice the key count)
constexpr int CS_EPOCH_SHIFT = 35;
constexpr int CS_FLAG_SHIFT = 33;
constexpr unsigned long long CS_TAG_MASK = 0x1fffffffull << CS_EPOCH_SHIFT;
constexpr unsigned long long CS_FLAG_MASK = 3ull << CS_FLAG_SHIFT;
constexpr unsigned long long CS_AGG = 1ull << CS_FLAG_SHIFT;
constexpr unsigned long long CS_PRE = 2ull << CS_FLAG_SHIFT;
constexpr unsigned long long CS_VAL = (1ull << CS_FLAG_SHIFT) - 1;
constexpr long SPIN_LIMIT = 1l << 20;

__global__ __launch_bounds__(FB) void k_project_hist(const RecordSrc src, int64_t n,
                                                     ImgTable tab, float4 *__restrict__ proj,
                                                     int4 *__restrict__ rect,
                                                     uint2 *__restrict__ tinfo,
                                                     uint32_t *__restrict__ count,
                                                     uint32_t *__restrict__ scan, int32_t T,
                                                     int64_t nchunk, DevState *state) {
    extern __shared__ uint32_t h[];  // [T]
    // a new epoch for the scan that follows (see k_chained_scan)
    if (blockIdx.x == 0 && threadIdx.x == 0) state->scan_epoch += 1u;
    for (int t = threadIdx.x; t < T; t += FB) h[t] = 0;
    __syncthreads();
    const uint32_t chunk = xcd_chunk(blockIdx.x, (uint32_t)nchunk);
    const int64_t i = (int64_t)chunk * FB + threadIdx.x;
    bool nonfinite = false, bad = false;
    if (i < n) {
        int4 rc;
        uint2 inf;
        const uint32_t cnt = project_one<false>(src, i, tab, proj, rect, tinfo, count, &nonfinite,
                                                &bad, &rc, &inf);
        scan[i] = cnt;
        if (cnt) {
            for (int ty = rc.y; ty <= rc.w; ++ty)
                for (int tx = rc.x; tx <= rc.z; ++tx)
                    atomicAdd(&h[inf.x + (uint32_t)ty * inf.y + (uint32_t)tx], 1u);
        }
    }
    if (__ballot(nonfinite) && (threadIdx.x & 63) == 0) atomicOr(&state->flags, FLAG_NONFINITE);
    if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(&state->flags, FLAG_BAD_CODE);
    __syncthreads();
    for (int t = threadIdx.x; t < T; t += FB) scan[n + (int64_t)t * nchunk + chunk] = h[t];
}

__device__ inline unsigned long long load_status(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exclusive scan of data[0 .. L) in place, one pass.  Block w publishes its sum (flag CS_AGG)
// and then its inclusive prefix (flag CS_PRE) in status[w]; its first wave looks back over
// predecessors 64 at a time.  Each status word carries the launch's epoch (read from the context
// state, advanced by the kernel that runs just before every scan), so words left by earlier
// launches read as "not yet published" and nothing needs clearing between launches.  Blocks are dispatched in
// index order, so every predecessor a block waits for is already running; every wait is still
// bounded (SPIN_LIMIT polls, then a stall flag), so the grid always drains.
// *mark_out (if not null) receives the exclusive prefix at index `mark`.  L_dev (if not null)
// holds the length, at most L; blocks past it leave at once (no block before them waits on them).
__global__ __launch_bounds__(CS_T) void k_chained_scan(uint32_t *__restrict__ data, int64_t L,
                                                       unsigned long long *__restrict__ status,
                                                       int64_t mark,
                                                       unsigned long long *__restrict__ mark_out,
                                                       DevState *state,
                                                       const unsigned long long *L_dev) {
    __shared__ unsigned long long s_prefix;
    __shared__ unsigned long long tmp[CS_T / 64 + 1];
    __shared__ uint32_t stage[CS_TILE + CS_TILE / 32];
    if (L_dev && (int64_t)*L_dev < L) L = (int64_t)*L_dev;
    const uint32_t w = blockIdx.x;
    if ((int64_t)w * CS_TILE >= L) return;
    const unsigned long long tag = (unsigned long long)(state->scan_epoch & 0x1fffffffu) << CS_EPOCH_SHIFT;
    const int64_t base = (int64_t)w * CS_TILE;
    {
        // all loads first, then the LDS stores: a load per guarded step would be awaited before
        // the next one is issued
        uint32_t x[CS_IPT];
        if (base + CS_TILE <= L) {
#pragma unroll
            for (int j = 0; j < CS_IPT; ++j) x[j] = data[base + j * CS_T + threadIdx.x];
        } else {
#pragma unroll
            for (int j = 0; j < CS_IPT; ++j) {
                const int64_t idx = base + j * CS_T + threadIdx.x;
                x[j] = idx < L ? data[idx] : 0u;
            }
        }
#pragma unroll
        for (int j = 0; j < CS_IPT; ++j) stage[spad(j * CS_T + threadIdx.x)] = x[j];
    }
    __syncthreads();
    uint32_t v[CS_IPT];
    unsigned long long sum = 0;
#pragma unroll
    for (int j = 0; j < CS_IPT; ++j) {
        v[j] = stage[spad(threadIdx.x * CS_IPT + j)];
        sum += v[j];
    }
    unsigned long long agg;
    const unsigned long long loc = block_exclusive_scan<unsigned long long, CS_T>(sum, tmp, &agg);
    if (threadIdx.x == 0) {
        // relaxed: the word carries all it publishes, nothing else needs ordering with it
        __hip_atomic_store(&status[w], tag | (w == 0 ? CS_PRE : CS_AGG) | (agg & CS_VAL),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (w == 0) s_prefix = 0;
    }
    if (w > 0 && threadIdx.x < 64) {
        // Each lane polls two predecessors (j - lane and j - 64 - lane), both reads issued before
        // either is awaited, so a launch of up to 129 blocks finds block 0's inclusive prefix in
        // its first window: one round trip to the status words instead of two.
        const int lane = threadIdx.x;
        unsigned long long excl = 0;
        int64_t j = (int64_t)w - 1;
        bool stalled = false;
        const unsigned long long before0 = tag | CS_PRE;  // before block 0: prefix 0
        auto published = [&](unsigned long long st) {
            return (st & CS_TAG_MASK) == tag && (st & CS_FLAG_MASK) != 0;
        };
        while (true) {
            const int64_t qa = j - lane, qb = j - 64 - lane;
            unsigned long long sa = load_status(&status[qa >= 0 ? qa : 0]);
            unsigned long long sb = load_status(&status[qb >= 0 ? qb : 0]);
            if (qa < 0) sa = before0;
            if (qb < 0) sb = before0;
            long spins = 0;
            while (!published(sa) && spins < SPIN_LIMIT) {
                sa = load_status(&status[qa]);
                ++spins;
            }
            spins = 0;
            while (!published(sb) && spins < SPIN_LIMIT) {
                sb = load_status(&status[qb]);
                ++spins;
            }
            if (!published(sa)) {
                stalled = true;
                sa = before0;
            }
            if (!published(sb)) {
                stalled = true;
                sb = before0;
            }
            const unsigned long long fa = (sa >> CS_FLAG_SHIFT) & 3ull, va = sa & CS_VAL;
            const unsigned long long fb = (sb >> CS_FLAG_SHIFT) & 3ull, vb = sb & CS_VAL;
            const unsigned long long ma = __ballot(fa == 2), mb = __ballot(fb == 2);
            unsigned long long contrib;
            if (ma) {  // the nearest inclusive prefix lies in the first half of the window
                const int first = __ffsll((long long)ma) - 1;
                contrib = lane <= first ? va : 0ull;
            } else if (mb) {
                const int first = __ffsll((long long)mb) - 1;
                contrib = va + (lane <= first ? vb : 0ull);
            } else {
                contrib = va + vb;
            }
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) contrib += __shfl_xor(contrib, d, 64);
            excl += contrib;
            if (ma | mb) break;
            j -= 128;
        }
        if (__ballot(stalled) && lane == 0) atomicOr(&state->flags, FLAG_SCAN_STALL);
        if (lane == 0) {
            __hip_atomic_store(&status[w], tag | CS_PRE | ((excl + agg) & CS_VAL),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_prefix = excl;
        }
    }
    __syncthreads();
    unsigned long long run = s_prefix + loc;
#pragma unroll
    for (int j = 0; j < CS_IPT; ++j) {
        const int64_t idx = base + threadIdx.x * CS_IPT + j;
        if (mark_out && idx == mark) *mark_out = run;
        stage[spad(threadIdx.x * CS_IPT + j)] = (uint32_t)run;
        run += v[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < CS_IPT; ++j) {
        const int64_t idx = base + j * CS_T + threadIdx.x;
        if (idx < L) data[idx] = stage[spad(j * CS_T + threadIdx.x)];
    }
}

// Lanes of the wave whose tile equals this lane's, deciding `nbits` bits.
// v of the neighbouring lane (lane ^ 1), by a DPP quad permutation [1, 0, 3, 2].
__device__ inline int dpp_swap_pair(int v) {
    return __builtin_amdgcn_update_dpp(0, v, 0xb1, 0xf, 0xf, false);
}

__device__ inline unsigned long long match_bits(uint32_t d, bool valid, int nbits) {
    unsigned long long peers = __ballot(valid);
    for (int b = 0; b < nbits; ++b) {
        const bool bit = (d >> b) & 1u;
        const unsigned long long bal = __ballot(bit);
        peers &= bit ? bal : ~bal;
    }
    return peers;
}

template <int FUSED_WAVES>
__global__ __launch_bounds__(64 * FUSED_WAVES) void k_fused_scatter(
    const uint32_t *__restrict__ count, const int4 *__restrict__ rect,
    const uint2 *__restrict__ tinfo, const float4 *__restrict__ proj,
    const uint32_t *__restrict__ scan, int64_t n, int32_t T, int32_t tbits, int64_t nchunk,
    int64_t cap, float4 *__restrict__ rec, uint32_t *__restrict__ slot,
    uint32_t *__restrict__ ids, uint2 *__restrict__ ranges, const float *__restrict__ opac,
    float *__restrict__ rec_o, DevState *state) {
    extern __shared__ uint32_t dyn[];  // wh [FUSED_WAVES][T], then tbase [T]
    uint32_t *wh = dyn;
    uint32_t *tbase = dyn + FUSED_WAVES * T;
    constexpr int NT = 64 * FUSED_WAVES;  // threads; the first FB own the chunk's Gaussians
    __shared__ unsigned long long tmp[NT / 64 + 1];
    __shared__ uint32_t pre[FB];
    __shared__ int4 srect[FB];
    __shared__ uint2 sinfo[FB];
    __shared__ uint32_t soff[FB];
    // m = ceil(2^32 / w) for each rectangle's width w: a key's row within its rectangle is
    // (i m) >> 32, exact while i < 2^32 / w (here i < w h <= 2048 and w <= 2048)
    __shared__ unsigned long long smag[FB];
    __shared__ float4 sproj[2 * FB];
    __shared__ uint8_t owner[OWN_CAP];  // chunk-local key -> its Gaussian, when the keys fit
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t chunk = xcd_chunk(blockIdx.x, (uint32_t)nchunk);
    const bool own = threadIdx.x < FB;
    const int64_t i = (int64_t)chunk * FB + threadIdx.x;  // this thread's Gaussian when own
    const bool mine = own && i < n;
    // Every global read of the set-up is issued before any of them is used (a read under a
    // branch, or in a guarded loop, would be awaited before the next is issued): lanes without
    // a Gaussian or a tile read a valid entry and drop it.
    const int64_t ir = mine ? i : 0;
    const uint32_t c_in = count[ir];
    const uint32_t K = scan[n];  // exclusive prefix after all Gaussian counts = key total
    const int4 rc_in = rect[ir];
    const uint2 inf_in = tinfo[ir];
    const uint32_t off_in = scan[ir];
    const float4 pa_in = proj[2 * ir], pb_in = proj[2 * ir + 1];  // one-pass: 32-byte stride
    // the first tile whose range this thread writes (tiles chunk, chunk + nchunk, ...): both
    // ends' scanned positions, read with the rest (indices clamped, values dropped if unused)
    const int64_t tr = chunk + (int64_t)threadIdx.x * nchunk;
    const int64_t tra = tr < T ? tr : T - 1, trb = tr + 1 < T ? tr + 1 : T - 1;
    const uint32_t ra_in = scan[n + tra * nchunk], rb_in = scan[n + trb * nchunk];
    constexpr int TB_MAX = (int)((FUSED_MAX_TILES + NT - 1) / NT);
    uint32_t tb_in[TB_MAX];
#pragma unroll
    for (int k = 0; k < TB_MAX; ++k) {
        const int t = (int)threadIdx.x + k * NT;
        tb_in[k] = scan[n + (int64_t)(t < T ? t : T - 1) * nchunk + chunk];
    }
    const uint32_t c = mine ? c_in : 0u;
    unsigned long long tot;
    const unsigned long long loc = block_exclusive_scan<unsigned long long, NT>(c, tmp, &tot);
    if (own) pre[threadIdx.x] = (uint32_t)loc;
    const bool table = tot <= OWN_CAP;  // same for the whole block
    if (table)
        for (uint32_t k = 0; k < c; ++k) owner[loc + k] = (uint8_t)threadIdx.x;
    if (mine) {
        const uint32_t wd = rc_in.z >= rc_in.x ? (uint32_t)(rc_in.z - rc_in.x + 1) : 1u;
        smag[threadIdx.x] = (unsigned long long)(0xffffffffu / wd) + 1ull;  // = ceil(2^32 / w)
        srect[threadIdx.x] = rc_in;
        sinfo[threadIdx.x] = inf_in;
        soff[threadIdx.x] = off_in;
        sproj[2 * threadIdx.x] = pa_in;
        sproj[2 * threadIdx.x + 1] = pb_in;
    }
    for (int k = threadIdx.x; k < FUSED_WAVES * T; k += NT) wh[k] = 0u;
    // first position of this chunk's keys of each tile, in tile order
#pragma unroll
    for (int k = 0; k < TB_MAX; ++k) {
        const int t = (int)threadIdx.x + k * NT;
        if (t < T) tbase[t] = tb_in[k] - K;
    }
    // tile ranges: this chunk writes tiles chunk, chunk + nchunk, ... (the first one per
    // thread from the values read above)
    for (int64_t t = tr; t < T; t += (int64_t)NT * nchunk) {
        uint32_t a = (t == tr ? ra_in : scan[n + t * nchunk]) - K;
        uint32_t b = t + 1 < T ? (t == tr ? rb_in : scan[n + (t + 1) * nchunk]) - K : K;
        if (a > cap) a = (uint32_t)cap;
        if (b > cap) b = (uint32_t)cap;
        ranges[t] = make_uint2(a, b);
    }
    __syncthreads();
    const uint32_t total = (uint32_t)tot;
    const uint32_t q = (total + FUSED_WAVES - 1) / FUSED_WAVES;
    const uint32_t j0 = (uint32_t)wave * q;
    const uint32_t j1 = j0 + q < total ? j0 + q : total;
    uint32_t *my = wh + wave * T;
    // pass 1: per-wave counts per tile
    for (uint32_t base = j0; base < j1; base += 64) {
        const uint32_t j = base + lane;
        const bool valid = j < j1;
        uint32_t t = 0;
        if (valid) {
            int lo;
            if (table) {
                lo = owner[j];
            } else {
                lo = 0;
                int hi = FB - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (pre[mid] <= j) lo = mid; else hi = mid - 1;
                }
            }
            const int4 r = srect[lo];
            const uint2 inf = sinfo[lo];
            const uint32_t li = j - pre[lo], wd = (uint32_t)(r.z - r.x + 1);
            const uint32_t q = (uint32_t)(((unsigned long long)li * smag[lo]) >> 32);
            t = inf.x + ((uint32_t)r.y + q) * inf.y + (uint32_t)r.x + (li - q * wd);
        }
        // counts only (order does not matter here): one LDS atomic per key
        if (valid) atomicAdd(&my[t], 1u);
    }
    __syncthreads();
    // wave offsets within the chunk, per tile, on top of the chunk's base in tile order
    for (int t = threadIdx.x; t < T; t += NT) {
        uint32_t run = tbase[t];
#pragma unroll
        for (int w = 0; w < FUSED_WAVES; ++w) {
            const uint32_t x = wh[w * T + t];
            wh[w * T + t] = run;
            run += x;
        }
    }
    __syncthreads();
    // pass 2: stable ranks and the writes into tile order
    bool overflow = false;
    for (uint32_t base = j0; base < j1; base += 64) {
        const uint32_t j = base + lane;
        const bool valid = j < j1;
        uint32_t t = 0, li = 0;
        int g = 0;
        if (valid) {
            int lo;
            if (table) {
                lo = owner[j];
            } else {
                lo = 0;
                int hi = FB - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (pre[mid] <= j) lo = mid; else hi = mid - 1;
                }
            }
            g = lo;
            const int4 r = srect[lo];
            const uint2 inf = sinfo[lo];
            li = j - pre[lo];
            const uint32_t wd = (uint32_t)(r.z - r.x + 1);
            const uint32_t q = (uint32_t)(((unsigned long long)li * smag[lo]) >> 32);
            t = inf.x + ((uint32_t)r.y + q) * inf.y + (uint32_t)r.x + (li - q * wd);
        }
        const unsigned long long peers = match_bits(t, valid, tbits);
        const unsigned long long lt = (1ull << lane) - 1ull;
        const uint32_t old = valid ? my[t] : 0u;
        if (valid && lane == __ffsll((long long)peers) - 1) my[t] = old + __popcll(peers);
        const uint32_t pos = old + __popcll(peers & lt);
        const bool ok = valid && pos < cap;
        if (valid && !ok) overflow = true;
        if (ok) {
            // on key overflow a key below the capacity in tile order can lie above it in
            // Gaussian order; its partial sums then go to the last slot (the update is skipped
            // on overflow), never past the buffer
            const uint32_t sl = soff[g] + li;
            if (slot) slot[pos] = sl < cap ? sl : (uint32_t)(cap - 1);
            if (ids) ids[pos] = chunk * FB + (uint32_t)g;
            if (rec_o) rec_o[pos] = opac[(int64_t)chunk * FB + g];
        }
        // The 32-byte records go out two lanes per record: lanes 2m and 2m + 1 write the two
        // halves of lane 2m's record, then of lane 2m + 1's, so each store touches 32 records
        // instead of 64 (the partner's key comes over by a DPP swap of neighbouring lanes).
        const bool odd = lane & 1;
        const int pg = dpp_swap_pair(g);
        const uint32_t ppos = (uint32_t)dpp_swap_pair((int)pos);
        const bool pok = dpp_swap_pair(ok ? 1 : 0) != 0;
        {
            const int gg = odd ? pg : g;
            const uint32_t pp = odd ? ppos : pos;
            if (odd ? pok : ok) rec[2 * (int64_t)pp + odd] = sproj[2 * gg + odd];
        }
        {
            const int gg = odd ? g : pg;
            const uint32_t pp = odd ? pos : ppos;
            if (odd ? ok : pok) rec[2 * (int64_t)pp + !odd] = sproj[2 * gg + !odd];
        }
    }
    if (__ballot(overflow) && lane == 0) atomicOr(&state->flags, FLAG_KEY_OVERFLOW);
}

// ---- row binning: a counting sort in two levels, for many tiles ------------------------------
//
// Level one puts the (global tile row, Gaussian) pairs into row order (a Gaussian's rectangle
// spans a few rows, so there are far fewer pairs than keys): k_project counts each block's pairs
// per row, one chained scan gives each block's first position in every row, and k_rows_scatter
// writes the pairs there, in Gaussian order within a row.  Level two
// cuts every row's pairs (in Gaussian order) into chunks of ROW_CHUNK: k_row_table numbers the
// chunks and lays out one count per (row, column, chunk), row-major, then column, then chunk;
// k_row_hist fills the counts, one chained scan turns them into the first position of every
// chunk's keys of every tile (that order is tile order), and k_row_scatter ranks each chunk's
// keys per column in Gaussian order and writes records, slots and ranges there.  The result is
// that of the stable sort of all keys by tile.

// Level one.  Block b handles Gaussians [256 b, 256 b + 256): their key offsets (slot bases, in
// `off`), rebuilt from the scanned block sums, and their (row, Gaussian) pairs, enumerated in
// Gaussian order (a pair finds its Gaussian in an LDS table, one byte per pair, when the block's
// pairs fit, else by binary search), ranked stably per row by the waves (ballots on the row bits,
// per-wave counters, two passes) and written at the block's scanned first position in each row:
// the pairs in row order, and in Gaussian order within a row.
constexpr uint32_t PAIR_OWN_CAP = 8192;
__global__ __launch_bounds__(BLK) void k_rows_scatter(const uint32_t *__restrict__ count,
                                                      const float4 *__restrict__ proj,
                                                      const unsigned long long *__restrict__ bs,
                                                      const uint32_t *__restrict__ rscan,
                                                      const uint4 *__restrict__ bwin,
                                                      ImgTable tab, int64_t n, int64_t cap,
                                                      uint32_t *__restrict__ off,
                                                      uint32_t *__restrict__ rvals,
                                                      DevState *state) {
    constexpr int WV = BLK / 64;
    __shared__ unsigned long long tmp[BLK / 64 + 1];
    __shared__ uint32_t pre[BLK];
    __shared__ uint32_t srow[BLK];                 // first window row of each Gaussian
    __shared__ uint8_t owner[PAIR_OWN_CAP];
    __shared__ uint32_t wh[WV][ROW_WIN_MAX];       // per-wave counts, then wave offsets
    __shared__ uint32_t rbase[ROW_WIN_MAX];        // the block's first position in each row
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x;
    const int64_t ir = i < n ? i : n - 1;
    // reads issued together (clamped index), used after
    const uint32_t c_in = count[ir];
    const uint4 rl = __builtin_bit_cast(uint4, proj[PROJ_F4 * ir + 3]);  // first row, rows
    const unsigned long long kbase = bs[blockIdx.x];
    const uint4 win = bwin[blockIdx.x];
    const uint32_t w0 = win.x, W = win.y;
    const uint32_t blocks = (uint32_t)gridDim.x;
    constexpr int RB_MAX = ROW_WIN_MAX / BLK;
    uint32_t rb_in[RB_MAX];
#pragma unroll
    for (int k = 0; k < RB_MAX; ++k) {
        const uint32_t r = threadIdx.x + k * BLK;
        const uint32_t row = w0 + (r < W ? r : W - 1), fb = row_fb_of(tab, row);
        // (rows of an image without Gaussians hold no pairs and have no counts: index 0, dropped)
        const bool has = fb != 0xffffffffu;
        const uint32_t v = rscan[has ? row_seg_of(tab, row, blocks) + (blockIdx.x - fb) : 0ull];
        rb_in[k] = has ? v : 0u;
    }
    const uint32_t c = i < n ? c_in : 0u;
    const uint32_t h = i < n ? rl.y : 0u;
    unsigned long long ktot, rtot;
    const unsigned long long kloc = block_exclusive_scan<unsigned long long, BLK>(c, tmp, &ktot);
    const unsigned long long rloc = block_exclusive_scan<unsigned long long, BLK>(h, tmp, &rtot);
    const bool table = rtot <= PAIR_OWN_CAP;  // the same for the whole block
    if (table)
        for (uint32_t k = 0; k < h; ++k) owner[rloc + k] = (uint8_t)threadIdx.x;
    pre[threadIdx.x] = (uint32_t)rloc;
    srow[threadIdx.x] = rl.x - w0;
    if (i < n) off[i] = (uint32_t)(kbase + kloc);
#pragma unroll
    for (int k = 0; k < RB_MAX; ++k) {
        const uint32_t r = threadIdx.x + k * BLK;
        if (r < W) rbase[r] = rb_in[k];
    }
    for (int k = threadIdx.x; k < WV * ROW_WIN_MAX; k += BLK) (&wh[0][0])[k] = 0u;
    __syncthreads();
    int rbits = 1;
    while ((1u << rbits) < W) ++rbits;
    const uint32_t total = (uint32_t)rtot;
    const uint32_t q = (total + WV - 1) / WV;
    const uint32_t j0 = (uint32_t)wave * q < total ? (uint32_t)wave * q : total;
    const uint32_t j1 = j0 + q < total ? j0 + q : total;
    uint32_t *my = wh[wave];
    // pass 1: per-wave counts per row
    for (uint32_t base = j0; base < j1; base += 64) {
        const uint32_t j = base + lane;
        const bool valid = j < j1;
        uint32_t r = 0;
        if (valid) {
            int lo = 0;
            if (table) {
                lo = owner[j];
            } else {
                int hi = BLK - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (pre[mid] <= j) lo = mid; else hi = mid - 1;
                }
            }
            r = srow[lo] + (j - pre[lo]);
        }
        // counts only (order does not matter here): one LDS atomic per key
        if (valid) atomicAdd(&my[r], 1u);
    }
    __syncthreads();
    for (uint32_t r = threadIdx.x; r < W; r += BLK) {
        uint32_t run = rbase[r];
#pragma unroll
        for (int v = 0; v < WV; ++v) {
            const uint32_t x = wh[v][r];
            wh[v][r] = run;
            run += x;
        }
    }
    __syncthreads();
    // pass 2: stable ranks and the writes
    bool overflow = false;
    for (uint32_t base = j0; base < j1; base += 64) {
        const uint32_t j = base + lane;
        const bool valid = j < j1;
        uint32_t r = 0;
        int lo = 0;
        if (valid) {
            if (table) {
                lo = owner[j];
            } else {
                int hi = BLK - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (pre[mid] <= j) lo = mid; else hi = mid - 1;
                }
            }
            r = srow[lo] + (j - pre[lo]);
        }
        const unsigned long long peers = match_bits(r, valid, rbits);
        const unsigned long long lt = (1ull << lane) - 1ull;
        const uint32_t old = valid ? my[r] : 0u;
        if (valid && lane == __ffsll((long long)peers) - 1) my[r] = old + __popcll(peers);
        const uint32_t pos = old + __popcll(peers & lt);
        if (valid) {
            if (pos < cap) rvals[pos] = (uint32_t)((int64_t)blockIdx.x * BLK + lo);
            else overflow = true;
        }
    }
    if (__ballot(overflow) && lane == 0) atomicOr(&state->flags, FLAG_KEY_OVERFLOW);
}

// First global tile and tiles per row of global tile row r.
__device__ inline uint2 row_tiles(const ImgTable &t, uint32_t r) {
    if (t.B == 1) return make_uint2(r * (uint32_t)t.TW, (uint32_t)t.TW);
    return t.row_tiles[r];
}

constexpr int RT_T = 1024;  // threads of the row table
constexpr int RT_PER = 8;   // rows per thread and round

// One block.  Rows in rounds of RT_T * RT_PER (each thread RT_PER consecutive rows): chunk
// counts and count-array sizes, scanned with the totals of earlier rounds carried; rinfo per
// row; the row of every chunk (found by binary search over the round's chunk bases in LDS).
// The count array gets one more entry, a zero, so that its scan ends with the total of the
// keys written.  On overflow of the bounds the kernels after it see zero chunks and the
// overflow flag is set.
__global__ __launch_bounds__(RT_T) void k_row_table(const uint32_t *__restrict__ rscan,
                                                    uint32_t blocks, int64_t pcap, ImgTable tab,
                                                    int64_t rows, int64_t nch_max,
                                                    int64_t scan_max, uint4 *__restrict__ rinfo,
                                                    uint32_t *__restrict__ chunk_row,
                                                    uint32_t *__restrict__ scan,
                                                    DevState *state) {
    __shared__ unsigned long long tmp[RT_T / 64 + 1];
    __shared__ uint32_t lcb[RT_T * RT_PER];
    unsigned long long cc = 0, cs = 0;  // chunks and counts of earlier rounds
    for (int64_t r0 = 0; r0 < rows; r0 += RT_T * RT_PER) {
        const int64_t nr = rows - r0 < RT_T * RT_PER ? rows - r0 : RT_T * RT_PER;
        uint2 rr[RT_PER], rt[RT_PER];
#pragma unroll
        for (int j = 0; j < RT_PER; ++j) {
            int64_t q = (int64_t)threadIdx.x * RT_PER + j;
            q = r0 + (q < nr ? q : nr - 1);
            // the row's pairs: from its first block's scanned position to the next row's, cut at
            // the pair capacity (pairs beyond it were not written; the overflow flag is set)
            const unsigned long long a = rscan[row_seg_of(tab, (uint32_t)q, blocks)];
            const unsigned long long b = rscan[row_seg_of(tab, (uint32_t)q + 1, blocks)];
            rr[j] = make_uint2((uint32_t)(a < (unsigned long long)pcap ? a : pcap),
                               (uint32_t)(b < (unsigned long long)pcap ? b : pcap));
            rt[j] = row_tiles(tab, (uint32_t)q);
        }
        uint32_t nch[RT_PER];
        unsigned long long sc = 0, ss = 0;
#pragma unroll
        for (int j = 0; j < RT_PER; ++j) {
            const bool ok = (int64_t)threadIdx.x * RT_PER + j < nr && rr[j].y > rr[j].x;
            nch[j] = ok ? (rr[j].y - rr[j].x + ROW_CHUNK - 1) / ROW_CHUNK : 0u;
            sc += nch[j];
            ss += (unsigned long long)nch[j] * rt[j].y;
        }
        unsigned long long tc, ts;
        unsigned long long cb = cc + block_exclusive_scan<unsigned long long, RT_T>(sc, tmp, &tc);
        unsigned long long sb = cs + block_exclusive_scan<unsigned long long, RT_T>(ss, tmp, &ts);
#pragma unroll
        for (int j = 0; j < RT_PER; ++j) {
            const int64_t q = (int64_t)threadIdx.x * RT_PER + j;
            if (q < nr) {
                rinfo[2 * (r0 + q)] = make_uint4(rr[j].x, rr[j].x + (nch[j] ? rr[j].y - rr[j].x : 0u),
                                                 (uint32_t)cb, (uint32_t)sb);
                rinfo[2 * (r0 + q) + 1] = make_uint4(rt[j].x, rt[j].y, nch[j], 0u);
                lcb[q] = (uint32_t)(cb - cc);
            }
            cb += nch[j];
            sb += (unsigned long long)nch[j] * rt[j].y;
        }
        __syncthreads();
        // the row of each of this round's chunks: the last row whose first chunk is at most it
        // (rows without chunks share the next row's first chunk and come before it)
        for (unsigned long long k = threadIdx.x; k < tc; k += RT_T) {
            int lo = 0, hi = (int)nr - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (lcb[mid] <= (uint32_t)k) lo = mid; else hi = mid - 1;
            }
            if (cc + k < (unsigned long long)nch_max) chunk_row[cc + k] = (uint32_t)(r0 + lo);
        }
        __syncthreads();
        cc += tc;
        cs += ts;
    }
    if (threadIdx.x == 0) {
        const bool fits = cc <= (unsigned long long)nch_max && cs < (unsigned long long)scan_max;
        if (fits) scan[cs] = 0u;
        state->row_chunks = fits ? (uint32_t)cc : 0u;
        state->row_scan_len = fits ? cs + 1 : 0ull;
        if (!fits) atomicOr(&state->flags, FLAG_KEY_OVERFLOW);
    }
}

// Chunk-local key -> its pair (one byte while a chunk has at most 256 pairs), for chunks of up
// to ROW_OWN_CAP keys (else binary search).
using RowOwner = typename std::conditional<(ROW_CHUNK <= 256), uint8_t, uint16_t>::type;
constexpr uint32_t ROW_OWN_CAP = 16 * ROW_CHUNK;
constexpr int ROW_WAVES = ROW_CHUNK / 64;  // scatter waves: one thread per pair

// The chunk of workgroup blockIdx.x (contiguous ranges of chunks per XCD, so that a row's
// chunks share an L2), its row and the row's table entries.
struct RowChunk {
    uint32_t k;      // chunk within the row
    uint32_t first;  // first pair of the chunk
    uint32_t pairs;  // pairs in the chunk (1 .. ROW_CHUNK)
    uint32_t sofs;   // the row's first count
    uint32_t nch;    // the row's chunks
    uint32_t tile0;  // the row's first global tile
    uint32_t tw;     // the row's tiles
    uint32_t row;
};

__device__ inline RowChunk row_chunk(const uint4 *__restrict__ rinfo,
                                     const uint32_t *__restrict__ chunk_row, uint32_t nc) {
    RowChunk rc;
    const uint32_t c = xcd_chunk(blockIdx.x, nc);
    rc.row = chunk_row[c];
    const uint4 a = rinfo[2 * rc.row], b = rinfo[2 * rc.row + 1];
    rc.k = c - a.z;
    rc.first = a.x + rc.k * ROW_CHUNK;
    rc.pairs = a.y - rc.first < (uint32_t)ROW_CHUNK ? a.y - rc.first : (uint32_t)ROW_CHUNK;
    rc.sofs = a.w;
    rc.nch = b.z;
    rc.tile0 = b.x;
    rc.tw = b.y;
    return rc;
}

// Per chunk: the number of its Gaussians covering each column of the row (a difference array:
// +1 at the rectangle's first column, -1 after its last, then the prefix sums), stored at
// scan[sofs + column * nch + k].
__global__ __launch_bounds__(ROW_CHUNK) void k_row_hist(const uint32_t *__restrict__ rvals,
                                                        const uint4 *__restrict__ rinfo,
                                                        const uint32_t *__restrict__ chunk_row,
                                                        const float4 *__restrict__ proj,
                                                        uint32_t *__restrict__ scan,
                                                        DevState *state) {
    __shared__ uint32_t d[ROW_MAX_TW + 1];
    __shared__ unsigned long long tmp[ROW_CHUNK / 64 + 1];
    // a new epoch for the scan that follows (see k_chained_scan)
    if (blockIdx.x == 0 && threadIdx.x == 0) state->scan_epoch += 1u;
    const uint32_t nc = state->row_chunks;
    if (blockIdx.x >= nc) return;
    const RowChunk rc = row_chunk(rinfo, chunk_row, nc);
    const uint32_t e = rc.first + (threadIdx.x < rc.pairs ? threadIdx.x : 0u);
    const uint32_t g = rvals[e];
    const uint4 f = __builtin_bit_cast(uint4, proj[PROJ_F4 * (int64_t)g + 2]);
    for (uint32_t x = threadIdx.x; x <= rc.tw; x += ROW_CHUNK) d[x] = 0u;
    __syncthreads();
    if (threadIdx.x < rc.pairs) {
        const uint32_t x0 = f.w & 0xffffu, w = f.z >> 16;
        atomicAdd(&d[x0], 1u);
        atomicSub(&d[x0 + w], 1u);
    }
    __syncthreads();
    // prefix sums: thread t takes columns [t per, t per + per)
    const uint32_t per = (rc.tw + ROW_CHUNK - 1) / ROW_CHUNK;
    const uint32_t x0 = threadIdx.x * per;
    uint32_t s = 0;
    for (uint32_t x = x0; x < x0 + per && x < rc.tw; ++x) s += d[x];
    unsigned long long tot;
    uint32_t run = (uint32_t)block_exclusive_scan<unsigned long long, ROW_CHUNK>(s, tmp, &tot);
    for (uint32_t x = x0; x < x0 + per && x < rc.tw; ++x) {
        run += d[x];
        scan[rc.sofs + (int64_t)x * rc.nch + rc.k] = run;
    }
}

// Per chunk: its keys in Gaussian order (a pair's keys are its columns left to right), ranked
// stably per column by the waves (each takes a contiguous share), written at the scanned
// positions: the records, slots, Gaussian ids and opacities wanted; the first chunk of a row
// also writes the row's tile ranges.
template <int WV>
__global__ __launch_bounds__(64 * WV) void k_row_scatter(
    const uint32_t *__restrict__ rvals, const uint4 *__restrict__ rinfo,
    const uint32_t *__restrict__ chunk_row, const float4 *__restrict__ proj,
    const uint32_t *__restrict__ scan, const uint32_t *__restrict__ off, int64_t cap,
    float4 *__restrict__ rec,
    uint32_t *__restrict__ slot, uint32_t *__restrict__ ids, uint2 *__restrict__ ranges,
    const float *__restrict__ opac, float *__restrict__ rec_o, DevState *state) {
    extern __shared__ uint32_t dyn[];  // wh [WV][tw], tbase [tw], lcs [tw]
    constexpr int NT = 64 * WV;
    static_assert(NT >= ROW_CHUNK, "one thread per pair of a chunk");
    static_assert(ROW_CHUNK <= 256, "staged positions hold the pair in 8 bits");
    __shared__ unsigned long long tmp[NT / 64 + 1];
    __shared__ uint32_t pre[ROW_CHUNK];
    __shared__ uint32_t sx0[ROW_CHUNK];    // first column
    __shared__ uint32_t sbase[ROW_CHUNK];  // slot of the key in column 0 (modulo 2^32)
    __shared__ float4 sproj[2 * ROW_CHUNK];
    __shared__ RowOwner owner[ROW_OWN_CAP];
    // chunk-local position in tile order -> pair | (column - first column) << 8
    __shared__ uint16_t inv[ROW_OWN_CAP];
    const uint32_t nc = state->row_chunks;
    if (blockIdx.x >= nc) return;
    const RowChunk rc = row_chunk(rinfo, chunk_row, nc);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t tw = rc.tw;
    uint32_t *wh = dyn;
    uint32_t *tbase = dyn + WV * tw;
    uint32_t *lcs = tbase + tw;  // chunk-local first position of each column
    // set-up reads issued together (clamped indices), used after
    const bool mine = threadIdx.x < rc.pairs;
    const uint32_t g = rvals[rc.first + (mine ? threadIdx.x : 0u)];
    const float4 pa = proj[PROJ_F4 * (int64_t)g], pb = proj[PROJ_F4 * (int64_t)g + 1];
    const uint4 f = __builtin_bit_cast(uint4, proj[PROJ_F4 * (int64_t)g + 2]);
    const uint4 rl = __builtin_bit_cast(uint4, proj[PROJ_F4 * (int64_t)g + 3]);
    const uint32_t koff = off[g];  // the Gaussian's first slot
    constexpr int TB_MAX = (ROW_MAX_TW + NT - 1) / NT;
    uint32_t tb_in[TB_MAX];
#pragma unroll
    for (int k = 0; k < TB_MAX; ++k) {
        const uint32_t x = threadIdx.x + k * NT;
        tb_in[k] = scan[rc.sofs + (int64_t)(x < tw ? x : tw - 1) * rc.nch + rc.k];
    }
    const uint32_t w = mine ? f.z >> 16 : 0u;
    unsigned long long tot;
    const unsigned long long loc = block_exclusive_scan<unsigned long long, NT>(w, tmp, &tot);
    // the staged path: the chunk's keys fit the tables and every rectangle is at most 256
    // tiles wide (the same for the whole block)
    const bool table = __syncthreads_and(tot <= ROW_OWN_CAP && w <= 256u) != 0;
    if (table)
        for (uint32_t k = 0; k < w; ++k) owner[loc + k] = (RowOwner)threadIdx.x;
    if (mine) {
        const uint32_t x0 = f.w & 0xffffu;
        pre[threadIdx.x] = (uint32_t)loc;
        sx0[threadIdx.x] = x0;
        // slot = key offset + (row - first row) w + (column - first column)
        sbase[threadIdx.x] = koff + (rc.row - rl.x) * w - x0;
        sproj[2 * threadIdx.x] = pa;
        sproj[2 * threadIdx.x + 1] = pb;
    } else if (threadIdx.x < ROW_CHUNK) {
        pre[threadIdx.x] = 0xffffffffu;  // never the owner of a key
    }
    for (uint32_t k = threadIdx.x; k < WV * tw; k += NT) wh[k] = 0u;
#pragma unroll
    for (int k = 0; k < TB_MAX; ++k) {
        const uint32_t x = threadIdx.x + k * NT;
        if (x < tw) tbase[x] = tb_in[k];
    }
    // the row's tile ranges, by its first chunk (a tile ends where the next count begins;
    // after the last row that is the closing zero entry, i.e. the total)
    if (rc.k == 0) {
        for (uint32_t x = threadIdx.x; x < tw; x += NT) {
            const int64_t ia = rc.sofs + (int64_t)x * rc.nch, ib = ia + rc.nch;
            unsigned long long a = scan[ia];
            unsigned long long b = scan[ib];
            if (a > (unsigned long long)cap) a = (unsigned long long)cap;
            if (b > (unsigned long long)cap) b = (unsigned long long)cap;
            ranges[rc.tile0 + x] = make_uint2((uint32_t)a, (uint32_t)b);
        }
    }
    __syncthreads();
    int xbits = 1;
    while ((1u << xbits) < tw) ++xbits;
    const uint32_t total = (uint32_t)tot;
    const uint32_t q = (total + WV - 1) / WV;
    const uint32_t j0 = (uint32_t)wave * q < total ? (uint32_t)wave * q : total;
    const uint32_t j1 = j0 + q < total ? j0 + q : total;
    uint32_t *my = wh + wave * tw;
    // pass 1: per-wave counts per column
    for (uint32_t base = j0; base < j1; base += 64) {
        const uint32_t j = base + lane;
        const bool valid = j < j1;
        uint32_t x = 0;
        if (valid) {
            int lo;
            if (table) {
                lo = owner[j];
            } else {
                lo = 0;
                int hi = ROW_CHUNK - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (pre[mid] <= j) lo = mid; else hi = mid - 1;
                }
            }
            x = sx0[lo] + (j - pre[lo]);
        }
        // counts only (order does not matter here): one LDS atomic per key
        if (valid) atomicAdd(&my[x], 1u);
    }
    __syncthreads();
    if (table) {
        // Staged: the chunk's keys are ranked into chunk-local positions in tile order (LDS),
        // then written out in that order, so that each column's keys go out as one contiguous
        // run and the stores are coalesced.  Wave offsets within each column's run, the
        // chunk's count per column, and the columns' chunk-local starts:
        const uint32_t per = (tw + NT - 1) / NT, cx0 = threadIdx.x * per;
        const uint32_t cx1 = cx0 + per < tw ? cx0 + per : tw;
        uint32_t csum = 0;
        for (uint32_t x = cx0; x < cx1; ++x) {
            uint32_t run = 0;
#pragma unroll
            for (int v = 0; v < WV; ++v) {
                const uint32_t c = wh[v * tw + x];
                wh[v * tw + x] = run;
                run += c;
            }
            lcs[x] = run;
            csum += run;
        }
        unsigned long long ctot;
        uint32_t run = (uint32_t)block_exclusive_scan<unsigned long long, NT>(csum, tmp, &ctot);
        for (uint32_t x = cx0; x < cx1; ++x) {
            const uint32_t c = lcs[x];
            lcs[x] = run;
            run += c;
        }
        __syncthreads();
        // pass 2: stable ranks, as chunk-local positions
        for (uint32_t base = j0; base < j1; base += 64) {
            const uint32_t j = base + lane;
            const bool valid = j < j1;
            const int e = valid ? (int)owner[j] : 0;
            const uint32_t x = valid ? sx0[e] + (j - pre[e]) : 0u;
            const unsigned long long peers = match_bits(x, valid, xbits);
            const unsigned long long lt = (1ull << lane) - 1ull;
            const uint32_t old = valid ? my[x] : 0u;
            if (valid && lane == __ffsll((long long)peers) - 1) my[x] = old + __popcll(peers);
            if (valid)
                inv[lcs[x] + old + __popcll(peers & lt)] = (uint16_t)(e | ((x - sx0[e]) << 8));
        }
        __syncthreads();
        // pass 3: the writes, in tile order
        bool overflow = false;
        for (uint32_t base = 0; base < total; base += NT) {
            const uint32_t j = base + threadIdx.x;
            const bool valid = j < total;
            const uint32_t v = inv[valid ? j : 0u];
            const int e = (int)(v & 0xffu);
            const uint32_t x = sx0[e] + (v >> 8);
            const uint32_t pos = tbase[x] + (j - lcs[x]);
            const bool ok = valid && pos < cap;
            if (valid && !ok) overflow = true;
            if (ok) {
                const uint32_t sl = sbase[e] + x;  // kept below the capacity, as in k_fused_scatter
                if (slot) slot[pos] = sl < cap ? sl : (uint32_t)(cap - 1);
                if (ids || rec_o) {
                    const uint32_t g = rvals[rc.first + e];
                    if (ids) ids[pos] = g;
                    if (rec_o) rec_o[pos] = opac[g];
                }
            }
            // records two lanes per record (see k_fused_scatter): consecutive lanes hold
            // consecutive positions, so each store covers a contiguous stretch
            const bool odd = lane & 1;
            const int pe = dpp_swap_pair(e);
            const uint32_t ppos = (uint32_t)dpp_swap_pair((int)pos);
            const bool pok = dpp_swap_pair(ok ? 1 : 0) != 0;
            {
                const int ee = odd ? pe : e;
                const uint32_t pp = odd ? ppos : pos;
                if (odd ? pok : ok) rec[2 * (int64_t)pp + odd] = sproj[2 * ee + odd];
            }
            {
                const int ee = odd ? e : pe;
                const uint32_t pp = odd ? pos : ppos;
                if (odd ? ok : pok) rec[2 * (int64_t)pp + !odd] = sproj[2 * ee + !odd];
            }
        }
        if (__ballot(overflow) && lane == 0) atomicOr(&state->flags, FLAG_KEY_OVERFLOW);
        return;
    }
    // wave offsets per column, on top of the chunk's first position in the column's tile
    for (uint32_t x = threadIdx.x; x < tw; x += NT) {
        uint32_t run = tbase[x];
#pragma unroll
        for (int v = 0; v < WV; ++v) {
            const uint32_t c = wh[v * tw + x];
            wh[v * tw + x] = run;
            run += c;
        }
    }
    __syncthreads();
    // pass 2: stable ranks and the writes into tile order
    bool overflow = false;
    for (uint32_t base = j0; base < j1; base += 64) {
        const uint32_t j = base + lane;
        const bool valid = j < j1;
        uint32_t x = 0;
        int e = 0;
        if (valid) {
            int lo;
            if (table) {
                lo = owner[j];
            } else {
                lo = 0;
                int hi = ROW_CHUNK - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (pre[mid] <= j) lo = mid; else hi = mid - 1;
                }
            }
            e = lo;
            x = sx0[lo] + (j - pre[lo]);
        }
        const unsigned long long peers = match_bits(x, valid, xbits);
        const unsigned long long lt = (1ull << lane) - 1ull;
        const uint32_t old = valid ? my[x] : 0u;
        if (valid && lane == __ffsll((long long)peers) - 1) my[x] = old + __popcll(peers);
        const uint32_t pos = old + __popcll(peers & lt);
        const bool ok = valid && pos < cap;
        if (valid && !ok) overflow = true;
        if (ok) {
            const uint32_t sl = sbase[e] + x;  // kept below the capacity, as in k_fused_scatter
            if (slot) slot[pos] = sl < cap ? sl : (uint32_t)(cap - 1);
            if (ids || rec_o) {
                const uint32_t g = rvals[rc.first + e];
                if (ids) ids[pos] = g;
                if (rec_o) rec_o[pos] = opac[g];
            }
        }
        // records two lanes per record (see k_fused_scatter)
        const bool odd = lane & 1;
        const int pe = dpp_swap_pair(e);
        const uint32_t ppos = (uint32_t)dpp_swap_pair((int)pos);
        const bool pok = dpp_swap_pair(ok ? 1 : 0) != 0;
        {
            const int ee = odd ? pe : e;
            const uint32_t pp = odd ? ppos : pos;
            if (odd ? pok : ok) rec[2 * (int64_t)pp + odd] = sproj[2 * ee + odd];
        }
        {
            const int ee = odd ? e : pe;
            const uint32_t pp = odd ? pos : ppos;
            if (odd ? ok : pok) rec[2 * (int64_t)pp + !odd] = sproj[2 * ee + !odd];
        }
    }
    if (__ballot(overflow) && lane == 0) atomicOr(&state->flags, FLAG_KEY_OVERFLOW);
}

inline unsigned grid_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

// Compressed set -> float records [N][8]; a Gaussian with an invalid code or index gets NaN
// in every slot (so that rendering the records leaves it out, as the fused decode does).
__global__ __launch_bounds__(BLK) void k_codec_decode(const CodecArgs c, int64_t n,
                                                      float4 *__restrict__ out,
                                                      DevState *state) {
    const int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x;
    bool bad = false;
    if (i < n) {
        RecordSrc src;
        src.params = nullptr;
        src.codec = c;
        float q[8];
        bad = !load_record(src, i, q);
        if (bad) {
#pragma unroll
            for (int k = 0; k < 8; ++k) q[k] = __builtin_nanf("");
        }
        out[2 * i] = make_float4(q[0], q[1], q[2], q[3]);
        out[2 * i + 1] = make_float4(q[4], q[5], q[6], q[7]);
    }
    if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(&state->flags, FLAG_BAD_CODE);
}

}  // namespace

// ---- launchers -----------------------------------------------------------------------------

hipError_t launch_codec_decode(const CodecArgs &c, int64_t n, float *params, DevState *state,
                               hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_codec_decode, dim3(grid_for(n, BLK)), dim3(BLK), 0, s, c, n,
                       reinterpret_cast<float4 *>(params), state);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, BLK)), dim3(BLK), 0, s, p, v, n);
    return hipGetLastError();
}

static RecordSrc record_src(const BinBuffers &b) {
    RecordSrc r;
    memset(&r, 0, sizeof(r));
    r.params = reinterpret_cast<const float4 *>(b.params);
    if (b.codec) r.codec = *b.codec;
    r.opacity = b.opacity;
    r.blend = b.blend;
    r.recipe = b.recipe;
    r.qat = b.qat;
    return r;
}

hipError_t launch_project(const BinBuffers &b, const ImgTable &tab, hipStream_t s) {
    if (b.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_project, dim3(grid_for(b.n, BLK)), dim3(BLK), 0, s, record_src(b), b.n, tab,
                       reinterpret_cast<float4 *>(b.proj), b.rect, b.tinfo, b.count, b.blocksum,
                       RowHistArgs{nullptr, 0, nullptr}, b.state);
    return hipGetLastError();
}

hipError_t launch_count_scan(const BinBuffers &b, hipStream_t s) {
    if (b.n <= 0) {
        // zero keys: write the total directly (a fill kernel, so that graphs hold no memset)
        return launch_fill_u32(reinterpret_cast<uint32_t *>(&b.state->keys_total), 0u, 2, s);
    }
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, b.blocksum,
                       (int64_t)grid_for(b.n, BLK), &b.state->keys_total, nullptr, nullptr);
    return hipGetLastError();
}

hipError_t launch_duplicate(const BinBuffers &b, hipStream_t s) {
    if (b.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_duplicate, dim3(grid_for(b.n, BLK)), dim3(BLK), 0, s, b.count, b.rect,
                       b.tinfo, b.blocksum, b.n, b.cap, b.off, b.keys[0], b.vals[0],
                       reinterpret_cast<float4 *>(b.proj), b.state);
    return hipGetLastError();
}

int64_t scan_scratch_entries(int64_t n) { return n <= 16384 ? 1 : (n + SCAN_TILE - 1) / SCAN_TILE; }

hipError_t launch_scan_u32(const uint32_t *in, uint32_t *out, int64_t n,
                           unsigned long long *blocksum, unsigned long long *total,
                           hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (n <= 16384) {
        hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(1024), 0, s, in, out, n, total);
        return hipGetLastError();
    }
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(SCAN_T), 0, s, in, n, blocksum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, blocksum, nb, total, nullptr,
                       nullptr);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(SCAN_T), 0, s, in, out, n, blocksum);
    return hipGetLastError();
}

int auto_digit_bits(int key_bits, int64_t n) {
    if (key_bits <= 0) return 1;
    if (key_bits <= 11 && n <= (int64_t)1 << 22) return key_bits;  // one counting pass
    const int passes = (key_bits + 7) / 8;
    return (key_bits + passes - 1) / passes;
}

int64_t sort_hist_entries(int64_t n, int digit_bits) {
    const int64_t nblk = n > 0 ? (n + SORT_TILE - 1) / SORT_TILE : 1;
    return nblk << digit_bits;
}

template <int BITS>
static hipError_t sort_pass(const uint32_t *kin, const uint32_t *vin, uint32_t *kout, uint32_t *vout,
                      int64_t n, const unsigned long long *n_dev, int shift, uint32_t *hist,
                      unsigned long long *scan_bs, const ChainedScan &cs, hipStream_t s) {
    const int64_t nblk = (n + SORT_TILE - 1) / SORT_TILE;
    hipLaunchKernelGGL(k_radix_hist<BITS>, dim3((unsigned)nblk), dim3(SORT_T), 0, s, kin, n_dev, n,
                       shift, hist, nblk, cs.status ? cs.state : nullptr);
    const int64_t L = nblk << BITS;
    hipError_t e = hipSuccess;
    if (cs.status) {  // one launch instead of three
        hipLaunchKernelGGL(k_chained_scan, dim3((unsigned)chained_scan_blocks(L)), dim3(CS_T), 0,
                           s, hist, L, cs.status, (int64_t)-1, nullptr, cs.state, nullptr);
    } else {
        e = launch_scan_u32(hist, hist, L, scan_bs, nullptr, s);
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_radix_scatter<BITS>, dim3((unsigned)nblk), dim3(SORT_T), 0, s, kin, vin,
                       kout, vout, n_dev, n, shift, hist, nblk);
    return hipGetLastError();
}

hipError_t launch_sort_pairs(const uint32_t *kin, const uint32_t *vin, uint32_t *kout,
                             uint32_t *vout, uint32_t *ktmp, uint32_t *vtmp, int64_t n,
                             const unsigned long long *n_dev, int key_bits, int digit_bits,
                             uint32_t *hist, unsigned long long *scan_bs, int *which_out,
                             hipStream_t s, const ChainedScan &cs) {
    // Passes alternate out -> tmp -> out ...; the number of passes decides where the result
    // lands.  *which_out = 0: kout/vout, 1: ktmp/vtmp.
    if (n <= 0) {
        *which_out = 0;
        return hipSuccess;
    }
    if (digit_bits <= 0) digit_bits = auto_digit_bits(key_bits, n);
    if (digit_bits > 11) digit_bits = 11;
    const int passes = (key_bits + digit_bits - 1) / digit_bits;
    const uint32_t *ck = kin, *cv = vin;
    int where = 0;
    hipError_t e = hipSuccess;
    for (int p = 0; p < passes; ++p) {
        const int shift = p * digit_bits;
        const int bits = key_bits - shift < digit_bits ? key_bits - shift : digit_bits;
        uint32_t *ok = (p % 2 == 0) ? kout : ktmp;
        uint32_t *ov = (p % 2 == 0) ? vout : vtmp;
        switch (bits) {
#define GI_SORT_CASE(B) \
    case B: e = sort_pass<B>(ck, cv, ok, ov, n, n_dev, shift, hist, scan_bs, cs, s); break;
            GI_SORT_CASE(1) GI_SORT_CASE(2) GI_SORT_CASE(3) GI_SORT_CASE(4) GI_SORT_CASE(5)
            GI_SORT_CASE(6) GI_SORT_CASE(7) GI_SORT_CASE(8) GI_SORT_CASE(9) GI_SORT_CASE(10)
            GI_SORT_CASE(11)
#undef GI_SORT_CASE
            default: return hipErrorInvalidValue;
        }
        if (e != hipSuccess) return e;
        ck = ok;
        cv = ov;
        where = p % 2;
    }
    *which_out = where;
    return hipGetLastError();
}

hipError_t launch_sort(const BinBuffers &b, int key_bits, int digit_bits, int64_t n_max,
                       int *which, hipStream_t s) {
    // input keys[0]/vals[0]; passes go to keys[1], keys[0], ...
    int w = 0;
    hipError_t e = launch_sort_pairs(b.keys[0], b.vals[0], b.keys[1], b.vals[1], b.keys[0],
                                     b.vals[0], n_max, &b.state->keys_total, key_bits, digit_bits,
                                     b.hist, b.scan_blocksum, &w, s);
    // result in keys[1] when w == 0 (odd number of passes), in keys[0] when w == 1
    *which = (n_max <= 0) ? 0 : (w == 0 ? 1 : 0);
    return e;
}

int64_t fused_chunks(int64_t n) { return (n + FB - 1) / FB; }
int64_t fused_scan_entries(int64_t n, int64_t n_tiles) { return n + n_tiles * fused_chunks(n); }
int64_t fused_scan_blocks(int64_t n, int64_t n_tiles) {
    return (fused_scan_entries(n, n_tiles) + CS_TILE - 1) / CS_TILE;
}

hipError_t launch_fused_a(const FusedBuffers &f, const ImgTable &tab, hipStream_t s) {
    const int64_t nchunk = fused_chunks(f.b.n);
    hipLaunchKernelGGL(k_project_hist, dim3((unsigned)nchunk), dim3(FB),
                       sizeof(uint32_t) * (size_t)f.b.n_tiles, s,
                       record_src(f.b), f.b.n, tab,
                       reinterpret_cast<float4 *>(f.b.proj), f.b.rect, f.b.tinfo, f.b.count,
                       f.scan, (int32_t)f.b.n_tiles, nchunk, f.b.state);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t L = fused_scan_entries(f.b.n, f.b.n_tiles);
    hipLaunchKernelGGL(k_chained_scan, dim3((unsigned)fused_scan_blocks(f.b.n, f.b.n_tiles)),
                       dim3(CS_T), 0, s, f.scan, L, f.status, f.b.n, &f.b.state->keys_total,
                       f.b.state, nullptr);
    return hipGetLastError();
}

// Waves of the scatter for this device: 8 where the per-workgroup LDS (static plus 9 words per
// tile at the largest tile count of the one-pass path) fits, else 4.  (16 waves were measured
// slower at 768x512: 29 us against 23 us.)  Decided
// once per device at the first one-pass binning, which is never inside a graph capture
// (captured steps are preceded by an eager sizing pass); the kernel's dynamic LDS limit is
// raised then, once.
template <int WV>
static bool scatter_fits(int dev_lds) {
    hipFuncAttributes fa;
    const void *fn = reinterpret_cast<const void *>(&k_fused_scatter<WV>);
    const size_t dyn = sizeof(uint32_t) * (WV + 1) * (size_t)FUSED_MAX_TILES;
    if (hipFuncGetAttributes(&fa, fn) != hipSuccess || fa.sharedSizeBytes + dyn > (size_t)dev_lds)
        return false;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn) ==
           hipSuccess;
}

static int scatter_waves() {
    static int dev_cached = -1;
    static int waves = 4;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 4;
    if (dev != dev_cached) {
        dev_cached = dev;
        waves = 4;
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) ==
            hipSuccess) {
            if (scatter_fits<8>(v)) waves = 8;
        }
        (void)hipGetLastError();
    }
    return waves;
}

hipError_t launch_fused_c(const FusedBuffers &f, uint32_t *ids, hipStream_t s) {
    const int64_t nchunk = fused_chunks(f.b.n);
    int tbits = 1;
    while (((int64_t)1 << tbits) < f.b.n_tiles) ++tbits;
#define GI_LAUNCH_SCATTER(WV)                                                                   \
    hipLaunchKernelGGL(k_fused_scatter<WV>, dim3((unsigned)nchunk), dim3(64 * (WV)),            \
                       sizeof(uint32_t) * ((WV) + 1) * (size_t)f.b.n_tiles, s, f.b.count,      \
                       f.b.rect, f.b.tinfo, reinterpret_cast<const float4 *>(f.b.proj), f.scan, \
                       f.b.n, (int32_t)f.b.n_tiles, tbits, nchunk, f.b.cap,                     \
                       reinterpret_cast<float4 *>(f.b.rec), f.b.slot, ids, f.b.ranges,          \
                       f.b.opacity, f.b.rec_o, f.b.state)
    if (scatter_waves() == 8)
        GI_LAUNCH_SCATTER(8);
    else
        GI_LAUNCH_SCATTER(4);
#undef GI_LAUNCH_SCATTER
    return hipGetLastError();
}

int64_t row_chunks_max(int64_t cap_p, int64_t rows) {
    return (cap_p + ROW_CHUNK - 1) / ROW_CHUNK + rows;
}
int64_t row_scan_max(int64_t cap_p, int64_t rows, int32_t max_tw) {
    return row_chunks_max(cap_p, rows) * (int64_t)max_tw + 1;  // + the closing zero
}
int64_t chained_scan_blocks(int64_t len) { return (len + CS_TILE - 1) / CS_TILE; }

hipError_t launch_rows_a(const RowBuffers &r, const ImgTable &tab, hipStream_t s) {
    const BinBuffers &b = r.b;
    if (b.n <= 0) return hipErrorInvalidValue;
    const int64_t nb = grid_for(b.n, BLK);
    hipLaunchKernelGGL(k_project, dim3((unsigned)nb), dim3(BLK), 0, s, record_src(b), b.n, tab,
                       reinterpret_cast<float4 *>(b.proj), b.rect, b.tinfo, b.count, b.blocksum,
                       RowHistArgs{r.rhist, r.rhist_len, r.bwin}, b.state);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, b.blocksum, nb,
                       &b.state->keys_total, nullptr, nullptr);
    // the row counts and their closing zero; the prefix at the zero is the pair total
    const int64_t L = r.rhist_len + 1;
    hipLaunchKernelGGL(k_chained_scan, dim3((unsigned)chained_scan_blocks(L)), dim3(CS_T), 0, s,
                       r.rhist, L, r.status, r.rhist_len, &b.state->rows_total, b.state, nullptr);
    return hipGetLastError();
}

hipError_t launch_rows_b(const RowBuffers &r, const ImgTable &tab, bool want_ids, int *which,
                         hipStream_t s) {
    const BinBuffers &b = r.b;
    if (b.n <= 0 || tab.rows <= 0 || tab.max_tw < 1 || tab.max_tw > ROW_MAX_TW)
        return hipErrorInvalidValue;
    const int64_t pcap = b.cap_p < b.cap ? b.cap_p : b.cap;
    const int64_t nb = grid_for(b.n, BLK);
    float4 *proj = reinterpret_cast<float4 *>(b.proj);
    // the pairs go to vals[0]; the sorted Gaussian ids, when wanted, to vals[1]
    *which = 0;
    uint32_t *rv = b.vals[0];
    uint32_t *ids = want_ids ? b.vals[1] : nullptr;
    hipLaunchKernelGGL(k_rows_scatter, dim3((unsigned)nb), dim3(BLK), 0, s, b.count, proj,
                       b.blocksum, r.rhist, r.bwin, tab, b.n, pcap, b.off, rv, b.state);
    hipLaunchKernelGGL(k_row_table, dim3(1), dim3(RT_T), 0, s, r.rhist, (uint32_t)nb, pcap, tab,
                       (int64_t)tab.rows, r.nch_max, r.scan_max, r.rinfo, r.chunk_row, r.scan,
                       b.state);
    hipLaunchKernelGGL(k_row_hist, dim3((unsigned)r.nch_max), dim3(ROW_CHUNK), 0, s, rv, r.rinfo,
                       r.chunk_row, proj, r.scan, b.state);
    hipLaunchKernelGGL(k_chained_scan, dim3((unsigned)chained_scan_blocks(r.scan_max)), dim3(CS_T),
                       0, s, r.scan, r.scan_max, r.status, (int64_t)-1, nullptr, b.state,
                       &b.state->row_scan_len);
    hipError_t e;
    if ((e = launch_fill_u32(reinterpret_cast<uint32_t *>(b.ranges), 0u, 2 * b.n_tiles, s)) !=
        hipSuccess)
        return e;
    constexpr int WV = ROW_WAVES;
    hipLaunchKernelGGL(k_row_scatter<WV>, dim3((unsigned)r.nch_max), dim3(64 * WV),
                       sizeof(uint32_t) * (WV + 2) * (size_t)tab.max_tw, s, rv, r.rinfo,
                       r.chunk_row, proj, r.scan, b.off, b.cap,
                       reinterpret_cast<float4 *>(b.rec), b.slot, ids, b.ranges, b.opacity,
                       b.rec_o, b.state);
    return hipGetLastError();
}

hipError_t launch_ranges_gather(const BinBuffers &b, int which, const ImgTable &tab,
                                int64_t n_max, hipStream_t s) {
    (void)tab;
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(b.ranges), 0u, 2 * b.n_tiles, s);
    if (e != hipSuccess || n_max <= 0) return e;
    hipLaunchKernelGGL(k_ranges_gather, dim3(grid_for(n_max, BLK)), dim3(BLK), 0, s, b.keys[which],
                       b.vals[which], &b.state->keys_total, n_max,
                       reinterpret_cast<const float4 *>(b.proj), b.ranges,
                       reinterpret_cast<float4 *>(b.rec), b.slot, b.opacity, b.rec_o, b.ids_out);
    return hipGetLastError();
}

}  // namespace gi
