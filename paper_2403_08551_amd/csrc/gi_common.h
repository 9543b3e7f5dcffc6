// Internal declarations shared by the gfx950 kernels and the host runtime.
//
// Data layout in device memory (one context):
//   params  [N][8]  f32   (mu_x, mu_y, l1, l2, l3, c0, c1, c2), caller owned
//   proj    [N][16] f32   one 64-byte line per Gaussian (radix and row paths; the one-pass path
//                          packs the 32-byte records at a stride of 8 floats): the record (mu_x, mu_y, a, b, k, c0,
//                          c1, c2) with a = s/l1, b = s/l3, k = s*l2/(l1*l3), s =
//                          sqrt(log2(e)/2): then u1 = a*dx and u2 = b*dy - k*dx satisfy
//                          u1^2 + u2^2 = log2(e)*sigma, so that exp(-sigma) = exp2(-(u1^2 +
//                          u2^2)) (Eq. rasterization2 through the Cholesky factor: sigma =
//                          |L^{-1} d|^2 / 2); then u32 (key offset, image's first tile, tiles
//                          across | rect width << 16, tx0 | ty0 << 16), then u32 (global tile
//                          row of the rectangle's first row, its rows) and 2 unused words
//   rect    [N]     int4  inclusive tile rectangle (tx0, ty0, tx1, ty1); (0, 0, -1, -1) if none
//   tinfo   [N]     uint2 (first global tile id of the Gaussian's image, tiles across)
//   count   [N]     u32   tiles covered;  off [N] u32 exclusive prefix sum of count
//   keys/vals [cap] u32   (global tile id, Gaussian id), two ping-pong pairs for the sort
//                          (row binning keeps its (row, Gaussian) pairs in vals[0])
//   rec     [cap][8] f32  proj records in tile-sorted order
//   slot    [cap]   u32   position of each sorted key in the unsorted (Gaussian-major) order
//   part    [cap][8] f32  per (tile, Gaussian) partial gradient sums, indexed by slot
//   ranges  [T]     uint2 [start, end) of each tile in the sorted order
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gi {

constexpr int TILE = 16;
constexpr int TILE_PX = TILE * TILE;
constexpr uint32_t FLAG_KEY_OVERFLOW = 1u;
constexpr uint32_t FLAG_NONFINITE = 2u;
constexpr uint32_t FLAG_SCAN_STALL = 4u;
constexpr uint32_t FLAG_BAD_CODE = 8u;
constexpr int64_t FUSED_MAX_TILES = 2048;
// Row binning (tile count above FUSED_MAX_TILES): images up to this many tiles per row, and
// at most this many tile rows in the images that one block of 256 Gaussians spans.
constexpr int32_t ROW_MAX_TW = 1024;
constexpr int32_t ROW_WIN_MAX = 1024;
// float4 words per projected Gaussian on the radix and row paths: the rasteriser record (2),
// the slot facts (1), the first tile row and row count (1): one 64-byte line, so that the
// kernels after the sort read one line per key.  The one-pass path stores the record alone (2
// words per Gaussian).
constexpr int PROJ_F4 = 4;

// sqrt(log2(e) / 2): scales L^{-1} d so that exp(-sigma) = exp2(-|u|^2)
constexpr double U_SCALE = 0.84932180028801904272;

// Device-resident scalars of one context.
struct DevState {
    unsigned long long keys_total;  // keys of the last binning (may exceed capacity)
    uint32_t flags;                 // sticky FLAG_*
    uint32_t spare;
    uint32_t scan_epoch;            // launch tag of the chained scans' status words
    uint32_t row_chunks;            // row binning: chunks of (row, Gaussian) pairs
    unsigned long long rows_total;  // row binning: (row, Gaussian) pairs (may exceed capacity)
    unsigned long long row_scan_len;  // row binning: length of the per-column count array
};

// Covariance factorisation read from params[2..4] (Sec. 3.1): (l1, l2, l3) of the Cholesky
// factor (Eq. cholesky), or (s1, s2, theta) of Sigma = (R S)(R S)^T (Eq. RSSR).
constexpr int32_t COV_CHOLESKY = 0;
constexpr int32_t COV_ROTATION_SCALE = 1;

// Image geometry, passed by value.  B == 1 uses the scalar fields; B > 1 reads the tables.
struct ImgTable {
    int32_t B;
    int32_t H, W, TW;                 // single image
    int32_t cov;                      // COV_* of the records
    const int4 *dims;                 // [B] (H, W, TW, TH)
    const uint32_t *tile_base;        // [B+1] first global tile id of each image
    const uint32_t *gauss_off;        // [B+1]
    const unsigned long long *pix_off;  // [B+1] first pixel of each image
    const uint32_t *row_base;         // [B+1] first global tile row of each image (B > 1)
    const uint2 *row_tiles;           // [rows] first global tile, tiles per row (B > 1)
    // row binning's per-block row counts, laid out image by image, then row, then the blocks
    // of 256 Gaussians that overlap the image (B > 1; one image: row * blocks + block):
    const unsigned long long *row_seg;  // [rows + 1] index of a row's first block's count
    const uint32_t *row_fb;             // [rows] first block overlapping the row's image
                                        // (0xffffffff: the image has no Gaussians)
    int32_t row_win;                  // most tile rows that one block's images hold (B > 1)
    int64_t row_len;                  // per-block row counts in all (B > 1)
    int32_t rows;                     // tile rows of all images
    int32_t max_tw;                   // most tiles per row of any image
};

struct TileInfo {
    int32_t img, tx, ty, H, W;
    unsigned long long pix_base;
};

__device__ inline int32_t upper_index(const uint32_t *arr, int32_t n, uint32_t v) {
    // largest i in [0, n) with arr[i] <= v (arr ascending, arr[0] = 0)
    int32_t lo = 0, hi = n - 1;
    while (lo < hi) {
        int32_t mid = (lo + hi + 1) >> 1;
        if (arr[mid] <= v) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ inline TileInfo tile_info(const ImgTable &t, uint32_t tile) {
    TileInfo ti;
    if (t.B == 1) {
        ti.img = 0; ti.H = t.H; ti.W = t.W;
        ti.tx = (int32_t)(tile % (uint32_t)t.TW);
        ti.ty = (int32_t)(tile / (uint32_t)t.TW);
        ti.pix_base = 0;
    } else {
        int32_t b = upper_index(t.tile_base, t.B, tile);
        int4 d = t.dims[b];
        uint32_t lt = tile - t.tile_base[b];
        ti.img = b; ti.H = d.x; ti.W = d.y;
        ti.tx = (int32_t)(lt % (uint32_t)d.z);
        ti.ty = (int32_t)(lt / (uint32_t)d.z);
        ti.pix_base = t.pix_off[b];
    }
    return ti;
}

// A compressed Gaussian set (Sec. 3.3): binary16 positions [N][2], b-bit covariance codes
// [N][3] with shared scale/offset, residual-VQ indices [N][M] into codebooks [M][B][3].
struct CodecArgs {
    const uint16_t *mu;
    const uint8_t *codes;
    const uint8_t *index;
    const float *book;
    float gamma[3], beta[3];
    int32_t bits, stages, size;
};

// Opacity renderings (Sec. 3.2): BLEND_SUM is C = sum c o exp(-sigma) (Eq. rasterization3),
// BLEND_ALPHA is alpha blending in index order (Eq. rasterization1) with alpha = min(o exp(-sigma),
// ALPHA_MAX).
constexpr int32_t BLEND_NONE = 0;
constexpr int32_t BLEND_SUM = 1;
constexpr int32_t BLEND_ALPHA = 2;
constexpr float ALPHA_MAX = 0.99f;

// Where the projection reads Gaussian records: float params, or (codec.mu != nullptr) a
// compressed set decoded on the fly; with an opacity per Gaussian for the opacity renderings
// (BLEND_SUM stores o * c as the record colour).  Passed to kernels by value.
// Quantiser of the quantisation-aware fine-tuning (Sec. 3.3): quant = gamma[3], beta[3], then
// codebooks [stages][size][3], all float32 on the device.
struct QatArgs {
    const float *quant;
    int32_t bits, stages, size;
};
constexpr int QAT_MAX_STAGES = 8;
constexpr int QAT_MAX_ENTRIES = 64;  // stages * size
constexpr int QAT_KMAX = 64;         // codebook size

struct RecordSrc {
    const float4 *params;
    CodecArgs codec;
    const float *opacity;
    int32_t blend;
    int32_t recipe;  // 1: params are raw records of the fitting recipe (see recipe_effective)
    QatArgs qat;     // quant != nullptr: render the fake-quantised records
};

// What the fake quantiser decided for one Gaussian (for its gradients).
struct QuantFacts {
    double x[3];      // scaled covariance values (l - beta) / gamma
    double code[3];   // their codes
    int32_t idx[8];   // RVQ index per stage
};

// Fake quantisation of one record (Sec. 3.3), in place: binary16 positions, LSQ+ codes
// code = round-to-even(clamp((l - beta) / gamma, 0, 2^b - 1)) dequantised as code * gamma + beta,
// and greedy residual VQ of the colour (nearest entry by squared distance, the lowest index on
// ties) summed over the stages.  Everything in float64 without contraction, each result rounded
// once to float32, so any IEEE machine that follows these steps decides the same codes.
__device__ inline void qat_fake_quant(float (&q)[8], const QatArgs &a, QuantFacts *f) {
#pragma clang fp contract(off)
    q[0] = (float)(_Float16)q[0];
    q[1] = (float)(_Float16)q[1];
    const double top = (double)((1 << a.bits) - 1);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double g = a.quant[i], b = a.quant[3 + i];
        const double x = ((double)q[2 + i] - b) / g;
        const double c = rint(x < 0.0 ? 0.0 : (x > top ? top : x));
        q[2 + i] = (float)(c * g + b);
        if (f) {
            f->x[i] = x;
            f->code[i] = c;
        }
    }
    const float *books = a.quant + 6;
    double r0 = q[5], r1 = q[6], r2 = q[7];
    double c0 = 0.0, c1 = 0.0, c2 = 0.0;
    // stages unrolled to the maximum so that idx[m] stays in registers
#pragma unroll
    for (int m = 0; m < QAT_MAX_STAGES; ++m) {
        if (m >= a.stages) break;
        const float *bk = books + (int64_t)m * a.size * 3;
        int best = 0;
        double bd = 0.0;
        for (int k = 0; k < a.size; ++k) {
            const double d0 = r0 - (double)bk[3 * k], d1 = r1 - (double)bk[3 * k + 1];
            const double d2 = r2 - (double)bk[3 * k + 2];
            const double d = (d0 * d0 + d1 * d1) + d2 * d2;
            if (k == 0 || d < bd) {
                bd = d;
                best = k;
            }
        }
        if (f) f->idx[m] = best;
        const double e0 = bk[3 * best], e1 = bk[3 * best + 1], e2 = bk[3 * best + 2];
        c0 += e0;
        c1 += e1;
        c2 += e2;
        r0 -= e0;
        r1 -= e1;
        r2 -= e2;
    }
    q[5] = (float)c0;
    q[6] = (float)c1;
    q[7] = (float)c2;
}

// The fitting recipe's parametrisation (App. C): raw (rho_x, rho_y, lam1, lam2, lam3, c) ->
// mu = extent (tanh(rho) + 1) / 2, and 0.5 added to l1, l3 (Cholesky) or s1, s2 (rotation-scale),
// in float64, rounded once to float32.
__device__ inline void recipe_effective(float (&q)[8], int32_t H, int32_t W, bool rs) {
    q[0] = (float)((double)W * (tanh((double)q[0]) + 1.0) * 0.5);
    q[1] = (float)((double)H * (tanh((double)q[1]) + 1.0) * 0.5);
    q[2] = (float)((double)q[2] + 0.5);
    if (rs)
        q[3] = (float)((double)q[3] + 0.5);
    else
        q[4] = (float)((double)q[4] + 0.5);
}

// ---- host-side launchers (defined next to their kernels) ------------------------------------

struct BinBuffers {
    const float *params;
    const CodecArgs *codec;  // non-null: decode the records from this compressed set instead
    const float *opacity;    // [N] for the opacity renderings, else null
    int32_t blend;           // BLEND_*
    float *rec_o;            // [cap] opacity in tile order (BLEND_ALPHA), else null
    int32_t recipe;          // 1: raw records of the fitting recipe
    QatArgs qat;             // quant != nullptr: fake-quantised records
    int64_t n;
    float *proj;
    int4 *rect;
    uint2 *tinfo;
    uint32_t *count;
    uint32_t *off;
    unsigned long long *blocksum;  // [ceil(n/256)]
    uint32_t *keys[2];
    uint32_t *vals[2];
    uint32_t *ids_out;              // sorted Gaussian ids, when wanted (radix path), else null
    float *rec;
    uint32_t *slot;
    uint2 *ranges;
    int64_t n_tiles;
    int64_t cap;
    int64_t cap_p;                  // row binning: (row, Gaussian) pairs the sort is sized for
    DevState *state;
    // sort scratch
    uint32_t *hist;                 // [2^bits * max_sort_blocks]
    unsigned long long *scan_blocksum;  // generic scan scratch
    int64_t hist_cap;               // entries available in hist
    int64_t scan_cap;               // entries available in scan_blocksum
};

hipError_t launch_project(const BinBuffers &b, const ImgTable &tab, hipStream_t s);
hipError_t launch_count_scan(const BinBuffers &b, hipStream_t s);
hipError_t launch_duplicate(const BinBuffers &b, hipStream_t s);
// Sort keys[0]/vals[0] -> result in keys[r]/vals[r]; returns r through *which.  n_max bounds
// the key count (the device total is read by the kernels); key_bits > 0.
hipError_t launch_sort(const BinBuffers &b, int key_bits, int digit_bits, int64_t n_max,
                       int *which, hipStream_t s);
hipError_t launch_ranges_gather(const BinBuffers &b, int which, const ImgTable &tab,
                                int64_t n_max, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
// Decode a compressed set into float records [N][8] (invalid Gaussians: NaN records).
hipError_t launch_codec_decode(const CodecArgs &c, int64_t n, float *params, DevState *state,
                               hipStream_t s);

// One-pass binning (n_tiles <= FUSED_MAX_TILES): A = projection + per-chunk tile counts +
// chained scan (writes state->keys_total); C = stable scatter into tile order + ranges.
struct FusedBuffers {
    BinBuffers b;
    uint32_t *scan;                 // [fused_scan_entries]
    unsigned long long *status;     // [fused_scan_blocks], epoch-tagged
};
int64_t fused_chunks(int64_t n);
int64_t fused_scan_entries(int64_t n, int64_t n_tiles);
int64_t fused_scan_blocks(int64_t n, int64_t n_tiles);
hipError_t launch_fused_a(const FusedBuffers &f, const ImgTable &tab, hipStream_t s);
hipError_t launch_fused_c(const FusedBuffers &f, uint32_t *ids, hipStream_t s);

// Row binning (n_tiles > FUSED_MAX_TILES, every image at most ROW_MAX_TW tiles wide and the
// images of any block of 256 Gaussians at most ROW_WIN_MAX tile rows), a counting sort in two
// levels.  A: projection (64-byte lines) with per-block key sums (scanned: state->keys_total)
// and per-block row counts (one chained scan: state->rows_total).  B: the (global tile row,
// Gaussian) pairs scattered stably into row order; each row's pairs cut into chunks of
// ROW_CHUNK; per (row, column, chunk) key counts, one chained scan over them (row major, then
// column, then chunk: exactly tile order), and the scatter of every chunk's keys in Gaussian
// order into tile order with the records, slots and ranges.
constexpr int ROW_CHUNK = 256;
struct RowBuffers {
    BinBuffers b;
    uint32_t *rhist;             // [rhist_len + 1] per-block row counts (layout: ImgTable), a
                                 // closing zero, then their scan
    int64_t rhist_len;
    uint4 *bwin;                 // [blocks] first global row and rows of each block's images
    uint4 *rinfo;                // [2 rows] {first pair, end pair, first chunk, scan offset},
                                 // {first tile, tiles per row, chunks, 0}
    uint32_t *chunk_row;         // [nch_max] the row of each chunk
    uint32_t *scan;              // [scan_max] per-chunk column counts, then their scan
    unsigned long long *status;  // [ceil(scan_max / 4096)] chained-scan status, epoch-tagged
    int64_t nch_max, scan_max;
};
// Chunk and count-array bounds of row binning for a pair capacity.
int64_t row_chunks_max(int64_t cap_p, int64_t rows);
int64_t row_scan_max(int64_t cap_p, int64_t rows, int32_t max_tw);
int64_t chained_scan_blocks(int64_t len);
hipError_t launch_rows_a(const RowBuffers &r, const ImgTable &tab, hipStream_t s);
// *which receives the buffer pair holding the (row, Gaussian) pairs (0); the sorted Gaussian
// ids go to the other pair's values when wanted.
hipError_t launch_rows_b(const RowBuffers &r, const ImgTable &tab, bool want_ids, int *which,
                         hipStream_t s);

// generic pieces, also exported for testing
hipError_t launch_scan_u32(const uint32_t *in, uint32_t *out, int64_t n,
                           unsigned long long *blocksum, unsigned long long *total,
                           hipStream_t s);
int64_t scan_scratch_entries(int64_t n);
// Resources for scanning the digit histograms with the one-pass chained scan (status words of
// at least chained_scan_blocks(entries) and the context state whose epoch tags them); with a
// null status the three-launch scan is used.
struct ChainedScan {
    unsigned long long *status = nullptr;
    DevState *state = nullptr;
};
hipError_t launch_sort_pairs(const uint32_t *kin, const uint32_t *vin, uint32_t *kout,
                             uint32_t *vout, uint32_t *ktmp, uint32_t *vtmp, int64_t n,
                             const unsigned long long *n_dev, int key_bits, int digit_bits,
                             uint32_t *hist, unsigned long long *scan_bs, int *which_out,
                             hipStream_t s, const ChainedScan &cs = ChainedScan{});
int64_t sort_hist_entries(int64_t n, int digit_bits);
int auto_digit_bits(int key_bits, int64_t n);

struct RasterArgs {
    const float *rec;
    const uint32_t *slot;
    const uint2 *ranges;
    int64_t n_tiles;
    ImgTable tab;
    const uint32_t *order = nullptr;  // workgroup w rasterises tile order[w]; null: tile w
};

// Tile order for the raster kernels, longest list first (a counting sort by list length, one
// workgroup; lengths over TILE_ORDER_BINS - 1 share the first bin).  The order only changes
// which workgroup takes which tile, never a tile's arithmetic, so results are the same bits.
constexpr int TILE_ORDER_BINS = 4096;
hipError_t launch_tile_order(const uint2 *ranges, int64_t n_tiles, uint32_t *order,
                             hipStream_t s);

// flag_state (optional): block 0 hands that state's flags to flags_out (if given) and clears them
hipError_t launch_raster_fwd(const RasterArgs &a, float *image, int px_per_lane, hipStream_t s,
                             DevState *flag_state = nullptr, uint32_t *flags_out = nullptr);
hipError_t launch_raster_bwd(const RasterArgs &a, const float *dl_dimage, float *part,
                             hipStream_t s);
// step_inc (may be null): advanced by one by the kernel; the update kernel that follows reads
// the step number as *step - 1.
hipError_t launch_raster_fit(const RasterArgs &a, const float *target, float *part,
                             float *image_out, float *loss_part, int px_per_lane,
                             int waves_per_simd, int32_t *step_inc, hipStream_t s);
// Alpha blending (BLEND_ALPHA): rec_o [cap] holds the opacities in tile order; part12 has
// three float4 per key (colour sums, P1; P2, Q11, Q12, Q22; opacity sum).
hipError_t launch_alpha_fwd(const RasterArgs &a, const float *rec_o, float *image, hipStream_t s);
hipError_t launch_alpha_bwd(const RasterArgs &a, const float *rec_o, const float *dl_dimage,
                            float *part12, hipStream_t s);
hipError_t launch_alpha_fit(const RasterArgs &a, const float *rec_o, const float *target,
                            float *part12, float *image_out, float *loss_part, int32_t *step_inc,
                            hipStream_t s);

struct UpdateArgs {
    const float *params_in;  // read (l1, l2, l3) or (s1, s2, theta); Adam updates in place
    float *params_out;
    int64_t n;
    const uint32_t *count;
    const uint32_t *off;
    const float *part;
    DevState *state;
    int64_t cap;
    int32_t cov;             // COV_*
};
hipError_t launch_grad_out(const UpdateArgs &u, float *dparams, hipStream_t s);
// Gradient of the opacity renderings: dparams [N][8] (colour slots = dL/dc) and dopacity [N].
// For BLEND_SUM u.part holds the merged-colour sums (8 floats per key); for BLEND_ALPHA the
// 12-float sums of launch_alpha_bwd.
hipError_t launch_grad_opacity(const UpdateArgs &u, const float *opacity, int32_t blend,
                               float *dparams, float *dopacity, hipStream_t s);
struct AdamArgs {
    float lr_mu, lr_l, lr_c, beta1, beta2, eps, l_min;
};
// Adam update with step number *step - 1 (the fit kernel advanced the counter); also writes the
// per-image losses when loss_out != nullptr, and with order_out the longest-first order of the
// n_tiles lists in `ranges` (a permutation of the tiles, in one extra block of the same launch).
hipError_t launch_adam(const UpdateArgs &u, float *params, float *m, float *v,
                       int32_t *step, const AdamArgs &hp, const float *loss_part,
                       const ImgTable &tab, int64_t n_tiles, float *loss_out, hipStream_t s,
                       const uint2 *ranges = nullptr, uint32_t *order_out = nullptr);
// Adam over params and opacities of an opacity rendering (opacity uses the colour rate), as
// launch_adam.
hipError_t launch_adam_opacity(const UpdateArgs &u, float *params, float *opacity, float *m,
                               float *v, float *mo, float *vo, int32_t *step, const AdamArgs &hp,
                               int32_t blend, const float *loss_part, const ImgTable &tab,
                               int64_t n_tiles, float *loss_out, hipStream_t s);
// The fitting recipe's update (App. C parametrisation, Adan): gradients of the raw records and
// the Adan step; state = m, v, n, previous gradient, each [N][8].
struct AdanArgs {
    float lr, beta1, beta2, beta3, eps, weight_decay;
    int32_t halve_every;
};
hipError_t launch_adan(const UpdateArgs &u, float *raw, float *state, int32_t *step,
                       const AdanArgs &hp, const ImgTable &tab, const float *loss_part,
                       int64_t n_tiles, float *loss_out, hipStream_t s);
// Quantisation-aware fine-tuning update: the Gaussians' Adam step (straight-through gradients
// of the fake-quantised records), then the quantiser's step (Adam on gamma and beta from their
// LSQ+ gradients, the moving average of the codebooks); qpart holds qat_part_floats(n, stages,
// size) floats of block sums (its start 8-byte aligned).
hipError_t launch_qat_update(const UpdateArgs &u, float *params, float *m, float *v,
                             int32_t *step, const AdamArgs &hp, const QatArgs &qa, float lambda,
                             float lr_q, float *quant_m, float *quant_v, float *ema, float decay,
                             float *qpart, const float *loss_part, const ImgTable &tab,
                             int64_t n_tiles, float *loss_out, hipStream_t s);
int64_t qat_part_floats(int64_t n, int stages, int size);
// Quantiser initialisation and encoding (k_qat.hip): gamma, beta from the covariance range,
// codebooks by K-means per stage; scratch: at least qat_init_scratch_bytes(n, size) bytes.
size_t qat_init_scratch_bytes(int64_t n, int size);
hipError_t launch_qat_init(const float *params, int64_t n, const QatArgs &qa, int kmeans_iters,
                           float *ema, void *scratch, hipStream_t s);
hipError_t launch_qat_encode(const float *params, int64_t n, const QatArgs &qa, uint16_t *mu,
                             uint8_t *codes, uint8_t *index, hipStream_t s);
// Effective records of raw recipe records.
hipError_t launch_recipe_effective(const float *raw, int64_t n, const ImgTable &tab, int32_t cov,
                                   float *params, hipStream_t s);
// Per-image loss from the per-tile sums when loss_out != nullptr (used when no update kernel runs).
hipError_t launch_finish(const float *loss_part, const ImgTable &tab, int64_t n_tiles,
                         float *loss_out, hipStream_t s);

}  // namespace gi
