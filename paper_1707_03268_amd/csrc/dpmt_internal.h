// Internal types shared by the host runtime (dpmt_host.cpp) and the HIP
// kernels (dpmt_kernels.hip).  Nothing here is part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace dpmt {

// Operand packing of one correlation flavour.  A "plane" is PB bytes of every
// cell (a run of channels); a K-step is 32 bytes of one flattened filter row
// of one plane (w cells x PB bytes, zero padded to S*32 bytes).
struct Packing {
    int esz;   // element bytes: 4 (fp32), 2 (bf16), 1 (fp8)
    int RP;    // channels per cell in the operand (32 for direct, padded rank otherwise)
    int PB;    // plane bytes per cell
    int Q;     // planes per cell: RP * esz / PB
};

// One (role, shape) group of filters.  Responses of a group on a level are
// stored filter-major: one Ho x ld float32 plane per filter of the group,
// position (y, x) at y * ld + x, ld = Wo rounded up to a multiple of 4.
struct GroupDesc {
    int32_t h, w;      // filter rows, cols
    int32_t ng;        // filters in the group
    int32_t S;         // K-steps per filter row per plane (32 bytes; 64 for FP8)
    int64_t g_off;     // byte offset of the group's packed operand in the G buffer
    int32_t t_off;     // first per-filter scale of the group (FP8)
    int32_t pad;
};

// One 32-filter block of a group, for the per-call FP8 requantisation.
struct RequantBlock {
    int64_t m_off;     // float offset of the block's FP32 master factors
    int64_t g_off;     // byte offset of the block's FP8 operand
    int32_t chunks;    // Q * S * h chunks of 64 lanes x 32 elements
    int32_t h, S;
    int32_t ng;        // filters in the group
    int32_t f0;        // first filter column of the block
    int32_t t_off;     // scale slot of the block's first filter
};

// One workgroup tile of the correlation: TYWG output rows x 32 output cols x
// nfb * BB * 32 filters of one group on one level (BB * 32 at a time).
struct CorrTile {
    int64_t z_cell;    // first cell of the level in the feature / projected buffer
    int64_t out_off;   // element offset of the group's first response plane on this level
    int32_t H, W;      // level rows, cols
    int32_t Ho, Wo;    // response rows, cols
    int32_t ld;        // row pitch of the response planes (multiple of 4)
    int32_t rng;       // range slot of the group's first plane (-1: no ranges)
    int32_t y0, x0;    // first output row, col
    int32_t fb0;       // first 32-filter block
    int32_t group;
    int32_t nfb;       // groups of BB filter blocks the tile walks over the same window
    int32_t pad;
};

// One part of one score map: where its response plane lives, its anchor and
// its deformation coefficients.
struct MapPart {
    int64_t plane;     // element offset of the part filter's response plane
    int32_t ld;        // plane row pitch
    int32_t Hp, Wp;    // part response map (0 x 0 when the filter does not fit)
    int32_t rng;       // range slot of the plane
    int32_t vy, vx;    // anchor (part-level cells)
    float d[4];        // d_x, d_xx, d_y, d_yy
    float inv2ax;      // 1 / (2 d_xx)
    float inv2ay;      // 1 / (2 d_yy)
    float bb4a;        // d_x^2 / (4 d_xx): how far a row-pass value can exceed the response maximum
    int32_t pad;
};

// One score map (image, root level, component).
struct MapDesc {
    int64_t score_off; // float offset into the caller's scores
    int64_t offs_off;  // int16 offset into the caller's offsets ([part][pos][2])
    int64_t root_plane;// element offset of the root filter's response plane
    int32_t Ho, Wo;
    int32_t ldr;       // root plane row pitch
    int32_t n_parts;
    int32_t part_base; // first MapPart of the map
    int32_t r1_rows;   // placement row-pass tile rows: tallest part map + 2 * PLACE_PAD
    int32_t ctab_words;// placement floats per cost table (multiple of 4)
    int32_t pad;
};

// One detection (the C ABI's dpmt_detection).
struct Detection {
    int32_t map;
    int32_t y, x;
    float score;
};

// Per-filter CP form (Section 4): filter k ~ sum_r a_r (x) b_r (x) c_r with
// its own rank R_k.  Responses go to the same filter-major planes as the
// other flavours.  A chunk is 4 consecutive filter columns of a group; its
// channel factors are packed for the MFMA B operand in batches of 16 columns
// (4 filters x 4 rank terms): [batch][lane][8] floats, lane = column + 16 * g
// holding c[8g + s] of column (filter lane%16 / 4, term 4*batch + lane%4) at
// K-step s.  Row and column factors of filter j: R_j x h floats a_r[n], then
// R_j x w floats b_r[m], at ab_off[j].
struct CpChunk {
    int64_t c_off;     // float offset of the chunk's packed channel factors
    int64_t ab_off[4]; // float offset of each filter's row / column factors
    int32_t R[4];      // ranks (0: no filter in that slot)
    int32_t nq;        // batches of 4 rank terms: max ceil(R / 4)
    int32_t pad;
};

// One workgroup tile of the CP correlation: up to 32 output cols x TYo rows of
// one level, the halo (HY x HX cells, HX a multiple of 4, HX * HY <= 1024)
// held in registers while the tile walks nchunk chunks of one group.
struct CpTile {
    int64_t x_cell;    // first cell of the level in the feature buffer
    int64_t out_off;   // element offset of the group's first response plane
    int32_t H, W;      // level rows, cols
    int32_t Ho, Wo;    // response rows, cols
    int32_t ld;        // plane row pitch
    int32_t rng;       // range slot of the group's first plane (-1: no ranges)
    int32_t y0, x0;    // first output row, col (x0 a multiple of 32)
    int32_t h, w;      // filter rows, cols
    int32_t HY, HX;    // halo rows, cols
    int32_t chunk0;    // first chunk (index into the chunk table)
    int32_t nchunk;    // chunks walked
    int32_t col0;      // filter column of the first chunk's first filter
    int32_t pad;
};
constexpr int CP_HALO = 1024;             // halo cells per CP tile
constexpr int CP_TX = 32;                 // output cols per CP tile
// halo geometry of a CP tile for a filter of w columns
inline int cp_halo_cols(int w) { return (CP_TX + w - 1 + 3) & ~3; }
inline int cp_halo_rows(int w) { return CP_HALO / cp_halo_cols(w); }
size_t cp_lds_bytes(int HX, int HY);

// Correlation kernel flavours.
enum CorrKind { CORR_F32 = 0, CORR_BF16 = 1, CORR_FP8 = 2 };

struct CorrLaunch {
    CorrKind kind;
    Packing pk;
    int ty;            // output rows per wave
    int bb;            // 32-filter blocks per wave
    int wy;            // waves per workgroup
    int persistent;    // 0: one workgroup per tile; 1: resident grid striding the tiles
    int wx;            // of them side by side along x (wy / wx stacked along rows)
    int hs;            // every tile has filters of exactly hs rows (6, 7, 8), or 0: any
};
// Tile shapes the correlation kernel is built for (ty, bb, wy, wx); filters
// taller than 8 rows only with (4, 2, 4, 1).  A workgroup tile covers
// ty * wy / wx output rows x 32 * wx output columns.
bool corr_shape_supported(int ty, int bb, int wy, int wx, int max_h);

// Placement kernel geometry.  A block owns PLACE_CW consecutive root columns
// of one score map; its LDS holds the score accumulator, the row-pass tile of
// the current part with PLACE_PAD -inf rows above and below, a staging area
// for response rows, and the two cost tables.
constexpr int PLACE_CW = 16;
constexpr int PLACE_RPW = 64 / PLACE_CW;  // rows per wavefront
// -inf rows above and below the row-pass tile: a wavefront's column-pass
// window clamp spans its PLACE_RPW target rows, plus 3 for the unroll by 4
constexpr int PLACE_PAD = 2 * (PLACE_RPW - 1) + 3;
constexpr int PLACE_STAGE = 2048;         // floats of the staging buffer (32 rows of 64)
// Workgroups of 256 threads a CU holds by registers: the kernel's 78 VGPRs
// (granules of 8, 80 allocated) allow 6 wavefronts per SIMD.
constexpr int PLACE_WG_PER_CU = 6;
// Workgroups are dealt to the 8 XCDs (each with its own L2) round-robin by
// launch index.  The placement's neighbouring strips stage overlapping
// response rows, so it remaps the launch index: clusters of 2^xcl consecutive
// strips run on one XCD, while the clusters still interleave over the XCDs in
// work order; the grid is padded to a multiple of 8 * 2^xcl and the padding
// exits.  Clusters of 16 strips span a 1080p root map's width: the fetch is
// then 1.13x the responses the kernel reads (1.25x with clusters of 8, 1.47x
// with clusters of 4).
constexpr int N_XCD = 8;
constexpr int PLACE_XCL = 4;
inline int xcd_grid(int n, int xcl) {
    const int g = N_XCD << xcl;
    return (n + g - 1) / g * g;
}
// LDS of one placement block, laid out from its own map: score accumulator,
// row-pass tile, staging, the two cost tables, row-pass argmax, rejection
// flags, part windows.  A launch gives every block the largest of its maps'.
struct PlaceLds {
    int acc_rows;      // map height
    int r1_rows;       // tallest part map + 2 * PLACE_PAD
    int stage_words;   // floats of the staging buffer (PLACE_STAGE)
    int ctab_words;    // floats per cost table (multiple of 4)
    int max_parts;     // parts of the map
};
size_t place_lds_bytes(const PlaceLds& l);
// Cost table floats for part maps of at most Hp x Wp: the row window spans
// at most Wp + 2 (CW - 1) + 3 (alignment) + 1 offsets, rounded up to 4; the
// column window at most 2 (Hp + 1) + 1 offsets, plus 4.
inline int place_ctab_words(int Hp, int Wp) {
    const int row = Wp + 2 * (PLACE_CW - 1) + 8, col = 2 * (Hp + 1) + 1 + 4;
    return ((row > col ? row : col) + 3) & ~3;
}
inline PlaceLds place_lds_of_map(const MapDesc& m) {
    return PlaceLds{m.Ho, m.r1_rows, PLACE_STAGE, m.ctab_words, m.n_parts};
}
// Dynamic LDS a placement block may use: 160 KB per CU, less 1 KB kept for
// the kernel's own static LDS (checked at launch).
constexpr size_t PLACE_LDS_MAX = 159 * 1024;
// Placement workgroups of nt threads (256 or 512) one CU holds, for blocks of
// `bytes` dynamic LDS: by LDS (allocated in 512-byte granules) and by
// registers (6 wavefronts per SIMD).
inline int place_blocks_per_cu(size_t bytes, int nt) {
    const size_t per = (bytes + 511) / 512 * 512;
    const int by_regs = PLACE_WG_PER_CU * 256 / nt;
    const size_t by_lds = per ? PLACE_LDS_MAX / per : (size_t)by_regs;
    return by_lds < (size_t)by_regs ? (int)by_lds : by_regs;
}
// Row span (floats) a part of response width Wp can need in the staging
// buffer: 2 * (PLACE_CW - 1) targets apart, plus a window clamped to the line
// and aligned to whole 16-byte runs.
inline int place_span_max(int Wp) { return Wp + 4 * (PLACE_CW - 1) + 12; }

// --- kernel launchers (dpmt_kernels.hip) -----------------------------------
// rkeys (may be NULL): 2 * n_slots range keys to reset along the way (as
// launch_range_init does).
hipError_t launch_project(bool bf16, const float* X, int64_t n_cells, const float* U,
                          int RP, void* Z, int* rkeys, int64_t n_slots, hipStream_t st);
// rkeys (may be NULL): 2 * n_slots range keys, maxima then minima, updated
// with the value range of every response plane whose tile names a slot.
hipError_t launch_corr(const CorrLaunch& cfg, const CorrTile* tiles, int n_tiles,
                       const GroupDesc* groups, const void* Z, const void* G, const float* tk,
                       float* out, int* rkeys, int64_t n_slots, int max_h, int max_S,
                       hipStream_t st);
// CP correlation of every tile (one workgroup per tile).  lds_bytes: the
// largest cp_lds_bytes over the tiles.
// flags (may be NULL): one byte per response, set where a partial sum fell
// below the filter's threshold (the thresholds follow each filter's column
// factors in fac).
hipError_t launch_cp_corr(const CpTile* tiles, int n_tiles, const CpChunk* chunks, const float* X,
                          const float* fac, float* out, int* rkeys, int64_t n_slots, uint8_t* flags,
                          size_t lds_bytes, hipStream_t st);
// chmax: per filter slot, the largest |factor| of each of the RP channels.
// rkeys (may be NULL): 2 * n_slots range keys to reset along the way.
hipError_t launch_fp8_prepare(const float* X, int64_t n_cells, const float* U, int RP,
                              float* partial, float* scales, const RequantBlock* blocks,
                              int n_blocks, const float* master, const float* chmax, uint8_t* G,
                              float* tk, int* rkeys, int64_t n_slots, hipStream_t st);
hipError_t launch_project_fp8(const float* X, int64_t n_cells, const float* U, int RP,
                              const float* scales, void* Z, hipStream_t st);
constexpr int FP8_PARTIALS = 512 * 32;   // floats of the channel-max scratch
size_t corr_lds_bytes(const CorrLaunch& cfg, int max_h, int S);
hipError_t launch_range_init(int* rkeys, int64_t n_slots, hipStream_t st);
// flags (may be NULL): the CP correlation's rejection bytes; rejected root
// positions get score -inf and offsets 0.
hipError_t launch_place(const MapDesc* maps, const MapPart* parts, const int2* blkmap,
                        int n_blocks, const float* resp, const int* rkeys, int64_t n_slots,
                        float* scores, int16_t* offs, size_t lds_bytes, const uint8_t* flags,
                        hipStream_t st);
hipError_t launch_planes_to_maps(const float* planes, int ng, int Ho, int Wo, int ld,
                                 const int64_t* dst_off, float* out, hipStream_t st);
// Detections: counts holds det_blocks(n) int64 of scratch: one count per
// block of 1024 positions, then one sum per segment of DET_SEG such counts.
constexpr int64_t DET_SEG = 1024;
constexpr int64_t det_blocks(int64_t n) {
    return (n + 1023) / 1024 + ((n + 1023) / 1024 + DET_SEG - 1) / DET_SEG;
}
hipError_t launch_detect(const float* scores, int64_t n, float tau, const MapDesc* maps, int n_maps,
                         int64_t* counts, int64_t* count, Detection* dets, int64_t capacity,
                         hipStream_t st);
hipError_t launch_dt_single(const float* resp, int rows, int cols, int ld, const float* d,
                            float* lmax, float* r1v, int32_t* r1a, float* out, int32_t* ay,
                            int32_t* ax, hipStream_t st);
// The same transform with its scratch (line maxima, row-pass values and
// argmax) in a file-scope device array of the kernels' source instead of
// allocations: maps up to DT_NOALLOC_MAX_CELLS cells and DT_NOALLOC_MAX_SIDE
// rows and columns (the caller checks), on the current device.
constexpr int DT_NOALLOC_MAX_SIDE = 16384;
constexpr int64_t DT_NOALLOC_MAX_CELLS = (int64_t)1 << 21;
// Single-map transform by lower envelopes (one thread per line).  hx, hz:
// rows * cols int32 / double of scratch; ay is required (the column pass's
// argmax), ax optional.
hipError_t launch_dt_envelope(const float* resp, int rows, int cols, int ld, const float* d, float* r1v,
                              int32_t* r1a, int32_t* hx, double* hz, float* out, int32_t* ay, int32_t* ax,
                              hipStream_t st);
hipError_t launch_dt_single_noalloc(const float* resp, int rows, int cols, int ld, const float* d,
                                    float* out, int32_t* ay, int32_t* ax, hipStream_t st);

}  // namespace dpmt
