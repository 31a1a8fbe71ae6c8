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
// stored as a [position][ng] float32 block, position = y * Wo + x.
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
// (BB * 32) filters of one group on one level.
struct CorrTile {
    int64_t z_cell;    // first cell of the level in the feature / projected buffer
    int64_t out_off;   // element offset of the group's response block on this level
    int32_t H, W;      // level rows, cols
    int32_t Ho, Wo;    // response rows, cols
    int32_t y0, x0;    // first output row, col
    int32_t fb0;       // first 32-filter block
    int32_t group;
};

// One (component, part slot) whose part filter belongs to a part group.
struct PairDesc {
    int32_t fcol;      // column of the part filter in the group's response block
    int32_t comp, slot;
    int32_t vy, vx;    // anchor (part-level cells)
    int32_t h0, w0;    // root filter shape of the component
    int32_t pad;
    float d[4];        // d_x, d_xx, d_y, d_yy
};

// Distance-transform work for one (image, root level, part group).
struct DTItem {
    int64_t resp_off;  // part responses [Hp][Wp][ng]
    int64_t r1_off;    // row-pass output [np][Hp][Wt] (value and argmax share indexing)
    int32_t Hp, Wp;    // part response map
    int32_t Ht, Wt;    // largest root map over the group's components
    int32_t Hr, Wr;    // root level rows, cols
    int32_t ng, np;    // filters in the group, pairs in the group
    int32_t pair_base; // first pair of the group in the pair table
    int32_t map_base;  // map index of component 0 at this (image, root level)
    int32_t cw;        // root columns per column-pass block
    int32_t pad;
};

// One score map (image, root level, component).
struct MapDesc {
    int64_t score_off; // float offset into the caller's scores
    int64_t offs_off;  // int16 offset into the caller's offsets ([part][pos][2])
    int64_t rresp_off; // root response block of the root group on this level
    int32_t Ho, Wo;
    int32_t n_parts;
    int32_t rng, rcol; // root group width and the root filter's column
    int32_t pad;
};

// Correlation kernel flavours.
enum CorrKind { CORR_F32 = 0, CORR_BF16 = 1, CORR_FP8 = 2 };

struct CorrLaunch {
    CorrKind kind;
    Packing pk;
    int ty;            // output rows per wave
    int bb;            // 32-filter blocks per wave
    int wy;            // waves per workgroup (stacked along rows)
};

// --- kernel launchers (dpmt_kernels.hip) -----------------------------------
hipError_t launch_project(bool bf16, const float* X, int64_t n_cells, const float* U,
                          int RP, void* Z, hipStream_t st);
hipError_t launch_corr(const CorrLaunch& cfg, const CorrTile* tiles, int n_tiles,
                       const GroupDesc* groups, const void* Z, const void* G, const float* tk,
                       float* out, int max_h, int max_S, hipStream_t st);
hipError_t launch_fp8_prepare(const float* X, int64_t n_cells, const float* U, int RP,
                              float* partial, float* scales, const RequantBlock* blocks,
                              int n_blocks, const float* master, uint8_t* G, float* tk,
                              hipStream_t st);
hipError_t launch_project_fp8(const float* X, int64_t n_cells, const float* U, int RP,
                              const float* scales, void* Z, hipStream_t st);
constexpr int FP8_PARTIALS = 512 * 32;   // floats of the channel-max scratch
size_t corr_lds_bytes(const CorrLaunch& cfg, int h, int S);
hipError_t launch_dt_row(const DTItem* items, const int2* blkmap, int n_blocks,
                         const PairDesc* pairs, const float* resp, float* r1v, int32_t* r1a,
                         int max_line, hipStream_t st);
hipError_t launch_dt_col(const DTItem* items, const int2* blkmap, int n_blocks,
                         const PairDesc* pairs, const MapDesc* maps, const float* r1v,
                         const int32_t* r1a, float* dbuf, int16_t* offs, int max_line,
                         hipStream_t st);
hipError_t launch_assemble(const MapDesc* maps, const int2* blkmap, int n_blocks,
                           const float* rresp, const float* dbuf, float* scores, hipStream_t st);
hipError_t launch_block_to_maps(const float* block, int64_t n_pos, int ng, const int64_t* dst_off,
                                float* out, hipStream_t st);
hipError_t launch_dt_single(const float* resp, int rows, int cols, int ld, const float* d,
                            float* lmax, float* r1v, int32_t* r1a, float* out, int32_t* ay,
                            int32_t* ax, hipStream_t st);

// Workgroup sizes used by the launchers (the planner sizes work lists with them).
constexpr int DT_ROW_PAIRS_PER_BLOCK = 32;   // row pass: one part row of 32 pairs per block
constexpr int DT_COL_LDS = 96 * 1024;        // column pass: LDS bytes of one staged [Hp][cw] tile
constexpr int ASM_BLOCK = 256;         // assembly: threads per block

}  // namespace dpmt
