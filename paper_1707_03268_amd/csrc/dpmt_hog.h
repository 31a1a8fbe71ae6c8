// Internal types of the HOG feature pyramid shared by the host runtime
// (dpmt_host.cpp) and its kernels (dpmt_hog.hip).  Nothing here is part of
// the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace dpmt {

// One level of the HOG feature pyramid (dpmt_hog_pyramid): where its padded
// cells go in the packed feature buffer and where its interior cells'
// histograms go in the scratch.
struct HogLevelDesc {
    int64_t cell_offset;  // first cell of the level in the packed float32 HWC buffer
    int64_t hist_off;     // first interior cell of the level in the histogram scratch
    int32_t rows, cols;   // padded cells
    int32_t pad_rows, pad_cols;
    int32_t nr, nc;       // interior cells
    int32_t cell;         // resized pixels per cell side (4 or 8)
    float inv_scale;      // source pixels per resized pixel
};
// The 9 directions o pi / 9 as float32 (cos, sin).
struct HogTable {
    float u[9], v[9];
};
// Histogram pass over tiles (level, tile row, tile col, 0) of 32 x 32 resized
// pixels, then the feature pass over blocks (level, first padded cell) of 256
// cells.  hist: 18 floats per interior cell, energy: 1 float per interior cell.
hipError_t launch_hog(const uint8_t* img, int H, int W, const HogLevelDesc* levels, const int4* tiles,
                      int n_tiles, const int2* blocks, int n_blocks, const HogTable& tab, float* hist,
                      float* energy, float* feats, hipStream_t st);
constexpr int HOG_TILE_PIXELS = 32;

}  // namespace dpmt
