// HOG feature pyramid on the GPU: the feature map phi that the scores are
// computed on (Section 2), 32 values per cell (Section 5, L = 32), in the
// 32-value variant of Felzenszwalb et al. (PAMI 2010, Section 6):
//
//   1. every level samples the image bilinearly at its own scale;
//   2. centred gradients, the colour channel with the largest squared norm;
//   3. the direction among 18 (o pi / 9) with the largest projection;
//   4. magnitude votes spread bilinearly over the 4 nearest cell centres;
//   5. 4 normalisers per cell from the energies of the 2x2-cell blocks that
//      contain it;
//   6. truncated ratios summed into 18 contrast-sensitive, 9 insensitive and
//      4 texture channels; channel 31 marks the padding band.
//
// Steps 1-3 decide integers from floating point.  They run in float32 with
// every product, sum and difference rounded on its own (contraction is off
// for this file), so the decisions are a fixed function of the inputs.  Ties
// go to the first channel and the first direction.
//
// Two kernels per call.  hog_hist_kernel: one workgroup per tile of 32 x 32
// resized pixels (8 x 8 cells of 4 pixels, or 4 x 4 cells of 8); the
// sampled tile with its halo, the per-pixel votes and per-thread partial
// histograms live in LDS; it writes the tile's 18-bin cell histograms and
// their energies.  hog_feat_kernel: one thread per padded cell; it reads its
// histogram and the 9 energies around it and writes the cell's 32 floats.
#include "dpmt_hog.h"

#include <cmath>

// Every product and sum in this file rounds on its own: no contraction into
// fused multiply-adds (fmaf, where written, is meant).
#pragma clang fp contract(off)

namespace dpmt {

namespace {

constexpr int HOG_TILE = HOG_TILE_PIXELS;          // resized pixels per tile side
constexpr int HOG_MAX_CELL = 8;
constexpr int HOG_S = HOG_TILE + HOG_MAX_CELL + 2; // sampled side: votes + gradient halo
constexpr int HOG_V = HOG_TILE + HOG_MAX_CELL;     // vote side: the cells' 2c windows
constexpr int HOG_BINS = 18;
constexpr float HOG_ALPHA = 0.2f;
constexpr float HOG_HALF = 0.5f;
constexpr float HOG_EPS = 1e-4f;

// Step 1 for one coordinate: source index pair and weight of the upper one.
__device__ __forceinline__ void hog_coord(int t, float k, int n, int& i0, int& i1, float& f) {
    float s = ((((float)t + 0.5f) * k) - 0.5f);
    s = fminf(fmaxf(s, 0.f), (float)(n - 1));
    const float fl = floorf(s);
    i0 = (int)fl;
    i1 = min(i0 + 1, n - 1);
    f = (s - fl);
}

__device__ __forceinline__ float hog_lerp(float g, float f, float a, float b) {
    return ((g * a) + (f * b));
}

}  // namespace

__global__ __launch_bounds__(256) void hog_hist_kernel(const uint8_t* __restrict__ img, int H, int W,
                                                       const HogLevelDesc* __restrict__ levels,
                                                       const int4* __restrict__ tiles, HogTable tab,
                                                       float* __restrict__ hist,
                                                       float* __restrict__ energy) {
    extern __shared__ __align__(16) float hsm[];
    float* simg = hsm;                                             // [3][HOG_S][HOG_S]
    float* smag = simg + 3 * HOG_S * HOG_S;                        // [HOG_V][HOG_V]
    uint8_t* sbin = reinterpret_cast<uint8_t*>(smag + HOG_V * HOG_V);   // [HOG_V][HOG_V]
    float* part = simg;                                            // [256][18], reuses simg

    const int4 tl = tiles[blockIdx.x];
    const HogLevelDesc L = levels[tl.x];
    const int c = L.cell, T = HOG_TILE / c;
    const int Hr = L.nr * c, Wr = L.nc * c;                        // resized pixels that vote
    const int Y0 = tl.y * HOG_TILE, X0 = tl.z * HOG_TILE;
    const int S = HOG_TILE + c + 2, V = HOG_TILE + c;
    const int ys = Y0 - c / 2 - 1, xs = X0 - c / 2 - 1;            // resized pixel of simg[.][0][0]
    const int tid = threadIdx.x;

    // 1. bilinear samples of the tile and its halo, three channels
    for (int p = tid; p < S * S; p += 256) {
        const int r = p / S, q = p - r * S;
        int y0, y1, x0, x1;
        float fy, fx;
        hog_coord(ys + r, L.inv_scale, H, y0, y1, fy);
        hog_coord(xs + q, L.inv_scale, W, x0, x1, fx);
        const float gy = (1.f - fy), gx = (1.f - fx);
        const uint8_t* a = img + ((int64_t)y0 * W) * 3;
        const uint8_t* b = img + ((int64_t)y1 * W) * 3;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const float top = hog_lerp(gx, fx, (float)a[x0 * 3 + ch], (float)a[x1 * 3 + ch]);
            const float bot = hog_lerp(gx, fx, (float)b[x0 * 3 + ch], (float)b[x1 * 3 + ch]);
            simg[(ch * HOG_S + r) * HOG_S + q] = hog_lerp(gy, fy, top, bot);
        }
    }
    __syncthreads();

    // 2, 3. per-pixel channel, direction and magnitude; pixels outside the
    // level's cell grid do not vote
    for (int p = tid; p < V * V; p += 256) {
        const int r = p / V, q = p - r * V;
        const int y = ys + 1 + r, x = xs + 1 + q;
        float m2b = -1.f, gxb = 0.f, gyb = 0.f;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const float* s = simg + (ch * HOG_S + r + 1) * HOG_S + q + 1;
            const float dx = (s[1] - s[-1]);
            const float dy = (s[HOG_S] - s[-HOG_S]);
            const float m2 = ((dx * dx) + (dy * dy));
            if (m2 > m2b) { m2b = m2; gxb = dx; gyb = dy; }
        }
        int bin = 0;
        float best = ((gxb * tab.u[0]) + (gyb * tab.v[0]));
#pragma unroll
        for (int o = 1; o < HOG_BINS; ++o) {
            const float pr = ((gxb * tab.u[o % 9]) + (gyb * tab.v[o % 9]));
            const float d = o < 9 ? pr : -pr;
            if (d > best) { best = d; bin = o; }
        }
        const bool in = (unsigned)y < (unsigned)Hr && (unsigned)x < (unsigned)Wr;
        smag[r * HOG_V + q] = in ? sqrtf(m2b) : 0.f;
        sbin[r * HOG_V + q] = (uint8_t)bin;
    }
    __syncthreads();

    // 4. votes: thread t < 4 T^2 owns quadrant item t (item = 4 * cell +
    // quadrant); a cell's window is its 2c x 2c pixels, the upper-left
    // quadrant taking the pixels whose upper-left cell centre is this cell's
    // upper-left neighbour
    const int items = 4 * T * T;                                   // 256 (c = 4) or 64 (c = 8)
    float* mine = part + tid * HOG_BINS;
    const float invc = 1.f / (float)c;                             // exact (power of two)
    if (tid < items) {
        for (int b = 0; b < HOG_BINS; ++b) mine[b] = 0.f;
        const int item = tid, cell = item >> 2, quad = item & 3;
        const int ci = cell / T, cj = cell - ci * T;
        const int gi = Y0 / c + ci, gj = X0 / c + cj;              // level cell
        const int r0 = ci * c + (quad >> 1) * c, q0 = cj * c + (quad & 1) * c;
        for (int rr = 0; rr < c; ++rr) {
            const int y = ys + 1 + r0 + rr;
            const float yp = ((((float)y + 0.5f) * invc) - 0.5f);
            const float iy = floorf(yp), w1 = (yp - iy);
            const float wy = (int)iy == gi ? (1.f - w1) : w1;
            for (int qq = 0; qq < c; ++qq) {
                const int x = xs + 1 + q0 + qq;
                const float xp = ((((float)x + 0.5f) * invc) - 0.5f);
                const float ix = floorf(xp), v1 = (xp - ix);
                const float wx = (int)ix == gj ? (1.f - v1) : v1;
                const int pi = (r0 + rr) * HOG_V + q0 + qq;
                mine[sbin[pi]] += smag[pi] * wy * wx;
            }
        }
    }
    __syncthreads();

    // cell totals (the 4 quadrant partials in order), histogram and energy out
    const int cells = T * T;
    for (int cell = tid; cell < cells; cell += 256) {
        const int ci = cell / T, cj = cell - ci * T;
        const int gi = Y0 / c + ci, gj = X0 / c + cj;
        if (gi >= L.nr || gj >= L.nc) continue;
        float h[HOG_BINS];
        const int t0 = 4 * cell;                                   // the 4 threads holding its quadrants
#pragma unroll
        for (int b = 0; b < HOG_BINS; ++b)
            h[b] = ((part[t0 * HOG_BINS + b] + part[(t0 + 1) * HOG_BINS + b]) + part[(t0 + 2) * HOG_BINS + b]) +
                   part[(t0 + 3) * HOG_BINS + b];
        float e = 0.f;
#pragma unroll
        for (int o = 0; o < 9; ++o) {
            const float d = h[o] + h[o + 9];
            e = fmaf(d, d, e);
        }
        const int64_t idx = L.hist_off + (int64_t)gi * L.nc + gj;
        float* out = hist + idx * HOG_BINS;
#pragma unroll
        for (int b = 0; b < HOG_BINS; ++b) out[b] = h[b];
        energy[idx] = e;
    }
}

__global__ __launch_bounds__(256) void hog_feat_kernel(const HogLevelDesc* __restrict__ levels,
                                                       const int2* __restrict__ blocks,
                                                       const float* __restrict__ hist,
                                                       const float* __restrict__ energy,
                                                       float* __restrict__ feats) {
    const int2 bk = blocks[blockIdx.x];
    const HogLevelDesc L = levels[bk.x];
    const int p = bk.y + (int)threadIdx.x;
    if (p >= L.rows * L.cols) return;
    const int r = p / L.cols, q = p - r * L.cols;
    const int i = r - L.pad_rows, j = q - L.pad_cols;
    float f[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) f[k] = 0.f;
    if ((unsigned)i < (unsigned)L.nr && (unsigned)j < (unsigned)L.nc) {
        auto E = [&](int a, int b) -> float {
            return ((unsigned)a < (unsigned)L.nr && (unsigned)b < (unsigned)L.nc)
                       ? energy[L.hist_off + (int64_t)a * L.nc + b] : 0.f;
        };
        const float e = E(i, j);
        const float up = E(i - 1, j), dn = E(i + 1, j), lf = E(i, j - 1), rt = E(i, j + 1);
        float inv[4];
        inv[0] = 1.f / sqrtf(e + up + lf + E(i - 1, j - 1) + HOG_EPS);
        inv[1] = 1.f / sqrtf(e + up + rt + E(i - 1, j + 1) + HOG_EPS);
        inv[2] = 1.f / sqrtf(e + dn + lf + E(i + 1, j - 1) + HOG_EPS);
        inv[3] = 1.f / sqrtf(e + dn + rt + E(i + 1, j + 1) + HOG_EPS);
        const float* h = hist + (L.hist_off + (int64_t)i * L.nc + j) * HOG_BINS;
        float hb[HOG_BINS];
#pragma unroll
        for (int b = 0; b < HOG_BINS; ++b) hb[b] = h[b];
        float tex[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int o = 0; o < HOG_BINS; ++o) {
            float s = 0.f;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float t = fminf(hb[o] * inv[k], HOG_ALPHA);
                s += t;
                tex[k] += t;
            }
            f[o] = HOG_HALF * s;
        }
#pragma unroll
        for (int o = 0; o < 9; ++o) {
            const float d = hb[o] + hb[o + 9];
            float s = 0.f;
#pragma unroll
            for (int k = 0; k < 4; ++k) s += fminf(d * inv[k], HOG_ALPHA);
            f[18 + o] = HOG_HALF * s;
        }
        const float tau = 0.23570226039551584f;                    // 1 / sqrt(18)
#pragma unroll
        for (int k = 0; k < 4; ++k) f[27 + k] = tau * tex[k];
    } else {
        f[31] = 1.f;                                               // padding band
    }
    float4* out = reinterpret_cast<float4*>(feats + (L.cell_offset + p) * 32);
#pragma unroll
    for (int k = 0; k < 8; ++k) out[k] = make_float4(f[4 * k], f[4 * k + 1], f[4 * k + 2], f[4 * k + 3]);
}

size_t hog_lds_bytes() {
    return (size_t)4 * (3 * HOG_S * HOG_S + HOG_V * HOG_V) + (size_t)HOG_V * HOG_V;
}

hipError_t launch_hog(const uint8_t* img, int H, int W, const HogLevelDesc* levels, const int4* tiles,
                      int n_tiles, const int2* blocks, int n_blocks, const HogTable& tab, float* hist,
                      float* energy, float* feats, hipStream_t st) {
    static_assert(256 * HOG_BINS <= 3 * HOG_S * HOG_S, "partial histograms fit in the sampled tile");
    static_assert(4 * (HOG_TILE / 4) * (HOG_TILE / 4) <= 256, "one quadrant item per thread");
    const size_t bytes = hog_lds_bytes();
    if (n_tiles > 0) {
        if (bytes > 65536) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(hog_hist_kernel),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(hog_hist_kernel, dim3((unsigned)n_tiles), dim3(256), bytes, st, img, H, W,
                           levels, tiles, tab, hist, energy);
    }
    if (n_blocks > 0)
        hipLaunchKernelGGL(hog_feat_kernel, dim3((unsigned)n_blocks), dim3(256), 0, st, levels, blocks,
                           hist, energy, feats);
    return hipGetLastError();
}

}  // namespace dpmt
