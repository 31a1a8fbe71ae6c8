// HIP kernels of libdpmt for gfx950 (CDNA4, 64-lane wavefronts).
//
//   project_kernel     Z = X x_3 U^T per cell (feature contraction of the
//                      tensor form, Section 4), VALU, HBM bound
//   corr_kernel        valid correlation of one level with a group of
//                      equally sized filters as a shift-GEMM on MFMA
//                      (positions x filters x (taps * channels)), FP32 or BF16
//                      operands, FP32 accumulation; used for the direct and
//                      the shortened (rank-R) responses
//   place_kernel       separable generalised distance transform (Section 2
//                      placement argmax) evaluated at the part anchors of
//                      every root position, exact windowed scans, fused with
//                      s(p0) = root response + sum of the parts' deformed
//                      scores (Section 2 score formula)
//   dt1_*_kernel       the same transform for every cell of one map
#include "dpmt_internal.h"

#include <algorithm>
#include <cfloat>
#include <climits>
#include <mutex>

namespace dpmt {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// Launch index -> work item for a grid padded by xcd_grid (clusters of 2^XCL
// consecutive items on one XCD); items >= n are padding.
template <int XCL>
__device__ __forceinline__ int xcd_item(int g) {
    const int xcd = g & (N_XCD - 1), k = g / N_XCD;
    return (((k >> XCL) * N_XCD + xcd) << XCL) + (k & ((1 << XCL) - 1));
}

// Order-preserving map between float32 and int32, so that integer atomic
// max / min keep float value ranges.
__device__ __forceinline__ int range_key(float f) {
    const int i = __float_as_int(f);
    return i >= 0 ? i : i ^ 0x7fffffff;
}
__device__ __forceinline__ float range_value(int k) {
    return __int_as_float(k >= 0 ? k : k ^ 0x7fffffff);
}

// ---------------------------------------------------------------------------
// projection: Z[c][r] = sum_l X[c][l] * U[l][r]   (U: 32 x RP fp32, row major)
// ---------------------------------------------------------------------------
// rkeys (may be NULL): the 2 * n_slots range keys, reset here (maxima to
// INT_MIN, minima to INT_MAX) in place of a launch of their own.
template <int RP, bool BF16>
__global__ __launch_bounds__(256) void project_kernel(const float* __restrict__ X, int64_t n_cells,
                                                      const float* __restrict__ U,
                                                      void* __restrict__ Zv, int* __restrict__ rkeys,
                                                      int64_t n_slots) {
    __shared__ float sU[32 * RP];
    if (rkeys != nullptr)
        for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n_slots; i += (int64_t)gridDim.x * 256) {
            rkeys[i] = INT_MIN;
            rkeys[n_slots + i] = INT_MAX;
        }
    for (int i = threadIdx.x; i < 32 * RP; i += 256) sU[i] = U[i];
    __syncthreads();
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= n_cells) return;
    const float4* x4 = reinterpret_cast<const float4*>(X + c * 32);
    float acc[RP];
#pragma unroll
    for (int r = 0; r < RP; ++r) acc[r] = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const float4 v = x4[k];
#pragma unroll
        for (int r = 0; r < RP; ++r) {
            acc[r] = fmaf(v.x, sU[(4 * k + 0) * RP + r], acc[r]);
            acc[r] = fmaf(v.y, sU[(4 * k + 1) * RP + r], acc[r]);
            acc[r] = fmaf(v.z, sU[(4 * k + 2) * RP + r], acc[r]);
            acc[r] = fmaf(v.w, sU[(4 * k + 3) * RP + r], acc[r]);
        }
    }
    if constexpr (BF16) {
        __bf16* z = reinterpret_cast<__bf16*>(Zv) + c * RP;
#pragma unroll
        for (int r = 0; r < RP; ++r) z[r] = static_cast<__bf16>(acc[r]);
    } else {
        float* z = reinterpret_cast<float*>(Zv) + c * RP;
#pragma unroll
        for (int r = 0; r < RP; ++r) z[r] = acc[r];
    }
}

hipError_t launch_project(bool bf16, const float* X, int64_t n_cells, const float* U, int RP,
                          void* Z, int* rkeys, int64_t n_slots, hipStream_t st) {
    if (n_cells <= 0) return rkeys ? launch_range_init(rkeys, n_slots, st) : hipSuccess;
    const unsigned nb = (unsigned)((n_cells + 255) / 256);
#define DPMT_PROJ(R)                                                                          \
    case R:                                                                                   \
        if (bf16) hipLaunchKernelGGL((project_kernel<R, true>), dim3(nb), dim3(256), 0, st,   \
                                     X, n_cells, U, Z, rkeys, n_slots);                       \
        else hipLaunchKernelGGL((project_kernel<R, false>), dim3(nb), dim3(256), 0, st, X,    \
                                n_cells, U, Z, rkeys, n_slots);                               \
        break;
    switch (RP) {
        DPMT_PROJ(4)
        DPMT_PROJ(8)
        DPMT_PROJ(16)
        DPMT_PROJ(24)
        DPMT_PROJ(32)
        default: return hipErrorInvalidValue;
    }
#undef DPMT_PROJ
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// correlation as a shift-GEMM on MFMA 32x32
//
// C[pos][f] = sum_{n < h} sum_{flattened row bytes o} Zrow(y+n)[x*PB + o] * Grow_f(n)[o]
// One wavefront owns TY output rows x 32 output cols x BB*32 filters.  The A
// operand (positions) is read from an LDS window of the level, one window row
// per fragment: the fragment of window row r serves output row i with filter
// row n = r - i, so a wave keeps TY row fragments live and slides them down
// the filter rows.  The B operand (filters) is pre-packed on the host in
// fragment order, 1 KB per (block, plane, step, filter row), and staged
// through a double-buffered LDS chunk per K-step.
// ---------------------------------------------------------------------------
constexpr int CORR_MAX_H = 16;
constexpr int CORR_NBUF = 3;                   // filter-chunk staging depth of the unrolled tiles

// Filter-chunk buffers of a tile: CORR_NBUF with direct global-to-LDS
// staging, two (plain double buffering) for the wide tiles, whose windows
// take the LDS, and for staging through registers.
__host__ __device__ constexpr int corr_chunk_buffers(bool dma, int wx) {
    return dma && wx == 1 ? CORR_NBUF : 2;
}

// Whether a correlation instance gives the 6-, 7- and 8-row filters fully
// unrolled bodies (staged CORR_NBUF chunks deep); host and device agree on it.
// FP8 fragments are twice as wide, so FP8 unrolls with one filter block per
// wavefront only.
__host__ __device__ constexpr bool corr_unrolls(CorrKind kind, int PB, int BB, int HMAX) {
    return HMAX >= 8 && !(PB == 32 && BB == 2) && (kind != CORR_FP8 || BB == 1);
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

// Per-lane operand fragment: 16 bytes (FP32: 4 x K=1 steps of 32x32x2; BF16:
// 8 values of 32x32x16) or 32 bytes (FP8: 32 values of 32x32x64).
template <CorrKind KIND> struct FragT { typedef u32x4 type; static constexpr int bytes = 16; };
template <> struct FragT<CORR_FP8> { typedef u32x8 type; static constexpr int bytes = 32; };

__device__ __forceinline__ u32x4 lds_load16(const char* p, int pb) {
    if (pb >= 16) return *reinterpret_cast<const u32x4*>(p);
    const u32x2 a = *reinterpret_cast<const u32x2*>(p);
    const u32x2 b = *reinterpret_cast<const u32x2*>(p + 8);
    return u32x4{a.x, a.y, b.x, b.y};
}

template <CorrKind KIND>
__device__ __forceinline__ v16f mfma_step(const typename FragT<KIND>::type& a,
                                          const typename FragT<KIND>::type& b, v16f c) {
    if constexpr (KIND == CORR_F32) {
        c = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.x), __uint_as_float(b.x), c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.y), __uint_as_float(b.y), c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.z), __uint_as_float(b.z), c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.w), __uint_as_float(b.w), c, 0, 0, 0);
        return c;
    } else if constexpr (KIND == CORR_BF16) {
        v8bf av, bv;
        __builtin_memcpy(&av, &a, 16);
        __builtin_memcpy(&bv, &b, 16);
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, c, 0, 0, 0);
    } else {
        // OCP e4m3 operands (format 0 for A and B), unit block scales (E8M0 127)
        i32x8 av, bv;
        __builtin_memcpy(&av, &a, 32);
        __builtin_memcpy(&bv, &b, 32);
        return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av, bv, c, 0, 0, 0, 127, 0, 127);
    }
}

// Fragment load from LDS at the alignment the plane width allows.
template <CorrKind KIND>
__device__ __forceinline__ typename FragT<KIND>::type lds_frag(const char* p, int pb) {
    if constexpr (FragT<KIND>::bytes == 16) {
        return lds_load16(p, pb);
    } else {
        const u32x4 lo = lds_load16(p, pb), hi = lds_load16(p + 16, pb);
        return u32x8{lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
    }
}

// Epilogue of one group of BB filter blocks (first block fbb): lane holds
// filter column p, positions x0 + 8*(k/4) + 4*j + k%4, i.e. four runs of 4
// consecutive positions stored as 16-byte vectors into the filter's plane (the
// pitch is a multiple of 4, so a run that starts inside the map ends inside
// the pitch).  The value range of every plane over its valid positions goes to
// the range slots.
template <CorrKind KIND, int TY, int BB, int WY, int WX>
__device__ __forceinline__ void corr_epilogue(const CorrTile& t, const GroupDesc& g, int fbb,
                                              const v16f (&acc)[TY][BB],
                                              const float* __restrict__ tk, float* __restrict__ out,
                                              int* __restrict__ rmax, int* __restrict__ rmin) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int p = lane & 31, j = lane >> 5;
    const int wr = wv / WX, x0 = t.x0 + 32 * (wv % WX);   // the wave's rows and columns
    float vmax[BB], vmin[BB];
#pragma unroll
    for (int b = 0; b < BB; ++b) {
        vmax[b] = -INFINITY;
        vmin[b] = INFINITY;
    }
#pragma unroll
    for (int i = 0; i < TY; ++i) {
        const int y = t.y0 + wr * TY + i;
        if (y >= t.Ho) continue;
#pragma unroll
        for (int b = 0; b < BB; ++b) {
            const int f = (fbb + b) * 32 + p;
            if (f >= g.ng) continue;
            float* orow = out + t.out_off + ((int64_t)f * t.Ho + y) * t.ld + x0 + 4 * j;
            const float sc = (KIND == CORR_FP8) ? tk[g.t_off + f] : 1.f;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int x = x0 + 8 * m + 4 * j;
                if (x >= t.Wo) continue;
                float4 v;
                v.x = acc[i][b][4 * m + 0] * sc;
                v.y = acc[i][b][4 * m + 1] * sc;
                v.z = acc[i][b][4 * m + 2] * sc;
                v.w = acc[i][b][4 * m + 3] * sc;
                *reinterpret_cast<float4*>(orow + 8 * m) = v;
                if (x + 3 < t.Wo) {                 // whole run inside the map: two 3-input max / min
                    vmax[b] = fmaxf(fmaxf(vmax[b], v.x), fmaxf(v.y, fmaxf(v.z, v.w)));
                    vmin[b] = fminf(fminf(vmin[b], v.x), fminf(v.y, fminf(v.z, v.w)));
                } else {                            // the run that crosses the last column
                    vmax[b] = fmaxf(vmax[b], v.x);
                    vmin[b] = fminf(vmin[b], v.x);
                    if (x + 1 < t.Wo) { vmax[b] = fmaxf(vmax[b], v.y); vmin[b] = fminf(vmin[b], v.y); }
                    if (x + 2 < t.Wo) { vmax[b] = fmaxf(vmax[b], v.z); vmin[b] = fminf(vmin[b], v.z); }
                }
            }
        }
    }
    if (rmax != nullptr && t.rng >= 0) {
#pragma unroll
        for (int b = 0; b < BB; ++b) {
            const float hi = fmaxf(vmax[b], __shfl_xor(vmax[b], 32, 64));
            const float lo = fminf(vmin[b], __shfl_xor(vmin[b], 32, 64));
            const int f = (fbb + b) * 32 + p;
            if (j == 0 && f < g.ng && hi >= lo) {
                atomicMax(rmax + t.rng + f, range_key(hi));
                atomicMin(rmin + t.rng + f, range_key(lo));
            }
        }
    }
}

// HS > 0: the tile's filters have exactly HS rows, and the filter-row loop is
// fully unrolled over a static ring of A fragments (no register rotation, exact
// LDS waits); HS = 0: any height up to HMAX with a rolled loop.
template <CorrKind KIND, int PB, int TY, int BB, int WY, int WX, int HMAX, int HS>
__device__ __forceinline__ void corr_tile(const CorrTile& t, const GroupDesc* __restrict__ groups,
                                          const char* __restrict__ Z, const char* __restrict__ G,
                                          const float* __restrict__ tk, float* __restrict__ out,
                                          int* __restrict__ rmax, int* __restrict__ rmin,
                                          int cell_bytes, int Q, int win_bytes) {
    extern __shared__ __align__(16) char smem[];
    constexpr int NT = 64 * WY;
    static_assert(WY % WX == 0, "waves along x must divide the workgroup");
    constexpr int TYWG = TY * (WY / WX);           // output rows of the workgroup tile
    constexpr int CH = PB >= 16 ? 16 : 8;          // window copy granule
    constexpr int FB = FragT<KIND>::bytes;         // fragment bytes per lane
    constexpr int KS = 2 * FB;                     // flattened row bytes per K-step
    constexpr int CU = 4 * FB;                     // u32x4 per (block, plane, step, row) chunk
    typedef typename FragT<KIND>::type Frag;
    constexpr int PFMAX = (BB * HMAX * CU + NT - 1) / NT;   // chunk u32x4 per thread, h <= HMAX
    constexpr int WBATCH = 4;                      // window loads in flight per thread

    const GroupDesc g = groups[t.group];
    const int h = HS > 0 ? HS : g.h, S = g.S;
    const int WC = 32 * WX - 1 + (KS * S) / PB;    // window cells per row
    const int pitch = WC * PB;
    const int nrows = TYWG + h - 1;
    char* win = smem;
    u32x4* gbuf0 = reinterpret_cast<u32x4*>(smem + win_bytes);
    u32x4* gbuf1 = gbuf0 + BB * h * CU;
    // Unrolled heights stage the filter chunks with direct global-to-LDS loads,
    // CORR_NBUF buffers deep (the chunks of steps gs + 1 .. gs + CORR_NBUF - 1
    // are in flight while step gs computes); each wavefront loads UPW units
    // of a chunk, a unit (one filter row of one block: 64 fragments) being
    // LPU loads of 1 KB.  Other tiles stage through registers, two buffers.
    constexpr bool DMA = HS > 0;
    constexpr int UPW = DMA ? (BB * HS + WY - 1) / WY : 1;
    constexpr int LPU = FB / 16;                   // 1 KB loads per unit
    constexpr int NB = corr_chunk_buffers(DMA, WX);
    static_assert(!DMA || (NB - 2) * UPW * LPU <= 15, "outstanding chunk loads must fit the vmcnt immediate");
    auto gbuf = [&](int k) { return gbuf0 + k * (BB * h * CU); };

    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int p = lane & 31, j = lane >> 5;
    // in a tile of several wavefronts along x, a wavefront whose 32 columns
    // all lie right of the map (the last tile of a level rarely fills all of
    // 32 * WX) loads and waits with the others but issues no MFMA
    const bool xlive = WX == 1 || t.x0 + 32 * (__builtin_amdgcn_readfirstlane(wv) % WX) < t.Wo;

    v16f acc[TY][BB];
#pragma unroll
    for (int i = 0; i < TY; ++i)
#pragma unroll
        for (int b = 0; b < BB; ++b)
#pragma unroll
            for (int k = 0; k < 16; ++k) acc[i][b][k] = 0.f;

    const int n_chunk = BB * h * CU;               // u32x4 per G chunk
    const int total = Q * S;
    // Element i of a chunk is [b][n][lane] of the packed operand; thread tid
    // owns elements tid + k*NT (clamped to the chunk's last element, whose value
    // surplus threads then store again).  Its source address for step `st` is
    // pf_base[k] + st * h * chunk bytes: the division by h happens once per tile.
    const int chunk_bytes = 64 * FB;
    uint32_t pf_base[PFMAX];                       // byte offsets into G (< 4 GiB)
    int pf_dst[PFMAX];
#pragma unroll
    for (int k = 0; k < PFMAX; ++k) {
        const int i = min(tid + k * NT, n_chunk - 1);
        const int l = i % CU;
        const int n = (i / CU) % h;
        const int b = i / (CU * h);
        pf_base[k] = (uint32_t)(g.g_off + (((int64_t)(t.fb0 + b) * Q * S) * h + n) * chunk_bytes + l * 16);
        pf_dst[k] = i;
    }
    const uint32_t step_bytes = (uint32_t)(h * chunk_bytes);
    auto chunk_ld = [&](int st, int k) -> u32x4 {
        return *reinterpret_cast<const u32x4*>(G + (pf_base[k] + (uint32_t)st * step_bytes));
    };

    // window fill: thread -> (row offset r0, 16/8-byte chunk c of a row), one
    // division per tile; rows advance by rpp
    const int cpc = PB / CH;
    const int cpr = WC * cpc;                      // chunks per window row
    const int rpp = max(NT / cpr, 1);              // rows per pass
    const int wr0 = tid / cpr, wc = tid - wr0 * cpr;
    const int wcc = wc / cpc, wk = wc - wcc * cpc; // cell, chunk within the cell
    const bool wact = wr0 < rpp;
    const int wx = t.x0 + wcc;

    // chunk cidx = group * BB * total + step: unit (b, n) of the packed operand
    // of block fb0 + b lies at ((fb0 + b) * total + cidx) * h + n units of
    // chunk_bytes (64 fragments: 1 KB, 2 KB for FP8)
    const int wvu = __builtin_amdgcn_readfirstlane(wv);
    auto dma_chunk = [&](int cidx, u32x4* dst) {
#pragma unroll
        for (int m = 0; m < UPW; ++m) {
            const int u = min(wvu + WY * m, BB * HS - 1);  // surplus waves reload the last unit
            const int b = u / (HS > 0 ? HS : 1), n = u - b * (HS > 0 ? HS : 1);
            const char* src = G + g.g_off +
                              ((int64_t)((t.fb0 + b) * total + cidx) * (HS > 0 ? HS : 1) + n) * chunk_bytes + lane * 16;
#pragma unroll
            for (int k = 0; k < LPU; ++k)
                __builtin_amdgcn_global_load_lds((__attribute__((address_space(1))) void*)(src + k * 1024),
                                                 (__attribute__((address_space(3))) void*)(reinterpret_cast<char*>(dst) + u * chunk_bytes + k * 1024),
                                                 16, 0, 0);
        }
    };

    // chunk index of global step gs2 (group gs2 / total, step gs2 % total)
    auto chunk_of = [&](int gs2) {
        const int f = gs2 / total;
        return f * BB * total + (gs2 - f * total);
    };
    // prologue: the chunks of steps 0 .. NB - 2 into buffers 0 .. NB - 2
    if constexpr (DMA) {
#pragma unroll
        for (int k = 0; k + 1 < NB; ++k)
            if (k < t.nfb * total) dma_chunk(chunk_of(k), gbuf(k));
    } else {
        u32x4 pf[PFMAX];
#pragma unroll
        for (int k = 0; k < PFMAX; ++k) pf[k] = chunk_ld(0, k);
#pragma unroll
        for (int k = 0; k < PFMAX; ++k) gbuf0[pf_dst[k]] = pf[k];
    }

    // The tile walks t.nfb groups of BB filter blocks over the same window:
    // global step gs = (group fbi, step st); the window of plane q is loaded
    // at the first group only when the level has one plane.  Each group ends
    // with its epilogue, whose stores drain while the next group computes.
    const int nsteps = t.nfb * total;
    int step = 0, fbi = 0, bi = 0;                 // bi = gs % NB (staging buffer of step gs)
    for (int gs = 0; gs < nsteps; ++gs) {
        const int q = step / S, s = step - q * S;
        if (s == 0 && (fbi == 0 || Q > 1)) {
            __syncthreads();                       // previous plane fully consumed
            if constexpr (DMA && PB >= 16) {
                // the whole window by direct global-to-LDS loads, 1 KB units
                // dealt to the wavefronts: lane byte o of the window is row
                // o / pitch, cell (o % pitch) / PB, byte o % PB of the cell's
                // plane-q run (16-byte pieces never straddle a cell).  Cells
                // beyond the level only feed outputs that are never kept, so
                // their addresses are clamped into the level.  One round trip,
                // then everything this wave issued has landed.
                const int nunits = (nrows * pitch + 1023) >> 10;
                const float inv_pitch = 1.f / (float)pitch;
                for (int u = wvu; u < nunits; u += WY) {
                    const int o = u * 1024 + lane * 16;
                    const int rr = (int)(((float)o + 0.5f) * inv_pitch);   // exact: o < 2^17
                    const int rem = o - rr * pitch;
                    const int y = min(t.y0 + rr, t.H - 1), x = min(t.x0 + rem / PB, t.W - 1);
                    const char* src = Z + ((t.z_cell + (int64_t)y * t.W + x) * cell_bytes + q * PB + (rem & (PB - 1)));
                    __builtin_amdgcn_global_load_lds((__attribute__((address_space(1))) void*)src,
                                                     (__attribute__((address_space(3))) void*)(win + u * 1024),
                                                     16, 0, 0);
                }
                __builtin_amdgcn_s_waitcnt(0xF70);                     // vmcnt(0)
            } else if (cpr <= NT) {
                for (int rb = 0; rb < nrows; rb += WBATCH * rpp) {
                    u32x4 r[WBATCH];
#pragma unroll
                    for (int u = 0; u < WBATCH; ++u) {
                        const int rr = min(rb + u * rpp + wr0, nrows - 1);
                        const int y = t.y0 + rr;
                        const bool in = wact && (y < t.H) && (wx < t.W);
                        const int64_t cell = t.z_cell + (in ? (int64_t)y * t.W + wx : 0);
                        const char* src = Z + (cell * cell_bytes + q * PB + wk * CH);
                        if constexpr (CH == 16) {
                            r[u] = *reinterpret_cast<const u32x4*>(src);
                        } else {
                            const u32x2 v = *reinterpret_cast<const u32x2*>(src);
                            r[u] = u32x4{v.x, v.y, 0u, 0u};
                        }
                        if (!in) r[u] = u32x4{0u, 0u, 0u, 0u};
                    }
#pragma unroll
                    for (int u = 0; u < WBATCH; ++u) {
                        const int rr = rb + u * rpp + wr0;
                        if (wact && rr < nrows) {
                            char* dst = win + rr * pitch + wcc * PB + wk * CH;
                            if constexpr (CH == 16) *reinterpret_cast<u32x4*>(dst) = r[u];
                            else *reinterpret_cast<u32x2*>(dst) = u32x2{r[u].x, r[u].y};
                        }
                    }
                }
            } else {                               // very wide rows: generic mapping
                const int nch = nrows * cpr;
                for (int i = tid; i < nch; i += NT) {
                    const int k = i % cpc, cc = (i / cpc) % WC, rr = i / cpr;
                    const int y = t.y0 + rr, x = t.x0 + cc;
                    const bool in = (y < t.H) && (x < t.W);
                    const int64_t cell = t.z_cell + (in ? (int64_t)y * t.W + x : 0);
                    const char* src = Z + (cell * cell_bytes + q * PB + k * CH);
                    char* dst = win + rr * pitch + cc * PB + k * CH;
                    if constexpr (CH == 16)
                        *reinterpret_cast<u32x4*>(dst) = in ? *reinterpret_cast<const u32x4*>(src) : u32x4{0u, 0u, 0u, 0u};
                    else
                        *reinterpret_cast<u32x2*>(dst) = in ? *reinterpret_cast<const u32x2*>(src) : u32x2{0u, 0u};
                }
            }
        }
        if constexpr (DMA) {
            // chunk gs has landed once at most the UPW loads of each later
            // chunk already issued (gs + 1 .. gs + NB - 2) are outstanding;
            // vmcnt(N) keeps expcnt and lgkmcnt at their maxima
            const int later = min(NB - 2, nsteps - 1 - gs);
            if (NB >= 4 && later >= 2) __builtin_amdgcn_s_waitcnt(0xF70 | (2 * UPW * LPU));
            else if (later >= 1) __builtin_amdgcn_s_waitcnt(0xF70 | (UPW * LPU));
            else __builtin_amdgcn_s_waitcnt(0xF70);
        }
        __syncthreads();                           // window and chunk `step` visible

        // issue the loads of a later chunk before this step's MFMAs (without
        // DMA: the next chunk through registers; the last step reloads its own
        // chunk and does not store it)
        u32x4 pf[PFMAX];
        const bool more = gs + 1 < nsteps;
        int nstep = step + 1, nfbi = fbi;
        if (nstep == total) {
            nstep = 0;
            ++nfbi;
        }
        if constexpr (DMA) {
            if (gs + NB - 1 < nsteps) {
                int st2 = step + NB - 1, f2 = fbi;
                while (st2 >= total) {
                    st2 -= total;
                    ++f2;
                }
                // into the buffer step gs - 1 used, free since the barrier above
                dma_chunk(f2 * BB * total + st2, gbuf(bi == 0 ? NB - 1 : bi - 1));
            }
        } else {
            const int cur = fbi * BB * total + step;   // chunk index within the tile's blocks
            const int nxt = more ? nfbi * BB * total + nstep : cur;
#pragma unroll
            for (int k = 0; k < PFMAX; ++k) pf[k] = chunk_ld(nxt, k);
        }

        const u32x4* gb = DMA ? gbuf(bi) : ((gs & 1) ? gbuf1 : gbuf0);
        const char* abase = win + ((wv / WX) * TY) * pitch + (32 * (wv % WX) + p) * PB + KS * s + FB * j;
        const char* gbb = reinterpret_cast<const char*>(gb) + lane * FB;
        if constexpr (HS > 0) {
            // window row n + i feeds output row i at filter row n; the TY live
            // rows and the one being fetched sit in ring slots (row % (TY + 1))
            Frag Ar[TY + 1];
            Frag Br[2][BB];
#pragma unroll
            for (int i = 0; i < TY; ++i) Ar[i] = lds_frag<KIND>(abase + i * pitch, PB);
#pragma unroll
            for (int b = 0; b < BB; ++b) Br[0][b] = *reinterpret_cast<const Frag*>(gbb + (b * HS) * chunk_bytes);
#pragma unroll
            for (int n = 0; n < HS; ++n) {
                if (n + 1 < HS) {
#pragma unroll
                    for (int b = 0; b < BB; ++b)
                        Br[(n + 1) & 1][b] = *reinterpret_cast<const Frag*>(gbb + (b * HS + n + 1) * chunk_bytes);
                    Ar[(n + TY) % (TY + 1)] = lds_frag<KIND>(abase + (n + TY) * pitch, PB);
                }
                if (xlive) {
#pragma unroll
                    for (int i = 0; i < TY; ++i)
#pragma unroll
                        for (int b = 0; b < BB; ++b)
                            acc[i][b] = mfma_step<KIND>(Ar[(n + i) % (TY + 1)], Br[n & 1][b], acc[i][b]);
                }
                // keep the source order: the next row's LDS reads are issued
                // ahead of this row's MFMAs and their latency hides behind them
                __builtin_amdgcn_sched_barrier(0);
            }
        } else {
            Frag A[TY];
#pragma unroll
            for (int i = 0; i < TY; ++i) A[i] = lds_frag<KIND>(abase + i * pitch, PB);
            Frag B[BB];
#pragma unroll
            for (int b = 0; b < BB; ++b) B[b] = *reinterpret_cast<const Frag*>(gbb + (b * h) * chunk_bytes);
            for (int n = 0; n < h; ++n) {
                Frag Bn[BB], An;
                const bool nx = n + 1 < h;
                if (nx) {
#pragma unroll
                    for (int b = 0; b < BB; ++b)
                        Bn[b] = *reinterpret_cast<const Frag*>(gbb + (b * h + n + 1) * chunk_bytes);
                    An = lds_frag<KIND>(abase + (n + TY) * pitch, PB);
                }
                if (xlive) {
#pragma unroll
                    for (int i = 0; i < TY; ++i)
#pragma unroll
                        for (int b = 0; b < BB; ++b) acc[i][b] = mfma_step<KIND>(A[i], B[b], acc[i][b]);
                }
                if (nx) {
#pragma unroll
                    for (int i = 0; i + 1 < TY; ++i) A[i] = A[i + 1];
                    A[TY - 1] = An;
#pragma unroll
                    for (int b = 0; b < BB; ++b) B[b] = Bn[b];
                }
            }
        }

        if (!DMA && more) {
            u32x4* nb = (gs & 1) ? gbuf0 : gbuf1;
#pragma unroll
            for (int k = 0; k < PFMAX; ++k) nb[pf_dst[k]] = pf[k];
        }
        if (step == total - 1) {
            corr_epilogue<KIND, TY, BB, WY, WX>(t, g, t.fb0 + fbi * BB, acc, tk, out, rmax, rmin);
#pragma unroll
            for (int i = 0; i < TY; ++i)
#pragma unroll
                for (int b = 0; b < BB; ++b)
#pragma unroll
                    for (int k = 0; k < 16; ++k) acc[i][b][k] = 0.f;
        }
        step = nstep;
        fbi = nfbi;
        bi = bi == NB - 1 ? 0 : bi + 1;
    }

}

// One workgroup per tile (grid = tiles), or a persistent grid that strides
// over the cost-sorted tile list; both produce the same bits.  HSO > 0: every
// tile's filters have HSO rows, and only that unrolled body is built (a
// kernel with one body needs far fewer registers than one that can take any
// height, so more wavefronts fit each SIMD).
template <CorrKind KIND, int PB, int TY, int BB, int WY, int WX, int HMAX, int HSO>
__global__ __launch_bounds__(64 * WY) __attribute__((amdgpu_waves_per_eu((HMAX <= 8 && KIND != CORR_FP8) ? 2 : 1))) void corr_kernel(const CorrTile* __restrict__ tiles, int n_tiles,
                                                       const GroupDesc* __restrict__ groups,
                                                       const char* __restrict__ Z,
                                                       const char* __restrict__ G,
                                                       const float* __restrict__ tk,
                                                       float* __restrict__ out,
                                                       int* __restrict__ rmax,
                                                       int* __restrict__ rmin, int cell_bytes,
                                                       int Q, int win_bytes) {
    for (int i = blockIdx.x; i < n_tiles; i += gridDim.x) {
        const CorrTile t = tiles[i];
        if constexpr (HSO > 0) {
            corr_tile<KIND, PB, TY, BB, WY, WX, HMAX, HSO>(t, groups, Z, G, tk, out, rmax, rmin, cell_bytes, Q, win_bytes);
        } else {
            const int h = groups[t.group].h;
            // the DPM filter heights get unrolled bodies where that costs no
            // occupancy (FP8 fragments and 64-filter tiles of 32-byte planes
            // would need too many registers)
            constexpr bool UNROLL = corr_unrolls(KIND, PB, BB, HMAX);
            if (UNROLL && h == 6)
                corr_tile<KIND, PB, TY, BB, WY, WX, HMAX, 6>(t, groups, Z, G, tk, out, rmax, rmin, cell_bytes, Q, win_bytes);
            else if (UNROLL && h == 7)
                corr_tile<KIND, PB, TY, BB, WY, WX, HMAX, 7>(t, groups, Z, G, tk, out, rmax, rmin, cell_bytes, Q, win_bytes);
            else if (UNROLL && h == 8)
                corr_tile<KIND, PB, TY, BB, WY, WX, HMAX, 8>(t, groups, Z, G, tk, out, rmax, rmin, cell_bytes, Q, win_bytes);
            else
                corr_tile<KIND, PB, TY, BB, WY, WX, HMAX, 0>(t, groups, Z, G, tk, out, rmax, rmin, cell_bytes, Q, win_bytes);
        }
        if (i + (int)gridDim.x < n_tiles) __syncthreads();   // LDS reused by the next tile
    }
}

static int frag_bytes(CorrKind k) { return k == CORR_FP8 ? 32 : 16; }

// LDS of a correlation launch whose groups have at most max_h filter rows and
// S K-steps: the window of max_h - 1 + ty * wy / wx rows of 32 * wx - 1 + S
// steps of cells, plus the filter staging of the tallest group height the
// kernel may see.  An unrolled group of h <= 8 rows stages CORR_NBUF chunks of
// h rows, a rolled one 2 chunks of h rows; with max_h > 8 the HMAX = 16
// kernel runs both kinds, so the staging takes the larger of 2 max_h and
// CORR_NBUF min(max_h, 8) rows.
size_t corr_lds_bytes(const CorrLaunch& cfg, int max_h, int S) {
    const int FB = frag_bytes(cfg.kind);
    const int WC = 32 * cfg.wx - 1 + (2 * FB * S) / cfg.pk.PB;
    const size_t win = (size_t)(cfg.ty * (cfg.wy / cfg.wx) + max_h - 1) * WC * cfg.pk.PB;
    const size_t winal = (win + 1023) & ~size_t(1023);   // whole 1 KB units (window DMA)
    const int hmax = max_h <= 8 ? 8 : CORR_MAX_H;         // the kernel instance launch_corr_t picks
    const bool unroll = corr_unrolls(cfg.kind, cfg.pk.PB, cfg.bb, hmax) && max_h >= 6;
    const int rows = std::max(2 * max_h, unroll ? corr_chunk_buffers(true, cfg.wx) * std::min(max_h, 8) : 0);
    return winal + (size_t)rows * cfg.bb * 64 * FB;
}

template <CorrKind KIND, int PB, int TY, int BB, int WY, int WX, int HMAX, int HSO>
static hipError_t launch_corr_k(const CorrLaunch& cfg, const CorrTile* tiles, int n_tiles,
                                const GroupDesc* groups, const void* Z, const void* G,
                                const float* tk, float* out, int* rkeys, int64_t n_slots,
                                int cell_bytes, int max_h, int max_S, hipStream_t st) {
    const size_t lds = corr_lds_bytes(cfg, max_h, max_S);
    const int FB = FragT<KIND>::bytes;
    const int WC = 32 * WX - 1 + (2 * FB * max_S) / PB;
    const size_t win = (size_t)(TY * (WY / WX) + max_h - 1) * WC * PB;
    const int win_bytes = (int)((win + 1023) & ~size_t(1023));
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    auto kern = corr_kernel<KIND, PB, TY, BB, WY, WX, HMAX, HSO>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    int grid = n_tiles;
    if (cfg.persistent) {
        int per_cu = 0, dev = 0, cus = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * WY, lds);
        if (e == hipSuccess) e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        grid = std::max(1, std::min(n_tiles, std::max(per_cu, 1) * cus));
    }
    hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * WY), lds, st, tiles, n_tiles, groups,
                       static_cast<const char*>(Z), static_cast<const char*>(G), tk, out,
                       rkeys, rkeys ? rkeys + n_slots : nullptr, cell_bytes, cfg.pk.Q, win_bytes);
    return hipGetLastError();
}

// Tiles whose filters all have 6, 7 or 8 rows go to a kernel built for that
// height alone when the kind unrolls it; others to the kernel that takes any
// height up to HMAX.
template <CorrKind KIND, int PB, int TY, int BB, int WY, int WX, int HMAX>
static hipError_t launch_corr_h(const CorrLaunch& cfg, const CorrTile* tiles, int n_tiles,
                                const GroupDesc* groups, const void* Z, const void* G,
                                const float* tk, float* out, int* rkeys, int64_t n_slots,
                                int cell_bytes, int max_h, int max_S, hipStream_t st) {
    if constexpr (HMAX == 8 && corr_unrolls(KIND, PB, BB, 8)) {
        if (cfg.hs == 6 && max_h == 6)
            return launch_corr_k<KIND, PB, TY, BB, WY, WX, HMAX, 6>(cfg, tiles, n_tiles, groups, Z, G, tk, out,
                                                                    rkeys, n_slots, cell_bytes, max_h, max_S, st);
        if (cfg.hs == 7 && max_h == 7)
            return launch_corr_k<KIND, PB, TY, BB, WY, WX, HMAX, 7>(cfg, tiles, n_tiles, groups, Z, G, tk, out,
                                                                    rkeys, n_slots, cell_bytes, max_h, max_S, st);
        if (cfg.hs == 8 && max_h == 8)
            return launch_corr_k<KIND, PB, TY, BB, WY, WX, HMAX, 8>(cfg, tiles, n_tiles, groups, Z, G, tk, out,
                                                                    rkeys, n_slots, cell_bytes, max_h, max_S, st);
    }
    return launch_corr_k<KIND, PB, TY, BB, WY, WX, HMAX, 0>(cfg, tiles, n_tiles, groups, Z, G, tk, out, rkeys,
                                                            n_slots, cell_bytes, max_h, max_S, st);
}

// Filters of at most 8 rows (every DPM root and part shape) get a kernel whose
// chunk prefetch needs half the registers; taller filters only the default tile.
template <CorrKind KIND, int PB, int TY, int BB, int WY, int WX>
static hipError_t launch_corr_t(const CorrLaunch& cfg, const CorrTile* tiles, int n_tiles,
                                const GroupDesc* groups, const void* Z, const void* G,
                                const float* tk, float* out, int* rkeys, int64_t n_slots,
                                int cell_bytes, int max_h, int max_S, hipStream_t st) {
    if (max_h <= 8)
        return launch_corr_h<KIND, PB, TY, BB, WY, WX, 8>(cfg, tiles, n_tiles, groups, Z, G, tk, out,
                                                          rkeys, n_slots, cell_bytes, max_h, max_S, st);
    if constexpr (TY == 4 && BB == 2 && WY == 4 && WX == 1)
        return launch_corr_h<KIND, PB, TY, BB, WY, WX, CORR_MAX_H>(cfg, tiles, n_tiles, groups, Z, G, tk,
                                                                   out, rkeys, n_slots, cell_bytes,
                                                                   max_h, max_S, st);
    return hipErrorInvalidValue;
}

template <CorrKind KIND, int PB>
static hipError_t launch_corr_p(const CorrLaunch& cfg, const CorrTile* tiles, int n_tiles,
                                const GroupDesc* groups, const void* Z, const void* G,
                                const float* tk, float* out, int* rkeys, int64_t n_slots,
                                int cell_bytes, int max_h, int max_S, hipStream_t st) {
#define DPMT_SHAPE(A, B, C, D)                                                                       \
    if (cfg.ty == A && cfg.bb == B && cfg.wy == C && cfg.wx == D)                                    \
        return launch_corr_t<KIND, PB, A, B, C, D>(cfg, tiles, n_tiles, groups, Z, G, tk, out, rkeys, \
                                                   n_slots, cell_bytes, max_h, max_S, st);
    DPMT_SHAPE(4, 2, 4, 1)
    DPMT_SHAPE(2, 2, 4, 1)
    DPMT_SHAPE(4, 1, 4, 1)
    DPMT_SHAPE(4, 1, 4, 4)
    DPMT_SHAPE(4, 1, 8, 8)
    DPMT_SHAPE(4, 1, 8, 4)
#undef DPMT_SHAPE
    return hipErrorInvalidValue;
}

bool corr_shape_supported(int ty, int bb, int wy, int wx, int max_h) {
    const bool listed = (ty == 4 && bb == 2 && wy == 4 && wx == 1) || (ty == 2 && bb == 2 && wy == 4 && wx == 1) ||
                        (ty == 4 && bb == 1 && wy == 4 && wx == 1) || (ty == 4 && bb == 1 && wy == 4 && wx == 4) ||
                        (ty == 4 && bb == 1 && wy == 8 && wx == 8) || (ty == 4 && bb == 1 && wy == 8 && wx == 4);
    if (!listed || max_h > CORR_MAX_H) return false;
    return max_h <= 8 || (ty == 4 && bb == 2 && wy == 4 && wx == 1);
}

hipError_t launch_corr(const CorrLaunch& cfg, const CorrTile* tiles, int n_tiles,
                       const GroupDesc* groups, const void* Z, const void* G, const float* tk,
                       float* out, int* rkeys, int64_t n_slots, int max_h, int max_S,
                       hipStream_t st) {
    if (n_tiles <= 0) return hipSuccess;
    if (!corr_shape_supported(cfg.ty, cfg.bb, cfg.wy, cfg.wx, max_h)) return hipErrorInvalidValue;
    const int cb = cfg.pk.RP * cfg.pk.esz;
#define DPMT_CORR(K, P) \
    case P: return launch_corr_p<K, P>(cfg, tiles, n_tiles, groups, Z, G, tk, out, rkeys, n_slots, cb, max_h, max_S, st);
    if (cfg.kind == CORR_F32) {
        switch (cfg.pk.PB) { DPMT_CORR(CORR_F32, 16) DPMT_CORR(CORR_F32, 32) default: break; }
    } else if (cfg.kind == CORR_BF16) {
        switch (cfg.pk.PB) { DPMT_CORR(CORR_BF16, 8) DPMT_CORR(CORR_BF16, 16) DPMT_CORR(CORR_BF16, 32) default: break; }
    } else if (cfg.kind == CORR_FP8) {
        switch (cfg.pk.PB) { DPMT_CORR(CORR_FP8, 16) DPMT_CORR(CORR_FP8, 32) default: break; }
    }
#undef DPMT_CORR
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// CP correlation (Section 4).  For every rank term r of filter k:
//   P_r = X x_3 c_r     channel contraction, MFMA 16x16x4 FP32: halo cells x
//                       16 columns (4 filters x 4 terms) x 32 channels
//   Q_r = P_r o_x b_r   1-D correlation along x (VALU, P from LDS)
//   S_k += Q_r o_y a_r  1-D correlation along y (VALU, registers)
// A tile loads its halo (HY x HX cells, 32 channels) into registers once and
// walks its chunks of 4 filters.  The 16 P planes of a batch live in LDS from
// the contraction to the end of the 1-D passes.  In the 1-D passes wave v owns
// filter v of the chunk; lane (cq = lane % 8, rg = lane / 8) owns output cols
// 4cq .. 4cq+3 of tile rows rg*RG .. rg*RG+RG-1, RG = ceil(TYo / 8) <= 4.
// ---------------------------------------------------------------------------
typedef float v4f __attribute__((ext_vector_type(4)));
constexpr int CP_RBW = CP_HALO / 16 / 4;   // 16-cell row blocks per wave

size_t cp_lds_bytes(int HX, int HY) {
    // 16 planes, plus the rows past the halo that lanes beyond the tile's last
    // output row read (their values are never stored) and the x-window overrun
    return ((size_t)16 * HX * HY + 8 * (size_t)HX + 8) * 4;
}

// One CP tile.  HS, WS > 0: a filter shape known at compile time (halo
// geometry, loop trip counts and the filter's row and column factors in
// registers, both 1-D passes fully unrolled); HS = WS = 0: any shape, with
// rolled loops and factors read as they are used.
template <int HS, int WS>
__device__ __forceinline__ void cp_tile(const CpTile& t, const CpChunk* __restrict__ chunks,
                                        const float* __restrict__ X, const float* __restrict__ fac,
                                        float* __restrict__ out, int* __restrict__ rmax,
                                        int* __restrict__ rmin, uint8_t* __restrict__ flags,
                                        float* __restrict__ lds) {
    constexpr bool FIXED = HS > 0 && WS > 0;
    constexpr int HXc = FIXED ? ((CP_TX + WS - 1 + 3) & ~3) : 4;
    constexpr int HYc = FIXED ? CP_HALO / HXc : 1;
    constexpr int RGc = FIXED ? (HYc - HS + 1 + 7) / 8 : 4;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int h = FIXED ? HS : t.h, w = FIXED ? WS : t.w;
    const int HX = FIXED ? HXc : t.HX, HY = FIXED ? HYc : t.HY;
    const int NPX = HX * HY;
    const float inv_hx = 1.f / (float)HX;
    // halo cell of row block b = wv + 4i: 16b + lane % 16, channels
    // 8 (lane / 16) .. +7 (the K index of step s is channel 8 (lane / 16) + s)
    float xr[CP_RBW][8];
#pragma unroll
    for (int i = 0; i < CP_RBW; ++i) {
        const int px = (wv + 4 * i) * 16 + (lane & 15);
        const int row = (int)(((float)px + 0.5f) * inv_hx);   // exact: px < 2^11, HX <= 64
        const int col = px - row * HX;
        const int gy = t.y0 + row, gx = t.x0 + col;
        const bool ok = px < NPX && gy < t.H && gx < t.W;
        const int cy = min(gy, t.H - 1), cx = min(gx, t.W - 1);
        const float4* src = reinterpret_cast<const float4*>(X + (t.x_cell + (int64_t)cy * t.W + cx) * 32 +
                                                            8 * (lane >> 4));
        const float4 v0 = src[0], v1 = src[1];
        xr[i][0] = ok ? v0.x : 0.f;
        xr[i][1] = ok ? v0.y : 0.f;
        xr[i][2] = ok ? v0.z : 0.f;
        xr[i][3] = ok ? v0.w : 0.f;
        xr[i][4] = ok ? v1.x : 0.f;
        xr[i][5] = ok ? v1.y : 0.f;
        xr[i][6] = ok ? v1.z : 0.f;
        xr[i][7] = ok ? v1.w : 0.f;
    }
    const int TYo = HY - h + 1;
    const int RG = FIXED ? RGc : (TYo + 7) >> 3;
    const int cq = lane & 7, ry = (lane >> 3) * RG;
    for (int ci = 0; ci < t.nchunk; ++ci) {
        const CpChunk& ch = chunks[t.chunk0 + ci];
        const int R = ch.R[wv];
        const float* fa = fac + ch.ab_off[wv];          // a_r[n] at r*h + n
        const float* fb = fa + R * h;                   // b_r[m] at r*w + m
        const float* ft = fb + R * w;                   // thresholds t_r (with flags)
        uint32_t below = 0;                             // bit 4j+c: a partial sum fell below its t_r
        float acc[4][4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[j][c] = 0.f;
        for (int q = 0; q < ch.nq; ++q) {
            {   // contraction: P planes of the batch's 16 columns at every halo cell
                const float4* bs = reinterpret_cast<const float4*>(fac + ch.c_off + ((int64_t)q * 64 + lane) * 8);
                const float4 b0 = bs[0], b1 = bs[1];
                const float bv[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
#pragma unroll
                for (int i = 0; i < CP_RBW; ++i) {
                    v4f d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int s = 0; s < 8; ++s) d = __builtin_amdgcn_mfma_f32_16x16x4f32(xr[i][s], bv[s], d, 0, 0, 0);
                    // D[cell 16b + 4 (lane / 16) + v][column lane % 16]
                    const int px = (wv + 4 * i) * 16 + 4 * (lane >> 4);
                    if (px < NPX)
                        *reinterpret_cast<float4*>(lds + (lane & 15) * NPX + px) = make_float4(d[0], d[1], d[2], d[3]);
                }
            }
            __syncthreads();
            for (int rr = 0; rr < 4; ++rr) {            // 1-D passes of this wave's filter
                const int r = 4 * q + rr;
                if (r >= R) break;
                const float* P = lds + (4 * wv + rr) * NPX + ry * HX + 4 * cq;
                const float* ar = fa + r * h;
                const float* br = fb + r * w;
                if constexpr (FIXED) {
                    constexpr int NW = (WS + 3 + 3) / 4;    // 16-byte reads covering x .. x+3+WS-1
                    float ac[HS], bc[WS];
#pragma unroll
                    for (int n = 0; n < HS; ++n) ac[n] = ar[n];
#pragma unroll
                    for (int m = 0; m < WS; ++m) bc[m] = br[m];
#pragma unroll
                    for (int hr = 0; hr < RGc + HS - 1; ++hr) {
                        float win[4 * NW];
#pragma unroll
                        for (int u = 0; u < NW; ++u) {
                            const float4 v = *reinterpret_cast<const float4*>(P + hr * HXc + 4 * u);
                            win[4 * u] = v.x;
                            win[4 * u + 1] = v.y;
                            win[4 * u + 2] = v.z;
                            win[4 * u + 3] = v.w;
                        }
                        float qv[4];
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            qv[c] = 0.f;
#pragma unroll
                            for (int m = 0; m < WS; ++m) qv[c] = fmaf(bc[m], win[c + m], qv[c]);
                        }
#pragma unroll
                        for (int j = 0; j < RGc; ++j) {
                            const int n = hr - j;
                            if (n >= 0 && n < HS) {
#pragma unroll
                                for (int c = 0; c < 4; ++c) acc[j][c] = fmaf(ac[n], qv[c], acc[j][c]);
                            }
                        }
                    }
                } else {
                    for (int hr = 0; hr < RG + h - 1; ++hr) {
                        const float* prow = P + hr * HX;
                        float qv[4] = {0.f, 0.f, 0.f, 0.f};
                        float4 lo = *reinterpret_cast<const float4*>(prow);
                        for (int m0 = 0; m0 < w; m0 += 4) {
                            const float4 hi = *reinterpret_cast<const float4*>(prow + m0 + 4);
                            const float win[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                if (m0 + e < w) {
                                    const float bm = br[m0 + e];
#pragma unroll
                                    for (int c = 0; c < 4; ++c) qv[c] = fmaf(bm, win[e + c], qv[c]);
                                }
                            }
                            lo = hi;
                        }
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const int n = hr - j;
                            if (j < RG && n >= 0 && n < h) {
                                const float an = ar[n];
#pragma unroll
                                for (int c = 0; c < 4; ++c) acc[j][c] = fmaf(an, qv[c], acc[j][c]);
                            }
                        }
                    }
                }
                if (flags != nullptr) {                 // Algorithm 1: partial sum after term r
                    const float tr = ft[r];
#pragma unroll
                    for (int j = 0; j < 4; ++j)
#pragma unroll
                        for (int c = 0; c < 4; ++c)
                            if (acc[j][c] < tr) below |= 1u << (4 * j + c);
                }
            }
            __syncthreads();
        }
        if (R > 0) {                                    // filter column col0 + 4 ci + wv
            const int f = t.col0 + 4 * ci + wv;
            const int x = t.x0 + 4 * cq;
            float vmax = -INFINITY, vmin = INFINITY;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int yr = ry + j, y = t.y0 + yr;
                if (j >= RG || yr >= TYo || y >= t.Ho || x >= t.Wo) continue;
                const int64_t o = t.out_off + ((int64_t)f * t.Ho + y) * t.ld + x;
                *reinterpret_cast<float4*>(out + o) = make_float4(acc[j][0], acc[j][1], acc[j][2], acc[j][3]);
                if (flags != nullptr)
                    *reinterpret_cast<uint32_t*>(flags + o) = ((below >> (4 * j)) & 1u) |
                                                               (((below >> (4 * j + 1)) & 1u) << 8) |
                                                               (((below >> (4 * j + 2)) & 1u) << 16) |
                                                               (((below >> (4 * j + 3)) & 1u) << 24);
                if (x + 3 < t.Wo) {                  // whole run inside the map: 3-input max / min
                    vmax = fmaxf(fmaxf(vmax, acc[j][0]), fmaxf(acc[j][1], fmaxf(acc[j][2], acc[j][3])));
                    vmin = fminf(fminf(vmin, acc[j][0]), fminf(acc[j][1], fminf(acc[j][2], acc[j][3])));
                } else {
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        if (x + c < t.Wo) {
                            vmax = fmaxf(vmax, acc[j][c]);
                            vmin = fminf(vmin, acc[j][c]);
                        }
                }
            }
            if (rmax != nullptr && t.rng >= 0) {
#pragma unroll
                for (int o = 32; o >= 1; o >>= 1) {
                    vmax = fmaxf(vmax, __shfl_xor(vmax, o, 64));
                    vmin = fminf(vmin, __shfl_xor(vmin, o, 64));
                }
                if (lane == 0 && vmax >= vmin) {
                    atomicMax(rmax + t.rng + f, range_key(vmax));
                    atomicMin(rmin + t.rng + f, range_key(vmin));
                }
            }
        }
    }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void cp_corr_kernel(
    const CpTile* __restrict__ tiles, const CpChunk* __restrict__ chunks, const float* __restrict__ X,
    const float* __restrict__ fac, float* __restrict__ out, int* __restrict__ rmax,
    int* __restrict__ rmin, uint8_t* __restrict__ flags) {
    extern __shared__ __align__(16) float cp_lds[];
    const CpTile& t = tiles[blockIdx.x];
    // compiled shapes: the DPM part filter and the usual root filters
    if (t.h == 6 && t.w == 6) cp_tile<6, 6>(t, chunks, X, fac, out, rmax, rmin, flags, cp_lds);
    else if (t.h == 6 && t.w == 11) cp_tile<6, 11>(t, chunks, X, fac, out, rmax, rmin, flags, cp_lds);
    else if (t.h == 7 && t.w == 13) cp_tile<7, 13>(t, chunks, X, fac, out, rmax, rmin, flags, cp_lds);
    else if (t.h == 8 && t.w == 15) cp_tile<8, 15>(t, chunks, X, fac, out, rmax, rmin, flags, cp_lds);
    else cp_tile<0, 0>(t, chunks, X, fac, out, rmax, rmin, flags, cp_lds);
}

hipError_t launch_cp_corr(const CpTile* tiles, int n_tiles, const CpChunk* chunks, const float* X,
                          const float* fac, float* out, int* rkeys, int64_t n_slots, uint8_t* flags,
                          size_t lds_bytes, hipStream_t st) {
    if (n_tiles <= 0) return hipSuccess;
    if (lds_bytes > 160 * 1024) return hipErrorInvalidValue;
    if (lds_bytes > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(cp_corr_kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(cp_corr_kernel, dim3(n_tiles), dim3(256), lds_bytes, st, tiles, chunks, X, fac, out,
                       rkeys, rkeys ? rkeys + n_slots : nullptr, flags);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP8 (OCP e4m3) operands with per-channel scales
//
// The contraction runs over projected channels r, so a scale per channel
// cannot be applied after the sum; it is folded into the filter factors
// instead.  Per call:
//   xmax_l = max over cells |X[c][l]|                       (fp8_chanmax_*)
//   s_r    = sum_l |U[l][r]| * xmax_l / 448 >= max_c |Z[c][r]| / 448, so
//            Zq = e4m3(Z / s_r) never overflows             (fp8_scales)
//   t_k    = max |G_k * s| / 448 per filter k, as max_r s_r M_kr / 448 with
//            M_kr = max |G_k| over the elements of channel r (kept from the
//            upload: rounding is monotonic, so this is the same value),
//   Gq_k   = e4m3(G_k * s / t_k)                            (fp8_requant)
//   resp_k = t_k * sum Gq_k Zq                               (corr epilogue)
// Conversions round to nearest even after an explicit clamp to +-448 (the
// hardware conversion does not saturate).
// ---------------------------------------------------------------------------
constexpr float FP8_MAX = 448.f;
constexpr int CHANMAX_BLOCKS = 256;
static_assert(CHANMAX_BLOCKS * 32 <= FP8_PARTIALS, "channel-max partials must fit their scratch");

__device__ __forceinline__ uint32_t fp8x4(float a, float b, float c, float d) {
    a = fminf(fmaxf(a, -FP8_MAX), FP8_MAX);
    b = fminf(fmaxf(b, -FP8_MAX), FP8_MAX);
    c = fminf(fmaxf(c, -FP8_MAX), FP8_MAX);
    d = fminf(fmaxf(d, -FP8_MAX), FP8_MAX);
    int w = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
    w = __builtin_amdgcn_cvt_pk_fp8_f32(c, d, w, true);
    return (uint32_t)w;
}

// partial[b][l] = max |X[c][l]| over the cells of block b's stride: thread
// (cell row cr, channel quad l4) reads 16-byte runs, four cells in flight
__global__ __launch_bounds__(256) void fp8_chanmax_kernel(const float* __restrict__ X, int64_t n_cells,
                                                          float* __restrict__ partial, int* __restrict__ rkeys,
                                                          int64_t n_slots) {
    __shared__ float4 sm[32][8];
    if (rkeys != nullptr)                          // the value-range reset, folded in
        for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n_slots; i += (int64_t)gridDim.x * 256) {
            rkeys[i] = INT_MIN;
            rkeys[n_slots + i] = INT_MAX;
        }
    const int l4 = threadIdx.x & 7, cr = threadIdx.x >> 3;
    const int64_t stride = (int64_t)gridDim.x * 32;
    float4 m = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int64_t c0 = (int64_t)blockIdx.x * 32 + cr; c0 < n_cells; c0 += 4 * stride) {
        float4 v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t c = c0 + k * stride;
            v[k] = c < n_cells ? reinterpret_cast<const float4*>(X + c * 32)[l4] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            m.x = fmaxf(m.x, fabsf(v[k].x));
            m.y = fmaxf(m.y, fabsf(v[k].y));
            m.z = fmaxf(m.z, fabsf(v[k].z));
            m.w = fmaxf(m.w, fabsf(v[k].w));
        }
    }
    sm[cr][l4] = m;
    __syncthreads();
    if (threadIdx.x < 32) {
        const int l = threadIdx.x, q = l >> 2, e = l & 3;
        float v = 0.f;
        for (int i = 0; i < 32; ++i) {
            const float4 t = sm[i][q];
            v = fmaxf(v, e == 0 ? t.x : e == 1 ? t.y : e == 2 ? t.z : t.w);
        }
        partial[blockIdx.x * 32 + l] = v;
    }
}

// s[r] = sum_l |U[l][r]| xmax_l / 448 (1 for an all-zero channel), one block
__global__ __launch_bounds__(256) void fp8_scales_kernel(const float* __restrict__ partial, int nb,
                                                         const float* __restrict__ U, int RP,
                                                         float* __restrict__ s) {
    __shared__ float xm[32];
    __shared__ float red[8][32];
    const int l = threadIdx.x & 31, r = threadIdx.x >> 5;
    float m = 0.f;
#pragma unroll 8
    for (int b = r; b < nb; b += 8) m = fmaxf(m, partial[b * 32 + l]);
    red[r][l] = m;
    __syncthreads();
    if (threadIdx.x < 32) {
        float v = red[0][l];
        for (int i = 1; i < 8; ++i) v = fmaxf(v, red[i][l]);
        xm[l] = v;
    }
    __syncthreads();
    for (int c = threadIdx.x; c < RP; c += 256) {
        float acc = 0.f;
        for (int k = 0; k < 32; ++k) acc = fmaf(fabsf(U[k * RP + c]), xm[k], acc);
        s[c] = acc > 0.f ? acc / FP8_MAX : 1.f;
    }
}

// Zq[c][r] = e4m3(Z[c][r] / s_r)
template <int RP>
__global__ __launch_bounds__(256) void project_fp8_kernel(const float* __restrict__ X, int64_t n_cells,
                                                          const float* __restrict__ U,
                                                          const float* __restrict__ s,
                                                          uint32_t* __restrict__ Zq) {
    __shared__ float sU[32 * RP];
    __shared__ float sinv[RP];
    for (int i = threadIdx.x; i < 32 * RP; i += 256) sU[i] = U[i];
    for (int i = threadIdx.x; i < RP; i += 256) sinv[i] = 1.f / s[i];
    __syncthreads();
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= n_cells) return;
    const float4* x4 = reinterpret_cast<const float4*>(X + c * 32);
    float acc[RP];
#pragma unroll
    for (int r = 0; r < RP; ++r) acc[r] = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const float4 v = x4[k];
#pragma unroll
        for (int r = 0; r < RP; ++r) {
            acc[r] = fmaf(v.x, sU[(4 * k + 0) * RP + r], acc[r]);
            acc[r] = fmaf(v.y, sU[(4 * k + 1) * RP + r], acc[r]);
            acc[r] = fmaf(v.z, sU[(4 * k + 2) * RP + r], acc[r]);
            acc[r] = fmaf(v.w, sU[(4 * k + 3) * RP + r], acc[r]);
        }
    }
    uint32_t* z = Zq + c * (RP / 4);
#pragma unroll
    for (int r = 0; r < RP; r += 4)
        z[r / 4] = fp8x4(acc[r] * sinv[r], acc[r + 1] * sinv[r + 1], acc[r + 2] * sinv[r + 2],
                         acc[r + 3] * sinv[r + 3]);
}

// `split` workgroups per 32-filter block of a group, each quantising a slice
// of its units.  The FP32 master factors are laid out exactly like the FP8
// operand (fragment order, 4 bytes per element); chmax holds M_kr for every
// filter slot (nch = Q * PB channels).
__global__ __launch_bounds__(256) void fp8_requant_kernel(const RequantBlock* __restrict__ blocks,
                                                          const float* __restrict__ master,
                                                          const float* __restrict__ s, int PB,
                                                          const float* __restrict__ chmax, int nch, int split,
                                                          uint8_t* __restrict__ G,
                                                          float* __restrict__ tk) {
    __shared__ float tsh[32];
    __shared__ float ss[64];                       // the channel scales (nch <= 64)
    const int rb = blockIdx.x / split, part = blockIdx.x - rb * split;
    const RequantBlock B = blocks[rb];
    if (threadIdx.x < 64) ss[threadIdx.x] = s[min((int)threadIdx.x, nch - 1)];
    __syncthreads();
    if (threadIdx.x < 32) {                        // t_k of the block's filter column threadIdx.x
        const float* mk = chmax + (int64_t)(B.t_off + threadIdx.x) * nch;
        float t = 0.f;
        for (int r = 0; r < nch; ++r) t = fmaxf(t, mk[r] * ss[r]);
        tsh[threadIdx.x] = t;
        if (part == 0 && B.f0 + (int)threadIdx.x < B.ng) tk[B.t_off + threadIdx.x] = t > 0.f ? t / FP8_MAX : 1.f;
    }
    __syncthreads();
    // unit = (chunk, lane): 32 consecutive elements of one filter's flattened
    // row; element e of the unit is plane byte o0 + e of plane q, channel
    // (o0 + e) % PB, stepped with a wrap instead of a division per element
    const int units = B.chunks * 64;
    const int per = (units + split - 1) / split;
    const int u1 = min(units, (part + 1) * per);
    for (int u = part * per + threadIdx.x; u < u1; u += 256) {
        const int lane = u & 63, ch = u >> 6;
        const int sidx = (ch / B.h) % B.S;         // K-step of this chunk
        const int q = (ch / B.h) / B.S;            // plane
        const float t = tsh[lane & 31];
        const float inv = t > 0.f ? FP8_MAX / t : 0.f;
        const float4* src = reinterpret_cast<const float4*>(master + B.m_off + (int64_t)u * 32);
        uint32_t* dst = reinterpret_cast<uint32_t*>(G + B.g_off + (int64_t)u * 32);
        int o = (64 * sidx + 32 * (lane >> 5)) % PB;
        const float* sq = ss + q * PB;
#pragma unroll
        for (int e4 = 0; e4 < 8; ++e4) {
            const float4 v = src[e4];
            const float a[4] = {v.x, v.y, v.z, v.w};
            float w[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                w[i] = a[i] * sq[o] * inv;
                o = o + 1 == PB ? 0 : o + 1;
            }
            dst[e4] = fp8x4(w[0], w[1], w[2], w[3]);
        }
    }
}

hipError_t launch_fp8_prepare(const float* X, int64_t n_cells, const float* U, int RP,
                              float* partial, float* scales, const RequantBlock* blocks,
                              int n_blocks, const float* master, const float* chmax, uint8_t* G,
                              float* tk, int* rkeys, int64_t n_slots, hipStream_t st) {
    if (RP > 32) return hipErrorInvalidValue;      // FP8 packs one plane of RP <= 32 channels
    hipLaunchKernelGGL(fp8_chanmax_kernel, dim3(CHANMAX_BLOCKS), dim3(256), 0, st, X, n_cells, partial,
                       rkeys, n_slots);
    hipLaunchKernelGGL(fp8_scales_kernel, dim3(1), dim3(256), 0, st, partial, CHANMAX_BLOCKS, U, RP, scales);
    constexpr int SPLIT = 4;                       // workgroups per 32-filter block
    if (n_blocks > 0)
        hipLaunchKernelGGL(fp8_requant_kernel, dim3(n_blocks * SPLIT), dim3(256), 0, st, blocks, master,
                           scales, RP, chmax, RP, SPLIT, G, tk);
    return hipGetLastError();
}

hipError_t launch_project_fp8(const float* X, int64_t n_cells, const float* U, int RP,
                              const float* scales, void* Z, hipStream_t st) {
    if (n_cells <= 0) return hipSuccess;
    const unsigned nb = (unsigned)((n_cells + 255) / 256);
    uint32_t* Zq = static_cast<uint32_t*>(Z);
    if (RP == 16) hipLaunchKernelGGL(project_fp8_kernel<16>, dim3(nb), dim3(256), 0, st, X, n_cells, U, scales, Zq);
    else if (RP == 32) hipLaunchKernelGGL(project_fp8_kernel<32>, dim3(nb), dim3(256), 0, st, X, n_cells, U, scales, Zq);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// distance transform
//
// Along a line with values v[0..n) the targets are t_k = ts*k + anchor and the
// cost of candidate x for target t is c(u) = b*u + a*u^2, u = x - t, a > 0.
// Two facts keep the exact search short:
//  * window: x can only beat the target itself if c(x - t) <= v[x] - v[t] <=
//    M - v[t] (M the line maximum); solving the quadratic bounds x to
//    [t + lo, t + hi], and a 1-cell margin absorbs FP32 rounding;
//  * monotonicity: v[x] - c(x - t) has strictly increasing differences in
//    (x, t) (the cross term is 2a*x*t), so the maximiser of a later target is
//    never left of the maximiser of an earlier one; a lane that owns several
//    consecutive targets starts each scan at the previous target's argmax.
// Scanning that range in ascending order with a strict > gives the exact
// maximum and its smallest maximiser, i.e. the lexicographic tie rule.
//
// ---------------------------------------------------------------------------
// Per-line constants of one pair's cost c(u) = b*u + a*u^2 and the line maximum.
struct LineConst {
    float a, b, inv2a, bb4a;   // inv2a = 1/(2a); bb4a unused slot kept for alignment
    float M;                   // line maximum
};

// Window [t + lo, t + hi] (clamped to [from, n-1]) holding every possible
// maximiser of target t: x can only beat t itself if c(x - t) <= M - v[t].
// The hardware square root and reciprocal are within a few ulp; the 1-cell
// margin on each side covers that and the FP32 rounding of the bound.
__device__ __forceinline__ void dt_bounds(float vt, const LineConst& c, int t, int from, int n,
                                          int& lo, int& hi) {
    const float delta = fmaxf(c.M - vt, 0.f);
    const float s = __builtin_amdgcn_sqrtf(fmaf(4.f * c.a, delta, c.b * c.b));
    const float ulo = floorf((-c.b - s) * c.inv2a) - 1.f;
    const float uhi = ceilf((-c.b + s) * c.inv2a) + 1.f;
    lo = t + (int)fmaxf(ulo, -(float)n);
    hi = t + (int)fminf(uhi, (float)n);
    hi = min(hi, n - 1);
    lo = min(max(max(lo, 0), from), hi);
}

// Exact maximum of v[x] - c(x - t) for x in [lo, hi] and its smallest
// maximiser, four candidates per iteration so that their loads overlap.
template <class Load>
__device__ __forceinline__ float scan_range(const Load& load, int lo, int hi, int t, float a,
                                            float b, int& arg) {
    float best = -INFINITY;
    arg = lo;
    int x = lo;
    for (; x + 3 <= hi; x += 4) {
        const float v0 = load(x), v1 = load(x + 1), v2 = load(x + 2), v3 = load(x + 3);
        const float u = (float)(x - t);
        const float e0 = v0 - u * fmaf(a, u, b);
        const float e1 = v1 - (u + 1.f) * fmaf(a, u + 1.f, b);
        const float e2 = v2 - (u + 2.f) * fmaf(a, u + 2.f, b);
        const float e3 = v3 - (u + 3.f) * fmaf(a, u + 3.f, b);
        if (e0 > best) { best = e0; arg = x; }
        if (e1 > best) { best = e1; arg = x + 1; }
        if (e2 > best) { best = e2; arg = x + 2; }
        if (e3 > best) { best = e3; arg = x + 3; }
    }
    for (; x <= hi; ++x) {
        const float u = (float)(x - t);
        const float e = load(x) - u * fmaf(a, u, b);
        if (e > best) { best = e; arg = x; }
    }
    return best;
}

// Generic form used by the single-map transform.
template <class Load>
__device__ __forceinline__ float window_max(const Load& load, int n, int t, int from, float a,
                                            float b, float M, int& arg) {
    LineConst c{a, b, 0.5f / a, 0.f, M};
    int lo, hi;
    dt_bounds(load(t), c, t, from, n, lo, hi);
    return scan_range(load, lo, hi, t, a, b, arg);
}

// Fixed window of a line: with D its value range (max - min), any candidate
// farther than [lo, hi] from its target costs more than D and so cannot beat
// the target itself; lo = floor((-b - s)/2a) - 1, hi = ceil((-b + s)/2a) + 1,
// s = sqrt(b^2 + 4aD).  The 1-cell margins cover FP32 rounding of the bound.
__device__ __forceinline__ void line_window(float a, float b, float range, int n, int& ulo,
                                           int& uhi) {
    const float s = sqrtf(fmaf(4.f * a, fmaxf(range, 0.f), b * b));
    const float inv = 0.5f / a;
    ulo = (int)fmaxf(floorf((-b - s) * inv) - 1.f, -(float)n);
    uhi = (int)fminf(ceilf((-b + s) * inv) + 1.f, (float)n);
}

// ---------------------------------------------------------------------------
// Placement: the distance transform evaluated at the part anchors of every
// root position, and the score assembly, in one kernel.
//
// Block = (score map, PLACE_CW consecutive root columns x0) of NT threads:
// 256, or 512 where LDS rather than registers limits the blocks per CU (tall
// maps), which gives such a CU twice the wavefronts.  For each part i
// of the map's component (anchor v, cost d) the block
//   1. row pass: for every part-map row y' it needs and every column of the
//      strip, R1[y'][x0] = max over x' of resp_i[y'][x'] - c_x(x' - t_x) with
//      t_x = 2 x0 + v_x, and the smallest maximiser; R1 stays in LDS;
//   2. column pass: for every root row y0, D = max over y' of R1[y'][x0] -
//      c_y(y' - t_y) with t_y = 2 y0 + v_y, the smallest maximiser, and the
//      (dy, dx) placement offset, written straight to the caller's layout;
//   3. adds D to the block's score accumulator.
// Finally score = root response + accumulator.
//
// Both passes use the window fact above with the value range of the part's
// whole response plane (the correlation records it per plane): with D_r the
// range, only |u| inside the roots of a u^2 + b u = D_r can beat the target
// itself.  Row-pass values exceed the plane maximum by at most b_x^2 / 4a_x,
// which widens the column window's range accordingly.  The window is thus
// uniform over the strip, so in every pass the wavefront walks the window
// offsets u in lockstep: the cost c(u) is one LDS broadcast shared by all
// lanes, and a lane's candidate is one conflict-free LDS read.  The staged
// response rows are split by parity of x' so that lanes whose targets are two
// apart read consecutive words.  Out-of-map candidates read -inf.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float quad_cost(float a, float b, int u) {
    const float fu = (float)u;
    return fu * fmaf(a, fu, b);
}

size_t place_lds_bytes(const PlaceLds& l) {
    return (size_t)4 * ((size_t)l.acc_rows * PLACE_CW + (size_t)l.r1_rows * PLACE_CW +
                        (size_t)l.stage_words + 2 * (size_t)l.ctab_words) +
           (size_t)2 * l.r1_rows * PLACE_CW + (size_t)l.acc_rows * PLACE_CW +
           (size_t)16 * l.max_parts;
}

// staged float4 per thread and round, for workgroups of NT threads
template <int NT>
constexpr int place_loads() { return PLACE_STAGE / (4 * NT); }

// Window of a line from its value range with the reciprocal 1/(2a) given;
// the hardware square root is within a few ulp, which the 1-cell margins of
// the bound absorb (as in line_window).
__device__ __forceinline__ void line_window_r(float a, float b, float inv2a, float range, int n,
                                              int& ulo, int& uhi) {
    const float s = __builtin_amdgcn_sqrtf(fmaf(4.f * a, fmaxf(range, 0.f), b * b));
    ulo = (int)fmaxf(floorf((-b - s) * inv2a) - 1.f, -(float)n);
    uhi = (int)fminf(ceilf((-b + s) * inv2a) + 1.f, (float)n);
}

// Geometry of one part inside a placement block; every thread computes the
// same values, without divisions.
struct PlaceGeo {
    int64_t plane;
    int ld, Hp, Wp, vy;
    float ax, bx, ay, by;
    int tx0;            // target column of lane 0
    int ulo, Wr, Wq;    // row window (clamped to the strip), length, rounded to 4
    int offA, offB;     // staging offsets of the scan's even and odd offsets (parity halves)
    int vlo, vhi, Wc;   // column window (clamped to the map +- 1 row) and its length
    int CH, SH;         // staged float4 per row, floats per parity half-row
    int SP;             // staged row pitch (>= 2 SH)
    int lrb, RB;        // rows per round RB = 2^lrb
    int ry0, ry1, rounds;
    int X0;             // first staged column (multiple of 4)
    int nq;             // float4 loads per thread and round
    int lrow, lcol, tpr;// this thread's staged row and first float4; threads per row
    int live;
};

// Windows of a part that do not depend on the strip: the row window
// [wx, wy] and the column window [wz, ww] (clamped to the map +- 1 row), from
// the value range of the part's plane.
__device__ __forceinline__ int4 part_windows(const MapPart& P, const int* __restrict__ rmax,
                                             const int* __restrict__ rmin) {
    const float hi = range_value(rmax[P.rng]), lo = range_value(rmin[P.rng]);
    const float range = hi >= lo ? hi - lo : 0.f;
    int ulo, uhi, vlo, vhi;
    line_window_r(P.d[1], P.d[0], P.inv2ax, range, P.Wp, ulo, uhi);
    line_window_r(P.d[3], P.d[2], P.inv2ay, range + P.bb4a, P.Hp, vlo, vhi);
    return make_int4(ulo, uhi, max(vlo, -(P.Hp + 1)), min(vhi, P.Hp + 1));
}

// win: the part's part_windows, read from LDS by every lane (made uniform
// here).  NT: threads of the workgroup (2^LNT).
template <int NT>
__device__ __forceinline__ PlaceGeo place_geo(const MapPart& P, const MapDesc& M, int xs, int4 win,
                                              int stage_words) {
    constexpr int CW = PLACE_CW;
    PlaceGeo G;
    G.plane = P.plane;
    G.ld = P.ld;
    G.Hp = P.Hp;
    G.Wp = P.Wp;
    G.vy = P.vy;
    G.ax = P.d[1];
    G.bx = P.d[0];
    G.ay = P.d[3];
    G.by = P.d[2];
    G.tx0 = 2 * xs + P.vx;
    int ulo = __builtin_amdgcn_readfirstlane(win.x), uhi = __builtin_amdgcn_readfirstlane(win.y);
    ulo = max(ulo, -(G.tx0 + 2 * (CW - 1)));              // beyond: left of every map column
    uhi = min(uhi, P.Wp - 1 - G.tx0);                     // beyond: right of every map column
    const int d = (G.tx0 + ulo) & 3;                      // staged rows start 16-byte aligned, d before the scan
    G.ulo = ulo;
    G.Wr = uhi - ulo + 1;
    G.Wq = (G.Wr + 3) & ~3;
    G.vlo = __builtin_amdgcn_readfirstlane(win.z);
    G.vhi = __builtin_amdgcn_readfirstlane(win.w);
    G.Wc = G.vhi - G.vlo + 1;
    G.live = P.Hp > 0 && P.Wp > 0 && G.Wr > 0;
    G.CH = (2 * (CW - 1) + d + G.Wq + 3) >> 2;
    G.SH = 2 * G.CH;
    // offset e of lane j is staged position 2 j + d + e: with e even it lies in
    // the half of d's parity, from d / 2 on; with e odd in the other half
    G.offA = (d & 1) ? G.SH + (d >> 1) : d >> 1;
    G.offB = (d & 1) ? (d + 1) >> 1 : G.SH + (d >> 1);
    int lrb = 5;                                          // up to 32 rows per round
    while (lrb > 0 && (2 * G.SH << lrb) > stage_words) --lrb;
    // pitch 16 mod 32 floats when that keeps the rows per round: the four rows
    // of a wavefront then start in four different 16-bank groups
    G.SP = 2 * G.SH + ((16 - 2 * G.SH) & 31);
    if ((G.SP << lrb) > stage_words) G.SP = 2 * G.SH;
    G.lrb = lrb;
    G.RB = 1 << lrb;
    G.ry0 = max(0, P.vy + G.vlo);
    // the column pass reads up to 3 rows past the last target's window (its
    // offsets go in groups of 4): those rows are row-pass rows too when they
    // lie in the map, and the -inf pad rows beyond it
    G.ry1 = min(P.Hp - 1, 2 * (M.Ho - 1) + P.vy + G.vhi + 3);
    G.rounds = (G.live && G.ry1 >= G.ry0) ? (G.ry1 - G.ry0 + G.RB) >> lrb : 0;
    G.X0 = G.tx0 + ulo - d;
    constexpr int LNT = NT == 512 ? 9 : 8;
    static_assert(NT == 1 << LNT, "256 or 512 threads");
    G.tpr = NT >> lrb;
    G.nq = (G.CH + G.tpr - 1) >> (LNT - lrb);             // <= place_loads<NT>() since RB * CH <= 512
    G.lrow = (int)threadIdx.x >> (LNT - lrb);
    G.lcol = (int)threadIdx.x & (G.tpr - 1);
    return G;
}

// Loads of one round of staged response rows into registers: thread (row
// lrow, float4 runs lcol + q * tpr).  Every load is issued at a clamped,
// aligned address with nothing depending on it until the store, so that all
// of them are in flight together; out-of-map columns are masked at the store
// (a clamped run lies wholly outside the map).
template <int LD>
__device__ __forceinline__ void place_load(const PlaceGeo& G, const float* __restrict__ resp,
                                           int round, float4 (&pf)[LD]) {
    const int y = min(G.ry0 + (round << G.lrb) + G.lrow, G.ry1);
    const float* base = resp + G.plane + __umul24(y, G.ld);     // full-rate 24-bit product
#pragma unroll
    for (int q = 0; q < LD; ++q) {
        const int x = G.X0 + 4 * (G.lcol + q * G.tpr);
        pf[q] = *reinterpret_cast<const float4*>(base + min(max(x, 0), G.ld - 4));
    }
}

// Store of a loaded round into the staging buffer, [row][parity][SH]: the
// run x, x+1, x+2, x+3 (x even) goes to even[x/2 .. x/2+1], odd[x/2 .. x/2+1].
template <int LD>
__device__ __forceinline__ void place_store(const PlaceGeo& G, float* stage, const float4 (&pf)[LD]) {
    if (G.lrow >= G.RB) return;
#pragma unroll
    for (int q = 0; q < LD; ++q) {
        const int c = G.lcol + q * G.tpr;
        if (q < G.nq && c < G.CH) {
            const int x = G.X0 + 4 * c;
            const float4 v = pf[q];
            const float v0 = (unsigned)x < (unsigned)G.Wp ? v.x : -INFINITY;
            const float v1 = (unsigned)(x + 1) < (unsigned)G.Wp ? v.y : -INFINITY;
            const float v2 = (unsigned)(x + 2) < (unsigned)G.Wp ? v.z : -INFINITY;
            const float v3 = (unsigned)(x + 3) < (unsigned)G.Wp ? v.w : -INFINITY;
            float* even = stage + __umul24(G.lrow, G.SP) + 2 * c;
            *reinterpret_cast<float2*>(even) = make_float2(v0, v2);
            *reinterpret_cast<float2*>(even + G.SH) = make_float2(v1, v3);
        }
    }
}

template <int NT>
__global__ __launch_bounds__(NT) void place_kernel(const MapDesc* __restrict__ maps,
                                                    const MapPart* __restrict__ parts,
                                                    const int2* __restrict__ blkmap,
                                                    const float* __restrict__ resp,
                                                    const int* __restrict__ rmax,
                                                    const int* __restrict__ rmin,
                                                    float* __restrict__ scores,
                                                    int16_t* __restrict__ offs, int n_blocks,
                                                    const uint8_t* __restrict__ flags) {
    constexpr int CW = PLACE_CW, PAD = PLACE_PAD, RPW = PLACE_RPW;
    constexpr int ROWS = NT / CW;                          // row slots of the workgroup
    constexpr int LD = place_loads<NT>();
    extern __shared__ __align__(16) float psm[];

    const int item = xcd_item<PLACE_XCL>(blockIdx.x);
    if (item >= n_blocks) return;
    const int2 bm = blkmap[item];                          // (map, strip)
    const MapDesc M = maps[bm.x];
    // LDS laid out for this map (every offset a multiple of 16 bytes, CW = 16)
    float* acc = psm;                                      // [Ho][CW]
    float* r1v = acc + M.Ho * CW;                          // [r1_rows][CW], row y' at y' + PAD
    float* stage = r1v + M.r1_rows * CW;                   // [PLACE_STAGE]
    float* crow = stage + PLACE_STAGE;                     // row-pass cost table
    float* ccol = crow + M.ctab_words;                     // column-pass cost table
    int16_t* r1a = reinterpret_cast<int16_t*>(ccol + M.ctab_words);   // [r1_rows][CW]
    uint8_t* rej = reinterpret_cast<uint8_t*>(r1a + M.r1_rows * CW); // [Ho][CW] rejected
    int4* win = reinterpret_cast<int4*>(rej + M.Ho * CW);             // [n_parts] part_windows
    const int xs = bm.y * CW;
    const int ncol = min(CW, M.Wo - xs);
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);    // wavefront-uniform
    const int j = tid % CW, rr = tid / CW, hr = rr % RPW;
    // position of (y0a + hr, xs + j) in a score map / the root plane: a
    // wave-uniform y0a * Wo (scalar) plus these per-thread offsets
    const uint32_t pos_hr = __umul24(hr, M.Wo) + xs + j;
    const uint32_t rpos_hr = __umul24(hr, M.ldr) + xs + j;

    // Algorithm 1's early exit: a root position is rejected when a partial CP
    // sum of its root (at the position) or of a part (at its anchor) fell
    // below that filter's threshold; its score is -inf and its offsets 0.  A
    // strip whose every position is rejected skips the transform.
    if (flags != nullptr) {
        int live = 0;
        for (int y0 = rr; y0 < M.Ho; y0 += ROWS) {
            if (j >= ncol) continue;
            bool out = flags[M.root_plane + (int64_t)y0 * M.ldr + xs + j] != 0;
            for (int s = 0; s < M.n_parts && !out; ++s) {
                const MapPart& P = parts[M.part_base + s];
                const int ay = 2 * y0 + P.vy, ax = 2 * (xs + j) + P.vx;
                if (ay < P.Hp && ax < P.Wp) out = flags[P.plane + (int64_t)ay * P.ld + ax] != 0;
            }
            rej[y0 * CW + j] = out;
            live |= !out;
        }
        if (!__syncthreads_or(live)) {
            for (int y0 = rr; y0 < M.Ho; y0 += ROWS) {
                if (j >= ncol) continue;
                scores[M.score_off + (int64_t)y0 * M.Wo + xs + j] = -INFINITY;
                for (int s = 0; s < M.n_parts && offs; ++s)
                    reinterpret_cast<uint32_t*>(offs + M.offs_off)[((int64_t)s * M.Ho + y0) * M.Wo + xs + j] = 0u;
            }
            return;
        }
    }

    for (int s = tid; s < M.n_parts; s += NT) win[s] = part_windows(parts[M.part_base + s], rmax, rmin);
    __syncthreads();

    float4 pf[LD];
    PlaceGeo G = place_geo<NT>(parts[M.part_base], M, xs, win[0], PLACE_STAGE);
    if (G.rounds > 0) place_load(G, resp, 0, pf);

    int pad_hp = -1;                                       // part height the -inf pad rows are at
    for (int s = 0; s < M.n_parts; ++s) {
        // pf holds round 0 of part s (when it has rows)
        if (G.live) {
            for (int e = tid; e < G.Wq; e += NT) crow[e] = e < G.Wr ? quad_cost(G.ax, G.bx, G.ulo + e) : INFINITY;
            for (int e = tid; e < G.Wc + 4; e += NT) ccol[e] = e < G.Wc ? quad_cost(G.ay, G.by, G.vlo + e) : INFINITY;
            if (G.Hp != pad_hp) {                          // the row pass writes rows [0, Hp) only
                for (int i = tid; i < 2 * PAD * CW; i += NT) {
                    const int r = i / CW;
                    r1v[(r < PAD ? r : G.Hp + r) * CW + (i - r * CW)] = -INFINITY;
                }
                pad_hp = G.Hp;
            }
            if (G.rounds > 0) place_store(G, stage, pf);
        }
        __syncthreads();                                   // tables, pads, round 0 staged
        const bool has_next = s + 1 < M.n_parts;
        PlaceGeo Gn = G;
        if (has_next) Gn = place_geo<NT>(parts[M.part_base + s + 1], M, xs, win[s + 1], PLACE_STAGE);
        if (G.live) {
            // row pass
            for (int r = 0; r < G.rounds; ++r) {
                const bool more = r + 1 < G.rounds;
                if (more) place_load(G, resp, r + 1, pf);
                else if (has_next && Gn.rounds > 0) place_load(Gn, resp, 0, pf);
                const int yr = G.ry0 + (r << G.lrb);
                for (int q = rr; q < G.RB; q += ROWS) {
                    const int y = yr + q;
                    if (y > G.ry1) break;
                    const float* SE = stage + __umul24(q, G.SP) + j + G.offA;   // even offsets
                    const float* SO = stage + __umul24(q, G.SP) + j + G.offB;   // odd offsets
                    // running maximum per group of 4 offsets; the first group
                    // that reaches the maximum holds the smallest maximiser
                    float best = -INFINITY;
                    int garg = 0;
                    for (int e = 0; e < G.Wq; e += 4) {
                        const int k = e >> 1;
                        const float4 c = *reinterpret_cast<const float4*>(crow + e);
                        const float v0 = SE[k] - c.x, v1 = SO[k] - c.y;
                        const float v2 = SE[k + 1] - c.z, v3 = SO[k + 1] - c.w;
                        const float m = fmaxf(fmaxf(v0, v1), fmaxf(v2, v3));
                        if (m > best) { best = m; garg = e; }
                    }
                    int arg;
                    {   // recompute the winning group: its first offset equal to the maximum
                        const int k = garg >> 1;
                        const float4 c = *reinterpret_cast<const float4*>(crow + garg);
                        const float v0 = SE[k] - c.x, v1 = SO[k] - c.y, v2 = SE[k + 1] - c.z;
                        arg = garg + min(min(v0 == best ? 0 : 3, v1 == best ? 1 : 3), v2 == best ? 2 : 3);
                    }
                    const bool ok = G.tx0 + 2 * j < G.Wp;
                    r1v[(y + PAD) * CW + j] = ok ? best : -INFINITY;
                    r1a[(y + PAD) * CW + j] = (int16_t)(G.tx0 + G.ulo + 2 * j + arg);
                }
                __syncthreads();                           // stage consumed, R1 rows visible
                if (more) {
                    place_store(G, stage, pf);
                    __syncthreads();
                }
            }
            if (G.rounds == 0 && has_next && Gn.rounds > 0) place_load(Gn, resp, 0, pf);
            // column pass: wave w takes RPW consecutive root rows of every ROWS;
            // window offsets clamped so that every skipped candidate lies
            // outside the map for all of them and every read stays in the pads
            for (int y0a = RPW * w; y0a < M.Ho; y0a += ROWS) {
                const int tya = 2 * y0a + G.vy;
                const int ulw = max(G.vlo, -2 * (RPW - 1) - tya), uhw = min(G.vhi, G.Hp - 1 - tya);
                float best = -INFINITY;
                int arg = 0;
                if (ulw <= uhw) {
                    const int e0 = (ulw - G.vlo) & ~3, e1 = uhw - G.vlo;
                    const float* col = r1v + (tya + 2 * hr + G.vlo + PAD) * CW + j;
                    int garg = e0;
                    for (int e = e0; e <= e1; e += 4) {
                        const float4 c = *reinterpret_cast<const float4*>(ccol + e);
                        const float* q = col + e * CW;
                        const float v0 = q[0] - c.x, v1 = q[CW] - c.y;
                        const float v2 = q[2 * CW] - c.z, v3 = q[3 * CW] - c.w;
                        const float m = fmaxf(fmaxf(v0, v1), fmaxf(v2, v3));
                        if (m > best) { best = m; garg = e; }
                    }
                    const float4 c = *reinterpret_cast<const float4*>(ccol + garg);
                    const float* q = col + garg * CW;
                    const float v0 = q[0] - c.x, v1 = q[CW] - c.y, v2 = q[2 * CW] - c.z;
                    arg = garg + min(min(v0 == best ? 0 : 3, v1 == best ? 1 : 3), v2 == best ? 2 : 3);
                }
                const int y0 = y0a + hr;
                if (y0 < M.Ho && j < ncol) {
                    const int ty = tya + 2 * hr, tx = G.tx0 + 2 * j;
                    float D = -INFINITY;
                    uint32_t packed = 0;
                    if (ty < G.Hp && tx < G.Wp) {
                        const int yb = ty + G.vlo + arg;
                        const int dx = r1a[(yb + PAD) * CW + j] - tx, dy = yb - ty;
                        D = best;
                        packed = (uint32_t)(uint16_t)(int16_t)dy | ((uint32_t)(uint16_t)(int16_t)dx << 16);
                    }
                    float* a = acc + y0 * CW + j;
                    *a = s == 0 ? D : *a + D;
                    if (flags != nullptr && rej[y0 * CW + j]) packed = 0u;
                    if (offs)
                        (reinterpret_cast<uint32_t*>(offs + M.offs_off) + (int64_t)s * M.Ho * M.Wo +
                         y0a * M.Wo)[pos_hr] = packed;
                }
            }
        } else {
            // no target of this strip lies inside the part map
            if (has_next && Gn.rounds > 0) place_load(Gn, resp, 0, pf);
            for (int y0a = RPW * w; y0a < M.Ho; y0a += ROWS) {
                const int y0 = y0a + hr;
                if (y0 < M.Ho && j < ncol) {
                    acc[y0 * CW + j] = -INFINITY;
                    if (offs)
                        (reinterpret_cast<uint32_t*>(offs + M.offs_off) + (int64_t)s * M.Ho * M.Wo +
                         y0a * M.Wo)[pos_hr] = 0u;
                }
            }
        }
        __syncthreads();                                   // R1, tables and stage reused by the next part
        G = Gn;
    }
    for (int y0a = RPW * w; y0a < M.Ho; y0a += ROWS) {
        const int y0 = y0a + hr;
        if (y0 < M.Ho && j < ncol)
            (scores + M.score_off + y0a * M.Wo)[pos_hr] =
                (flags != nullptr && rej[y0 * CW + j]) ? -INFINITY
                                                       : (resp + M.root_plane + y0a * M.ldr)[rpos_hr] + acc[y0 * CW + j];
    }
}

__global__ void range_init_kernel(int* __restrict__ rkeys, int64_t n_slots) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n_slots) {
        rkeys[i] = INT_MIN;             // maxima
        rkeys[n_slots + i] = INT_MAX;   // minima
    }
}

hipError_t launch_range_init(int* rkeys, int64_t n_slots, hipStream_t st) {
    if (n_slots <= 0) return hipSuccess;
    hipLaunchKernelGGL(range_init_kernel, dim3((unsigned)((n_slots + 255) / 256)), dim3(256), 0, st,
                       rkeys, n_slots);
    return hipGetLastError();
}

hipError_t launch_place(const MapDesc* maps, const MapPart* parts, const int2* blkmap,
                        int n_blocks, const float* resp, const int* rkeys, int64_t n_slots,
                        float* scores, int16_t* offs, size_t bytes, const uint8_t* flags,
                        hipStream_t st) {
    if (n_blocks <= 0) return hipSuccess;
    if (bytes == 0 || bytes > PLACE_LDS_MAX) return hipErrorInvalidValue;
    // A block's LDS does not grow with its threads: where LDS caps a CU below
    // the register limit, blocks of 512 threads give it more wavefronts.
    const bool wide = 8 * place_blocks_per_cu(bytes, 512) > 4 * place_blocks_per_cu(bytes, 256);
    const void* fn = wide ? reinterpret_cast<const void*>(place_kernel<512>)
                          : reinterpret_cast<const void*>(place_kernel<256>);
    // the kernel's own static LDS (queried once) must fit beside the dynamic part
    static const size_t static_lds = [] {
        hipFuncAttributes fa, fb;
        return hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(place_kernel<256>)) == hipSuccess &&
                       hipFuncGetAttributes(&fb, reinterpret_cast<const void*>(place_kernel<512>)) == hipSuccess
                   ? std::max(fa.sharedSizeBytes, fb.sharedSizeBytes) : ~size_t(0);
    }();
    if (static_lds > 160 * 1024 - PLACE_LDS_MAX) return hipErrorInvalidValue;
    if (bytes > 65536) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
    }
    const dim3 grid(xcd_grid(n_blocks, PLACE_XCL));
    if (wide)
        hipLaunchKernelGGL(place_kernel<512>, grid, dim3(512), bytes, st, maps, parts, blkmap, resp, rkeys,
                           rkeys + n_slots, scores, offs, n_blocks, flags);
    else
        hipLaunchKernelGGL(place_kernel<256>, grid, dim3(256), bytes, st, maps, parts, blkmap, resp, rkeys,
                           rkeys + n_slots, scores, offs, n_blocks, flags);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Detections (Algorithm 1: keep every hypothesis with score >= tau), as a
// deterministic stream compaction over the concatenated score maps: counts per
// block of DET_SPAN positions, an exclusive scan of the counts in two levels
// (within segments of DET_SEG counts in parallel, then of the segment sums),
// then every block writes its detections in position order at its offset.
// ---------------------------------------------------------------------------
constexpr int DET_PER_THREAD = 4;
constexpr int DET_SPAN = 256 * DET_PER_THREAD;

__device__ __forceinline__ int block_exclusive_scan(int v, int* sh, int& total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int x = v;                                         // inclusive scan within the wavefront
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) sh[w] = x;
    __syncthreads();
    int before = 0;
    total = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int t = sh[i];
        if (i < w) before += t;
        total += t;
    }
    __syncthreads();
    return before + x - v;
}

__global__ __launch_bounds__(256) void detect_count_kernel(const float* __restrict__ scores, int64_t n,
                                                           float tau, int64_t* __restrict__ counts) {
    __shared__ int sh[4];
    const int64_t p0 = (int64_t)blockIdx.x * DET_SPAN + (int64_t)threadIdx.x * DET_PER_THREAD;
    int c = 0;
#pragma unroll
    for (int k = 0; k < DET_PER_THREAD; ++k) c += (p0 + k < n && scores[p0 + k] >= tau) ? 1 : 0;
    int total;
    block_exclusive_scan(c, sh, total);
    if (threadIdx.x == 0) counts[blockIdx.x] = total;
}

// Exclusive scan of the block counts within every segment of DET_SEG of them
// (one workgroup per segment, 4 counts per thread), the segment's total to
// sums[segment].
__global__ __launch_bounds__(256) void detect_segscan_kernel(int64_t* __restrict__ counts, int nb,
                                                             int64_t* __restrict__ sums) {
    static_assert(DET_SEG == 4 * 256, "a segment is 4 counts per thread");
    __shared__ int sh[4];
    const int64_t i0 = (int64_t)blockIdx.x * DET_SEG + 4 * threadIdx.x;
    int v[4];
    int c = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] = i0 + k < nb ? (int)counts[i0 + k] : 0;      // each at most DET_SPAN
        c += v[k];
    }
    int total;
    int ex = block_exclusive_scan(c, sh, total);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (i0 + k < nb) counts[i0 + k] = ex;
        ex += v[k];
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Exclusive scan of the segment sums in place (one workgroup, chunks of 256),
// total count to *count.
__global__ __launch_bounds__(256) void detect_scan_kernel(int64_t* __restrict__ counts, int nb,
                                                          int64_t* __restrict__ count) {
    __shared__ int sh[4];
    int64_t carry = 0;
    for (int base = 0; base < nb; base += 256) {
        const int i = base + (int)threadIdx.x;
        const int v = i < nb ? (int)counts[i] : 0;     // at most DET_SEG * DET_SPAN
        int total;
        const int ex = block_exclusive_scan(v, sh, total);
        if (i < nb) counts[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) *count = carry;
}

__global__ __launch_bounds__(256) void detect_write_kernel(const float* __restrict__ scores, int64_t n,
                                                           float tau, const int64_t* __restrict__ counts,
                                                           const int64_t* __restrict__ sums,
                                                           const MapDesc* __restrict__ maps, int n_maps,
                                                           Detection* __restrict__ dets, int64_t capacity) {
    __shared__ int sh[4];
    const int64_t p0 = (int64_t)blockIdx.x * DET_SPAN + (int64_t)threadIdx.x * DET_PER_THREAD;
    bool hit[DET_PER_THREAD];
    float val[DET_PER_THREAD];
    int c = 0;
#pragma unroll
    for (int k = 0; k < DET_PER_THREAD; ++k) {
        val[k] = p0 + k < n ? scores[p0 + k] : -INFINITY;
        hit[k] = p0 + k < n && val[k] >= tau;
        c += hit[k] ? 1 : 0;
    }
    int total;
    int64_t out = sums[blockIdx.x / DET_SEG] + counts[blockIdx.x] + block_exclusive_scan(c, sh, total);
#pragma unroll
    for (int k = 0; k < DET_PER_THREAD; ++k) {
        if (!hit[k]) continue;
        if (out < capacity) {
            const int64_t p = p0 + k;
            int lo = 0, hi = n_maps - 1;              // last map whose scores start at or before p
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (maps[mid].score_off <= p) lo = mid;
                else hi = mid - 1;
            }
            const MapDesc M = maps[lo];
            const int64_t r = p - M.score_off;
            Detection d;
            d.map = lo;
            d.y = (int32_t)(r / M.Wo);
            d.x = (int32_t)(r - (int64_t)d.y * M.Wo);
            d.score = val[k];
            dets[out] = d;
        }
        ++out;
    }
}

hipError_t launch_detect(const float* scores, int64_t n, float tau, const MapDesc* maps, int n_maps,
                         int64_t* counts, int64_t* count, Detection* dets, int64_t capacity,
                         hipStream_t st) {
    const int64_t nb = (n + DET_SPAN - 1) / DET_SPAN;
    const int64_t nseg = (nb + DET_SEG - 1) / DET_SEG;
    if (nb > INT32_MAX) return hipErrorInvalidValue;
    int64_t* sums = counts + nb;                       // det_blocks(n) = nb + nseg
    if (nb > 0) {
        hipLaunchKernelGGL(detect_count_kernel, dim3((unsigned)nb), dim3(256), 0, st, scores, n, tau, counts);
        hipLaunchKernelGGL(detect_segscan_kernel, dim3((unsigned)nseg), dim3(256), 0, st, counts, (int)nb, sums);
    }
    hipLaunchKernelGGL(detect_scan_kernel, dim3(1), dim3(256), 0, st, sums, (int)nseg, count);
    if (nb > 0 && capacity > 0)
        hipLaunchKernelGGL(detect_write_kernel, dim3((unsigned)nb), dim3(256), 0, st, scores, n, tau,
                           counts, sums, maps, n_maps, dets, capacity);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// filter planes of one group (pitch ld) -> one row-major map per filter
// ---------------------------------------------------------------------------
__global__ void planes_to_maps_kernel(const float* __restrict__ planes, int ng, int Ho, int Wo,
                                      int ld, const int64_t* __restrict__ dst_off,
                                      float* __restrict__ out) {
    const int64_t n = (int64_t)ng * Ho * Wo;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int64_t row = i / Wo;                    // f * Ho + y
    const int x = (int)(i - row * Wo);
    const int f = (int)(row / Ho);
    const int y = (int)(row - (int64_t)f * Ho);
    out[dst_off[f] + (int64_t)y * Wo + x] = planes[row * ld + x];
}

hipError_t launch_planes_to_maps(const float* planes, int ng, int Ho, int Wo, int ld,
                                 const int64_t* dst_off, float* out, hipStream_t st) {
    const int64_t n = (int64_t)ng * Ho * Wo;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(planes_to_maps_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       planes, ng, Ho, Wo, ld, dst_off, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// single-map distance transform for every target cell: the same exact window
// scan with target stride 1; row pass with one thread per (row, target chunk),
// column pass with one thread per (column, target chunk), x fastest so that
// the column pass reads rows of the intermediate coalesced
// ---------------------------------------------------------------------------
constexpr int DT1_CHUNK = 16;                      // targets per thread

__global__ __launch_bounds__(256) void dt1_row_kernel(const float* __restrict__ v, int rows, int cols,
                                                      int64_t ld, const float* __restrict__ M,
                                                      float a, float b, float* __restrict__ ov,
                                                      int32_t* __restrict__ oa) {
    const int nch = (cols + DT1_CHUNK - 1) / DT1_CHUNK;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)rows * nch) return;
    const int y = (int)(i / nch), c = (int)(i - (int64_t)y * nch);
    const float* row = v + y * ld;
    int prev = 0;
    for (int k = c * DT1_CHUNK; k < min(cols, (c + 1) * DT1_CHUNK); ++k) {
        int arg;
        ov[(int64_t)y * cols + k] = window_max([&](int x) { return row[x]; }, cols, k, prev, a, b, M[y], arg);
        oa[(int64_t)y * cols + k] = arg;
        prev = arg;
    }
}

__global__ __launch_bounds__(256) void dt1_col_kernel(const float* __restrict__ r1v,
                                                      const int32_t* __restrict__ r1a, int rows,
                                                      int cols, const float* __restrict__ M, float a,
                                                      float b, float* __restrict__ out,
                                                      int32_t* __restrict__ ay,
                                                      int32_t* __restrict__ ax) {
    const int nch = (rows + DT1_CHUNK - 1) / DT1_CHUNK;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)cols * nch) return;
    const int c = (int)(i / cols), x = (int)(i - (int64_t)c * cols);
    int prev = 0;
    for (int k = c * DT1_CHUNK; k < min(rows, (c + 1) * DT1_CHUNK); ++k) {
        int arg;
        const int64_t o = (int64_t)k * cols + x;
        out[o] = window_max([&](int y) { return r1v[(int64_t)y * cols + x]; }, rows, k, prev, a, b, M[x], arg);
        if (ay) ay[o] = arg;
        if (ax) ax[o] = r1a[(int64_t)arg * cols + x];
        prev = arg;
    }
}

__global__ void dt1_rowmax_kernel(const float* __restrict__ v, int rows, int cols, int64_t ld,
                                  float* __restrict__ M) {
    const int y = blockIdx.x * 256 + threadIdx.x;
    if (y >= rows) return;
    float m = -FLT_MAX;
    for (int x = 0; x < cols; ++x) m = fmaxf(m, v[y * ld + x]);
    M[y] = m;
}

__global__ void dt1_colmax_kernel(const float* __restrict__ v, int rows, int cols,
                                  float* __restrict__ M) {
    const int x = blockIdx.x * 256 + threadIdx.x;
    if (x >= cols) return;
    float m = -FLT_MAX;
    for (int y = 0; y < rows; ++y) m = fmaxf(m, v[(int64_t)y * cols + x]);
    M[x] = m;
}

hipError_t launch_dt_single(const float* resp, int rows, int cols, int ld, const float* d,
                            float* lmax, float* r1v, int32_t* r1a, float* out, int32_t* ay,
                            int32_t* ax, hipStream_t st) {
    if ((int64_t)rows * cols <= 0) return hipSuccess;
    const int64_t nr = (int64_t)rows * ((cols + DT1_CHUNK - 1) / DT1_CHUNK);
    const int64_t nc = (int64_t)cols * ((rows + DT1_CHUNK - 1) / DT1_CHUNK);
    hipLaunchKernelGGL(dt1_rowmax_kernel, dim3((rows + 255) / 256), dim3(256), 0, st, resp, rows,
                       cols, (int64_t)ld, lmax);
    hipLaunchKernelGGL(dt1_row_kernel, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, st, resp,
                       rows, cols, (int64_t)ld, lmax, d[1], d[0], r1v, r1a);
    hipLaunchKernelGGL(dt1_colmax_kernel, dim3((cols + 255) / 256), dim3(256), 0, st, r1v, rows,
                       cols, lmax);
    hipLaunchKernelGGL(dt1_col_kernel, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st, r1v,
                       r1a, rows, cols, lmax, d[3], d[2], out, ay, ax);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// single-map distance transform by lower envelopes: the same result for every
// target, found in time linear in the line length whatever the deformation.
// Along a line, v[x] - c(x - t) = h_x + 2 a t x - a t^2 + b t with
// h_x = v[x] - a x^2 - b x, so the best x for target t is the line of largest
// value at t among the lines h_x + 2 a x t, whose slopes grow with x: their
// upper envelope is built in one pass over x (a stack; line x beats the top p
// for t > s = (h_p - h_x) / (2 a (x - p)); p leaves the stack when that
// happens at or before the point where p itself took over), and targets in
// increasing order walk it with one pointer.  The envelope is built in FP64
// (for lines up to 2^14 cells a x^2 and b x are exact there, so h_x carries
// a single FP64 rounding), and the answer is decided in FP32 among the
// envelope line found and its two neighbours, with the same value formula
// and tie rule (smallest x) as the window scan, so that the two methods pick
// the same maximiser wherever the FP32 values differ.  One thread per line;
// the envelope of line i lives in scratch element [k][i] (index k, line i
// fastest), so that the threads of a wavefront touch consecutive words.
// ---------------------------------------------------------------------------
template <class Load>
__device__ __forceinline__ void env_line(const Load& load, int n, int nl, int line, float a, float b,
                                         int32_t* __restrict__ hx, double* __restrict__ hz,
                                         float* __restrict__ ov, int64_t ostride, int32_t* __restrict__ oa) {
    const double A = a, B = b;
    // envelope: line hx[j] is the best from hz[j] on (hz[0] = -inf); -inf
    // values never win and are left out
    int m = 0;
    double htop = 0.0;
    for (int x = 0; x < n; ++x) {
        const float vx = load(x);
        if (vx == -INFINITY) continue;
        const double h = (double)vx - (A * x) * x - B * x;
        double s = -INFINITY;
        while (m > 0) {
            const int p = hx[(int64_t)(m - 1) * nl + line];
            s = (htop - h) / (2.0 * A * (double)(x - p));     // x beats p for t > s
            if (m > 1 && s <= hz[(int64_t)(m - 1) * nl + line]) {
                --m;                                           // p is never the smallest best
                const int q = hx[(int64_t)(m - 1) * nl + line];
                htop = (double)load(q) - (A * q) * q - B * q;
                continue;
            }
            break;
        }
        hx[(int64_t)m * nl + line] = x;
        hz[(int64_t)m * nl + line] = m == 0 ? -INFINITY : s;
        ++m;
        htop = h;
    }
    int k = 0;
    for (int t = 0; t < n; ++t) {
        float best = -INFINITY;
        int arg = t;                                   // a line of -inf only
        if (m > 0) {
            while (k + 1 < m && hz[(int64_t)(k + 1) * nl + line] < (double)t) ++k;
            // decided in FP32 among the envelope line and its neighbours,
            // in increasing x: the first of equal values wins
            const int j0 = max(k - 1, 0), j1 = min(k + 1, m - 1);
            arg = hx[(int64_t)j0 * nl + line];
            for (int j = j0; j <= j1; ++j) {
                const int x = hx[(int64_t)j * nl + line];
                const float u = (float)(x - t);
                const float e = load(x) - u * fmaf(a, u, b);
                if (e > best) { best = e; arg = x; }
            }
        }
        ov[(int64_t)t * ostride] = best;
        oa[(int64_t)t * ostride] = arg;
    }
}

__global__ __launch_bounds__(256) void dt1_env_row_kernel(const float* __restrict__ v, int rows, int cols,
                                                          int64_t ld, float a, float b,
                                                          int32_t* __restrict__ hx, double* __restrict__ hz,
                                                          float* __restrict__ ov, int32_t* __restrict__ oa) {
    const int y = blockIdx.x * 256 + threadIdx.x;
    if (y >= rows) return;
    const float* row = v + y * ld;
    env_line([&](int x) { return row[x]; }, cols, rows, y, a, b, hx, hz, ov + (int64_t)y * cols, 1,
             oa + (int64_t)y * cols);
}

__global__ __launch_bounds__(256) void dt1_env_col_kernel(const float* __restrict__ r1v,
                                                          const int32_t* __restrict__ r1a, int rows,
                                                          int cols, float a, float b,
                                                          int32_t* __restrict__ hx, double* __restrict__ hz,
                                                          float* __restrict__ out, int32_t* __restrict__ ay) {
    const int x = blockIdx.x * 256 + threadIdx.x;
    if (x >= cols) return;
    env_line([&](int y) { return r1v[(int64_t)y * cols + x]; }, rows, cols, x, a, b, hx, hz, out + x, cols,
             ay + x);
}

__global__ void dt1_env_ax_kernel(const int32_t* __restrict__ ay, const int32_t* __restrict__ r1a, int rows,
                                  int cols, int32_t* __restrict__ ax) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)rows * cols) return;
    const int x = (int)(i % cols);
    ax[i] = r1a[(int64_t)ay[i] * cols + x];
}

hipError_t launch_dt_envelope(const float* resp, int rows, int cols, int ld, const float* d, float* r1v,
                              int32_t* r1a, int32_t* hx, double* hz, float* out, int32_t* ay, int32_t* ax,
                              hipStream_t st) {
    if ((int64_t)rows * cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(dt1_env_row_kernel, dim3((rows + 255) / 256), dim3(256), 0, st, resp, rows, cols,
                       (int64_t)ld, d[1], d[0], hx, hz, r1v, r1a);
    hipLaunchKernelGGL(dt1_env_col_kernel, dim3((cols + 255) / 256), dim3(256), 0, st, r1v, r1a, rows, cols,
                       d[3], d[2], hx, hz, out, ay);
    if (ax)
        hipLaunchKernelGGL(dt1_env_ax_kernel, dim3((unsigned)(((int64_t)rows * cols + 255) / 256)), dim3(256), 0,
                           st, ay, r1a, rows, cols, ax);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// allocation-free single-map transform: the scratch of launch_dt_single (line
// maxima, then the row pass's values and argmax) lives in this file-scope
// array.  Every kernel writes each scratch element it later reads, so nothing
// needs clearing between calls.  Each GPU holds its own copy at its own
// address; host code uses that address (found once per device with
// hipGetSymbolAddress), never the array's name.  Calls on one GPU share the
// array, so calls that overlap on one GPU race.
// ---------------------------------------------------------------------------
constexpr size_t DT_NA_LMAX = (size_t)DT_NOALLOC_MAX_SIDE * sizeof(float);   // 64 KiB
constexpr size_t DT_NA_PLANE = (size_t)DT_NOALLOC_MAX_CELLS * sizeof(float); // 8 MiB
constexpr int DT_NA_MAX_DEVICES = 64;
static __device__ __align__(256) char scratch[DT_NA_LMAX + 2 * DT_NA_PLANE];

// Device address of the current device's scratch, looked up on the first call
// on that device (with it current) and kept.
static hipError_t dt_noalloc_scratch(char** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= DT_NA_MAX_DEVICES) return hipErrorInvalidDevice;
    static std::mutex mu;
    static char* addr[DT_NA_MAX_DEVICES] = {};
    std::lock_guard<std::mutex> lock(mu);
    if (addr[dev] == nullptr) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (p == nullptr) return hipErrorInvalidSymbol;
        addr[dev] = static_cast<char*>(p);
    }
    *out = addr[dev];
    return hipSuccess;
}

hipError_t launch_dt_single_noalloc(const float* resp, int rows, int cols, int ld, const float* d,
                                    float* out, int32_t* ay, int32_t* ax, hipStream_t st) {
    if (rows > DT_NOALLOC_MAX_SIDE || cols > DT_NOALLOC_MAX_SIDE ||
        (int64_t)rows * cols > DT_NOALLOC_MAX_CELLS)
        return hipErrorInvalidValue;
    char* base = nullptr;
    hipError_t e = dt_noalloc_scratch(&base);
    if (e != hipSuccess) return e;
    float* lmax = reinterpret_cast<float*>(base);
    float* r1v = reinterpret_cast<float*>(base + DT_NA_LMAX);
    int32_t* r1a = reinterpret_cast<int32_t*>(base + DT_NA_LMAX + DT_NA_PLANE);
    return launch_dt_single(resp, rows, cols, ld, d, lmax, r1v, r1a, out, ay, ax, st);
}

}  // namespace dpmt
