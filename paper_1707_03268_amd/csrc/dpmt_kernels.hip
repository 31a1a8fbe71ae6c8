// HIP kernels of libdpmt for gfx950 (CDNA4, 64-lane wavefronts).
//
//   project_kernel     Z = X x_3 U^T per cell (feature contraction of the
//                      tensor form, Section 4), VALU, HBM bound
//   corr_kernel        valid correlation of one level with a group of
//                      equally sized filters as a shift-GEMM on MFMA
//                      (positions x filters x (taps * channels)), FP32 or BF16
//                      operands, FP32 accumulation; used for the direct and
//                      the shortened (rank-R) responses
//   dt_row_kernel /    separable generalised distance transform (Section 2
//   dt_col_kernel      placement argmax) evaluated at the part anchors of
//                      every root position; exact windowed scan
//   assemble_kernel    s(p0) = root response + sum of the parts' deformed
//                      scores (Section 2 score formula)
#include "dpmt_internal.h"

#include <cfloat>
#include <climits>

namespace dpmt {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------
// projection: Z[c][r] = sum_l X[c][l] * U[l][r]   (U: 32 x RP fp32, row major)
// ---------------------------------------------------------------------------
template <int RP, bool BF16>
__global__ __launch_bounds__(256) void project_kernel(const float* __restrict__ X, int64_t n_cells,
                                                      const float* __restrict__ U,
                                                      void* __restrict__ Zv) {
    __shared__ float sU[32 * RP];
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
                          void* Z, hipStream_t st) {
    if (n_cells <= 0) return hipSuccess;
    const unsigned nb = (unsigned)((n_cells + 255) / 256);
#define DPMT_PROJ(R)                                                                          \
    case R:                                                                                   \
        if (bf16) hipLaunchKernelGGL((project_kernel<R, true>), dim3(nb), dim3(256), 0, st,   \
                                     X, n_cells, U, Z);                                       \
        else hipLaunchKernelGGL((project_kernel<R, false>), dim3(nb), dim3(256), 0, st, X,    \
                                n_cells, U, Z);                                               \
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

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ u32x4 lds_load16(const char* p, int pb) {
    if (pb >= 16) return *reinterpret_cast<const u32x4*>(p);
    const u32x2 a = *reinterpret_cast<const u32x2*>(p);
    const u32x2 b = *reinterpret_cast<const u32x2*>(p + 8);
    return u32x4{a.x, a.y, b.x, b.y};
}

template <CorrKind KIND>
__device__ __forceinline__ v16f mfma_step(const u32x4& a, const u32x4& b, v16f c) {
    if constexpr (KIND == CORR_F32) {
        c = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.x), __uint_as_float(b.x), c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.y), __uint_as_float(b.y), c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.z), __uint_as_float(b.z), c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.w), __uint_as_float(b.w), c, 0, 0, 0);
        return c;
    } else {
        v8bf av, bv;
        __builtin_memcpy(&av, &a, 16);
        __builtin_memcpy(&bv, &b, 16);
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, c, 0, 0, 0);
    }
}

template <CorrKind KIND, int PB, int TY, int BB, int WY, int HMAX>
__global__ __launch_bounds__(64 * WY) __attribute__((amdgpu_waves_per_eu(HMAX <= 8 ? 2 : 1))) void corr_kernel(const CorrTile* __restrict__ tiles,
                                                       const GroupDesc* __restrict__ groups,
                                                       const char* __restrict__ Z,
                                                       const char* __restrict__ G,
                                                       float* __restrict__ out, int cell_bytes,
                                                       int Q, int win_bytes) {
    extern __shared__ __align__(16) char smem[];
    constexpr int NT = 64 * WY;
    constexpr int TYWG = TY * WY;
    constexpr int CH = PB >= 16 ? 16 : 8;          // window copy granule
    constexpr int PFMAX = (BB * HMAX * 64 + NT - 1) / NT;   // chunk u32x4 per thread, h <= HMAX
    constexpr int WBATCH = 4;                      // window loads in flight per thread

    const CorrTile t = tiles[blockIdx.x];
    const GroupDesc g = groups[t.group];
    const int h = g.h, S = g.S;
    const int WC = 31 + (32 * S) / PB;             // window cells per row
    const int pitch = WC * PB;
    const int nrows = TYWG + h - 1;
    char* win = smem;
    u32x4* gbuf0 = reinterpret_cast<u32x4*>(smem + win_bytes);
    u32x4* gbuf1 = gbuf0 + BB * h * 64;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int p = lane & 31, j = lane >> 5;

    v16f acc[TY][BB];
#pragma unroll
    for (int i = 0; i < TY; ++i)
#pragma unroll
        for (int b = 0; b < BB; ++b)
#pragma unroll
            for (int k = 0; k < 16; ++k) acc[i][b][k] = 0.f;

    const int n_chunk = BB * h * 64;               // u32x4 per G chunk
    const int total = Q * S;
    // element i of chunk `step`: [b][n][lane] of the packed operand.  Indices
    // past the chunk are clamped to its last element, for the load and for the
    // LDS store alike, so surplus threads store that element's own value again.
    auto chunk_src = [&](int step, int i) -> const u32x4* {
        i = min(i, n_chunk - 1);
        const int q = step / S, s = step - q * S;
        const int l = i & 63;
        const int n = (i >> 6) % h;
        const int b = i / (64 * h);
        const int64_t blk = t.fb0 + b;
        return reinterpret_cast<const u32x4*>(
                   G + g.g_off + ((((blk * Q + q) * S + s) * (int64_t)h + n) << 10)) + l;
    };

    // prologue: chunk 0 straight into buffer 0
    {
        u32x4 pf[PFMAX];
#pragma unroll
        for (int k = 0; k < PFMAX; ++k) pf[k] = *chunk_src(0, tid + k * NT);
#pragma unroll
        for (int k = 0; k < PFMAX; ++k) gbuf0[min(tid + k * NT, n_chunk - 1)] = pf[k];
    }

    for (int step = 0; step < total; ++step) {
        const int q = step / S, s = step - q * S;
        if (s == 0) {
            __syncthreads();                       // previous plane fully consumed
            const int cpc = PB / CH;
            const int nch = nrows * WC * cpc;
            for (int i0 = tid; i0 < nch; i0 += WBATCH * NT) {
                u32x4 r[WBATCH];
#pragma unroll
                for (int u = 0; u < WBATCH; ++u) {
                    const int i = min(i0 + u * NT, nch - 1);
                    const int k = i % cpc;
                    const int cc = (i / cpc) % WC;
                    const int rr = i / (cpc * WC);
                    const int y = t.y0 + rr, x = t.x0 + cc;
                    const bool in = (y < t.H) && (x < t.W);
                    const int64_t cell = t.z_cell + (in ? (int64_t)y * t.W + x : 0);
                    const char* src = Z + (cell * cell_bytes + q * PB + k * CH);
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
                    const int i = min(i0 + u * NT, nch - 1);   // surplus: same value again
                    const int k = i % cpc;
                    const int cc = (i / cpc) % WC;
                    const int rr = i / (cpc * WC);
                    char* dst = win + rr * pitch + cc * PB + k * CH;
                    if constexpr (CH == 16) *reinterpret_cast<u32x4*>(dst) = r[u];
                    else *reinterpret_cast<u32x2*>(dst) = u32x2{r[u].x, r[u].y};
                }
            }
        }
        __syncthreads();                           // window and chunk `step` visible

        // issue the loads of the next chunk before this step's MFMAs (the last
        // step reloads its own chunk and does not store it)
        u32x4 pf[PFMAX];
        const bool more = step + 1 < total;
        const int nstep = more ? step + 1 : step;
#pragma unroll
        for (int k = 0; k < PFMAX; ++k) pf[k] = *chunk_src(nstep, tid + k * NT);

        const u32x4* gb = (step & 1) ? gbuf1 : gbuf0;
        const char* abase = win + (wv * TY) * pitch + p * PB + 32 * s + 16 * j;
        u32x4 A[TY];
#pragma unroll
        for (int i = 0; i < TY; ++i) A[i] = lds_load16(abase + i * pitch, PB);
        u32x4 B[BB];
#pragma unroll
        for (int b = 0; b < BB; ++b) B[b] = gb[(b * h) * 64 + lane];
        for (int n = 0; n < h; ++n) {
            u32x4 Bn[BB], An;
            const bool nx = n + 1 < h;
            if (nx) {
#pragma unroll
                for (int b = 0; b < BB; ++b) Bn[b] = gb[(b * h + n + 1) * 64 + lane];
                An = lds_load16(abase + (n + TY) * pitch, PB);
            }
#pragma unroll
            for (int i = 0; i < TY; ++i)
#pragma unroll
                for (int b = 0; b < BB; ++b) acc[i][b] = mfma_step<KIND>(A[i], B[b], acc[i][b]);
            if (nx) {
#pragma unroll
                for (int i = 0; i + 1 < TY; ++i) A[i] = A[i + 1];
                A[TY - 1] = An;
#pragma unroll
                for (int b = 0; b < BB; ++b) B[b] = Bn[b];
            }
        }

        if (more) {
            u32x4* nb = (step & 1) ? gbuf0 : gbuf1;
#pragma unroll
            for (int k = 0; k < PFMAX; ++k) nb[min(tid + k * NT, n_chunk - 1)] = pf[k];
        }
    }

    // epilogue: lane holds filter column p, positions 8*(k/4) + 4*j + k%4
#pragma unroll
    for (int i = 0; i < TY; ++i) {
        const int y = t.y0 + wv * TY + i;
        if (y >= t.Ho) continue;
#pragma unroll
        for (int b = 0; b < BB; ++b) {
            const int f = (t.fb0 + b) * 32 + p;
            if (f >= g.ng) continue;
            float* orow = out + t.out_off + (int64_t)y * t.Wo * g.ng + f;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int x = t.x0 + 8 * (k >> 2) + 4 * j + (k & 3);
                if (x < t.Wo) orow[(int64_t)x * g.ng] = acc[i][b][k];
            }
        }
    }
}

size_t corr_lds_bytes(const CorrLaunch& cfg, int h, int S) {
    const int WC = 31 + (32 * S) / cfg.pk.PB;
    const size_t win = (size_t)(cfg.ty * cfg.wy + h - 1) * WC * cfg.pk.PB;
    const size_t winal = (win + 15) & ~size_t(15);
    return winal + 2 * (size_t)cfg.bb * h * 1024;
}

template <CorrKind KIND, int PB, int TY, int BB, int WY, int HMAX>
static hipError_t launch_corr_h(const CorrTile* tiles, int n_tiles, const GroupDesc* groups,
                                const void* Z, const void* G, float* out, int cell_bytes, int Q,
                                int max_h, int max_S, hipStream_t st) {
    CorrLaunch cfg{KIND, Packing{0, 0, PB, Q}, TY, BB, WY};
    const size_t lds = corr_lds_bytes(cfg, max_h, max_S);
    const int WC = 31 + (32 * max_S) / PB;
    const size_t win = (size_t)(TY * WY + max_h - 1) * WC * PB;
    const int win_bytes = (int)((win + 15) & ~size_t(15));
    auto kern = corr_kernel<KIND, PB, TY, BB, WY, HMAX>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3(n_tiles), dim3(64 * WY), lds, st, tiles, groups,
                       static_cast<const char*>(Z), static_cast<const char*>(G), out, cell_bytes,
                       Q, win_bytes);
    return hipGetLastError();
}

// Filters of at most 8 rows (every DPM root and part shape) get a kernel whose
// chunk prefetch needs half the registers.
template <CorrKind KIND, int PB, int TY, int BB, int WY>
static hipError_t launch_corr_t(const CorrTile* tiles, int n_tiles, const GroupDesc* groups,
                                const void* Z, const void* G, float* out, int cell_bytes, int Q,
                                int max_h, int max_S, hipStream_t st) {
    if (max_h <= 8)
        return launch_corr_h<KIND, PB, TY, BB, WY, 8>(tiles, n_tiles, groups, Z, G, out,
                                                      cell_bytes, Q, max_h, max_S, st);
    return launch_corr_h<KIND, PB, TY, BB, WY, CORR_MAX_H>(tiles, n_tiles, groups, Z, G, out,
                                                           cell_bytes, Q, max_h, max_S, st);
}

hipError_t launch_corr(const CorrLaunch& cfg, const CorrTile* tiles, int n_tiles,
                       const GroupDesc* groups, const void* Z, const void* G, float* out,
                       int max_h, int max_S, hipStream_t st) {
    if (n_tiles <= 0) return hipSuccess;
    if (max_h > CORR_MAX_H) return hipErrorInvalidValue;
    if (cfg.ty != 4 || cfg.bb != 2 || cfg.wy != 4) return hipErrorInvalidValue;
    const int cb = cfg.pk.RP * cfg.pk.esz;
    const int Q = cfg.pk.Q;
    if (cfg.kind == CORR_F32) {
        switch (cfg.pk.PB) {
            case 16: return launch_corr_t<CORR_F32, 16, 4, 2, 4>(tiles, n_tiles, groups, Z, G, out, cb, Q, max_h, max_S, st);
            case 32: return launch_corr_t<CORR_F32, 32, 4, 2, 4>(tiles, n_tiles, groups, Z, G, out, cb, Q, max_h, max_S, st);
            default: return hipErrorInvalidValue;
        }
    } else if (cfg.kind == CORR_BF16) {
        switch (cfg.pk.PB) {
            case 8: return launch_corr_t<CORR_BF16, 8, 4, 2, 4>(tiles, n_tiles, groups, Z, G, out, cb, Q, max_h, max_S, st);
            case 16: return launch_corr_t<CORR_BF16, 16, 4, 2, 4>(tiles, n_tiles, groups, Z, G, out, cb, Q, max_h, max_S, st);
            case 32: return launch_corr_t<CORR_BF16, 32, 4, 2, 4>(tiles, n_tiles, groups, Z, G, out, cb, Q, max_h, max_S, st);
            default: return hipErrorInvalidValue;
        }
    }
    return hipErrorInvalidValue;
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
// Layouts are chosen so that every pass reads and writes whole cache lines:
//   part responses  [y'][x'][filter]     (correlation output)
//   row pass        [pair][y'][x0]       (lanes = target columns of one pair)
//   column pass     caller layout [map][part][y0][x0] (lanes = root columns)
// and each pass stages the lines it scans in LDS, laid out so that lanes
// reading different positions hit different banks.
// ---------------------------------------------------------------------------
constexpr int DT_STAGE_MAX = 96 * 1024;          // LDS bytes of one staged tile
constexpr int DT_ROW_PAIRS = 32;                 // pairs per row-pass block

__device__ __forceinline__ int find_item(const int32_t* __restrict__ prefix, int n, int b) {
    int lo = 0, hi = n - 1;                        // last item with prefix <= b
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

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

// Row pass: block = (item, part row y', 32 pairs).  The block stages the row
// of its 32 pairs in LDS split by parity, [pair][x' & 1][x' >> 1], so that
// lanes holding consecutive target columns (targets 2 apart) read
// consecutive words; then thread (column x0 = tid % Wt, pair slot tid / Wt)
// walks the block's pairs.  Writes the row maximum of
// resp[y'][x'] - (d_x (x'-x_t) + d_xx (x'-x_t)^2), x_t = 2*x0 + v_x, and its
// argmax x' at [pair][y'][x0].
template <bool STAGED>
__global__ __launch_bounds__(256) void dt_row_kernel(const DTItem* __restrict__ items,
                                                     const int32_t* __restrict__ prefix,
                                                     int n_items,
                                                     const PairDesc* __restrict__ pairs,
                                                     const float* __restrict__ resp,
                                                     float* __restrict__ r1v,
                                                     int32_t* __restrict__ r1a) {
    extern __shared__ float sline[];               // [DT_ROW_PAIRS][2][half] when STAGED
    __shared__ float smax[8][DT_ROW_PAIRS];
    __shared__ LineConst sc[DT_ROW_PAIRS];
    __shared__ int2 sv[DT_ROW_PAIRS];              // (v_x, root columns Wo_c)
    const int it = find_item(prefix, n_items, blockIdx.x);
    const DTItem I = items[it];
    const int local = blockIdx.x - prefix[it];
    const int pc = (I.np + DT_ROW_PAIRS - 1) / DT_ROW_PAIRS;
    const int p0 = (local % pc) * DT_ROW_PAIRS;
    const int yp = local / pc;                     // block-uniform
    if (yp >= I.Hp) return;
    const int npb = min(DT_ROW_PAIRS, I.np - p0);  // pairs of this block
    const int Wp = I.Wp;
    const int half = (Wp + 2) >> 1;                // words per parity plane (odd pitch below)
    const int hp = half | 1;
    const int64_t rs = I.ng;
    const float* rowbase = resp + I.resp_off + (int64_t)yp * Wp * rs;
    {   // stage: thread (pair q, x phase) -> coalesced 128-byte reads, 8 in flight
        constexpr int XS = 256 / DT_ROW_PAIRS;
        const int q = threadIdx.x & (DT_ROW_PAIRS - 1), ph = threadIdx.x / DT_ROW_PAIRS;
        const bool act = q < npb;
        const int fcol = act ? pairs[I.pair_base + p0 + q].fcol : 0;
        float M = -FLT_MAX;
        for (int xb = ph; xb < Wp; xb += 8 * XS) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = rowbase[min(xb + u * XS, Wp - 1) * rs + fcol];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int x = xb + u * XS;
                if (x < Wp) {
                    const float vv = act ? v[u] : 0.f;
                    if (STAGED) sline[(q * 2 + (x & 1)) * hp + (x >> 1)] = vv;
                    M = fmaxf(M, vv);
                }
            }
        }
        smax[ph][q] = M;
    }
    __syncthreads();
    if (threadIdx.x < npb) {
        const int q = threadIdx.x;
        const PairDesc P = pairs[I.pair_base + p0 + q];
        float M = smax[0][q];
#pragma unroll
        for (int i = 1; i < 8; ++i) M = fmaxf(M, smax[i][q]);
        sc[q] = LineConst{P.d[1], P.d[0], 0.5f / P.d[1], 0.f, M};
        sv[q] = make_int2(P.vx, min(I.Wr - P.w0 + 1, I.Wt));
    }
    __syncthreads();
    const int Wt = I.Wt;
    const int cols = min(Wt, 256);
    const int qstep = 256 / cols;
    const int x0s = threadIdx.x % cols, qs = threadIdx.x / cols;
    if (qs >= qstep) return;
    const int64_t obase = I.r1_off + ((int64_t)p0 * I.Hp + yp) * Wt;
    const int64_t opair = (int64_t)I.Hp * Wt;
    for (int q = qs; q < npb; q += qstep) {
        const LineConst c = sc[q];
        const int2 vw = sv[q];
        const float* sp = sline + q * 2 * hp;
        for (int x0 = x0s; x0 < vw.y; x0 += cols) {
            const int t = 2 * x0 + vw.x;
            float best = -INFINITY;
            int arg = -1;
            if (t >= 0 && t < Wp) {
                int lo, hi;
                if (STAGED) {
                    auto ld = [&](int x) { return sp[(x & 1) * hp + (x >> 1)]; };
                    dt_bounds(ld(t), c, t, 0, Wp, lo, hi);
                    best = scan_range(ld, lo, hi, t, c.a, c.b, arg);
                } else {
                    const float* grow = rowbase + pairs[I.pair_base + p0 + q].fcol;
                    auto ld = [&](int x) { return grow[x * rs]; };
                    dt_bounds(ld(t), c, t, 0, Wp, lo, hi);
                    best = scan_range(ld, lo, hi, t, c.a, c.b, arg);
                }
            }
            r1v[obase + q * opair + x0] = best;
            r1a[obase + q * opair + x0] = arg;
        }
    }
}

// Column pass: block = (item, pair, chunk of cw root columns).  The block
// stages the pair's row-pass output for its columns as [y'][cw] and the
// column maxima, then thread (column j, segment s) takes the target rows
// y_t = 2*y0 + v_y of one segment of y0, chaining the argmax from one target
// to the next.  All lanes of a wavefront scan the union of their windows, so
// every LDS read of the scan is one row of the tile (no bank conflicts) and
// the loop is uniform.  Maximises the row-pass value minus
// (d_y (y'-y_t) + d_yy (y'-y_t)^2) over y' and writes the deformed part score
// and the (dy, dx) placement offset of (map, part, y0, x0) straight into the
// caller's layout.
__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

template <bool STAGED>
__global__ __launch_bounds__(256) void dt_col_kernel(const DTItem* __restrict__ items,
                                                     const int32_t* __restrict__ prefix,
                                                     int n_items,
                                                     const PairDesc* __restrict__ pairs,
                                                     const MapDesc* __restrict__ maps,
                                                     const float* __restrict__ r1v,
                                                     const int32_t* __restrict__ r1a,
                                                     float* __restrict__ dbuf,
                                                     int16_t* __restrict__ offs) {
    extern __shared__ float sline[];               // [Hp][cw] when STAGED
    __shared__ float smax[256];
    const int it = find_item(prefix, n_items, blockIdx.x);
    const DTItem I = items[it];
    const int local = blockIdx.x - prefix[it];
    const int cw = I.cw;                           // columns per block
    const int xc = (I.Wt + cw - 1) / cw;
    const int pidx = local / xc;                   // block-uniform
    const int xb = (local - pidx * xc) * cw;       // first column of the block
    const PairDesc P = pairs[I.pair_base + pidx];
    const MapDesc Md = maps[I.map_base + P.comp];
    const int Ho_c = Md.Ho, Wo_c = Md.Wo;
    if (Ho_c <= 0 || xb >= Wo_c) return;           // block-uniform
    const int nseg = 256 / cw;                     // >= 1
    const int j = threadIdx.x % cw, sg = threadIdx.x / cw;
    const int x0 = xb + j;
    const int xt = 2 * x0 + P.vx;
    const bool colok = x0 < Wo_c && xt >= 0 && xt < I.Wp;
    const int Hp = I.Hp;
    const int64_t lbase = I.r1_off + (int64_t)pidx * Hp * I.Wt;   // this pair's [y'][Wt] plane
    float M = -FLT_MAX;
    if (sg < nseg) {                               // 8 loads in flight per thread
        const int64_t cbase = lbase + (colok ? x0 : 0);
        for (int yb = sg; yb < Hp; yb += 8 * nseg) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = r1v[cbase + (int64_t)min(yb + u * nseg, Hp - 1) * I.Wt];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int y = yb + u * nseg;
                if (y < Hp) {
                    const float vv = colok ? v[u] : 0.f;
                    if (STAGED) sline[y * cw + j] = vv;
                    M = fmaxf(M, vv);
                }
            }
        }
    }
    smax[threadIdx.x] = M;
    __syncthreads();
    const bool act = sg < nseg && x0 < Wo_c;
    if (act)
        for (int i = 0; i < nseg; ++i) M = fmaxf(M, smax[i * cw + j]);
    const int chunk = (Ho_c + nseg - 1) / nseg;
    const int k0 = sg * chunk, k1 = act ? min(k0 + chunk, Ho_c) : k0;
    const int64_t plane = (int64_t)Ho_c * Wo_c;
    float* dout = dbuf + (Md.offs_off >> 1) + P.slot * plane + x0;
    int32_t* oout = offs ? reinterpret_cast<int32_t*>(offs + Md.offs_off) + P.slot * plane + x0 : nullptr;
    const LineConst c{P.d[3], P.d[2], 0.5f / P.d[3], 0.f, M};
    // a wavefront whose lanes all lie in one segment (same targets) scans the
    // union of its lanes' windows; otherwise every lane scans its own window
    const int wfirst = threadIdx.x & ~63;
    const bool one_seg = wfirst / cw == (wfirst + 63) / cw;
    const int kmax = wave_max_i(k1 - k0);
    int prev = 0;
    for (int kk = 0; kk < kmax; ++kk) {
        const int k = k0 + kk;
        const bool live = k < k1;
        const int t = 2 * k + P.vy;
        const bool ok = live && colok && t >= 0 && t < Hp;
        int lo = INT_MAX, hi = INT_MIN;
        if (ok) {
            if (STAGED) dt_bounds(sline[t * cw + j], c, t, prev, Hp, lo, hi);
            else dt_bounds(r1v[lbase + (int64_t)t * I.Wt + x0], c, t, prev, Hp, lo, hi);
        }
        const int LO = wave_min_i(lo), HI = wave_max_i(hi);
        float best = -INFINITY;
        int ay = -1;
        if (ok) {
            const int from = (STAGED && one_seg) ? LO : lo;
            const int to = (STAGED && one_seg) ? HI : hi;
            if (STAGED)
                best = scan_range([&](int y) { return sline[y * cw + j]; }, from, to, t, c.a, c.b, ay);
            else
                best = scan_range([&](int y) { return r1v[lbase + (int64_t)y * I.Wt + x0]; }, from, to, t, c.a, c.b, ay);
            prev = ay;
        }
        if (live) {
            int32_t packed = 0;
            if (ok) {
                const int dx = r1a[lbase + (int64_t)ay * I.Wt + x0] - xt;
                const int dy = ay - t;
                packed = (int32_t)(((uint32_t)(uint16_t)(int16_t)dx << 16) | (uint16_t)(int16_t)dy);
            }
            dout[k * Wo_c] = best;
            if (oout) oout[k * Wo_c] = packed;
        }
    }
}

// Assembly: thread = (map, root position); adds the parts' deformed scores to
// the root response (Section 2 score formula).
__global__ __launch_bounds__(ASM_BLOCK) void assemble_kernel(const MapDesc* __restrict__ maps,
                                                             const int32_t* __restrict__ prefix,
                                                             int n_maps,
                                                             const float* __restrict__ rresp,
                                                             const float* __restrict__ dbuf,
                                                             float* __restrict__ scores) {
    const int mi = find_item(prefix, n_maps, blockIdx.x);
    const MapDesc Md = maps[mi];
    const int pos = (blockIdx.x - prefix[mi]) * ASM_BLOCK + threadIdx.x;
    const int plane = Md.Ho * Md.Wo;
    if (pos >= plane) return;
    float s = rresp[Md.rresp_off + (int64_t)pos * Md.rng + Md.rcol];
    const float* d = dbuf + (Md.offs_off >> 1) + pos;
    for (int i = 0; i < Md.n_parts; ++i) s += d[(int64_t)i * plane];
    scores[Md.score_off + pos] = s;
}

template <class K>
static hipError_t set_lds(K kern, size_t lds) {
    if (lds <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t launch_dt_row(const DTItem* items, const int32_t* prefix, int n_items, int n_blocks,
                         const PairDesc* pairs, const float* resp, float* r1v, int32_t* r1a,
                         int max_line, hipStream_t st) {
    if (n_blocks <= 0) return hipSuccess;
    const size_t lds = (size_t)((((max_line + 2) >> 1) | 1) * 2) * DT_ROW_PAIRS * sizeof(float);
    if (lds <= DT_STAGE_MAX) {
        hipError_t e = set_lds(dt_row_kernel<true>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(dt_row_kernel<true>, dim3(n_blocks), dim3(256), lds, st, items, prefix,
                           n_items, pairs, resp, r1v, r1a);
    } else {
        hipLaunchKernelGGL(dt_row_kernel<false>, dim3(n_blocks), dim3(256), 0, st, items, prefix,
                           n_items, pairs, resp, r1v, r1a);
    }
    return hipGetLastError();
}

hipError_t launch_dt_col(const DTItem* items, const int32_t* prefix, int n_items, int n_blocks,
                         const PairDesc* pairs, const MapDesc* maps, const float* r1v,
                         const int32_t* r1a, float* dbuf, int16_t* offs, int max_line,
                         hipStream_t st) {
    if (n_blocks <= 0) return hipSuccess;
    const size_t lds = (size_t)max_line * sizeof(float);    // largest Hp * cw
    if (lds <= DT_STAGE_MAX) {
        hipError_t e = set_lds(dt_col_kernel<true>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(dt_col_kernel<true>, dim3(n_blocks), dim3(256), lds, st, items, prefix,
                           n_items, pairs, maps, r1v, r1a, dbuf, offs);
    } else {
        hipLaunchKernelGGL(dt_col_kernel<false>, dim3(n_blocks), dim3(256), 0, st, items, prefix,
                           n_items, pairs, maps, r1v, r1a, dbuf, offs);
    }
    return hipGetLastError();
}

hipError_t launch_assemble(const MapDesc* maps, const int32_t* prefix, int n_maps, int n_blocks,
                           const float* rresp, const float* dbuf, float* scores, hipStream_t st) {
    if (n_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(assemble_kernel, dim3(n_blocks), dim3(ASM_BLOCK), 0, st, maps, prefix,
                       n_maps, rresp, dbuf, scores);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// [pos][ng] response block -> one row-major map per filter
// ---------------------------------------------------------------------------
__global__ void block_to_maps_kernel(const float* __restrict__ block, int64_t n_pos, int ng,
                                     const int64_t* __restrict__ dst_off, float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n_pos * ng) return;
    const int64_t pos = i / ng;
    const int f = (int)(i - pos * ng);
    out[dst_off[f] + pos] = block[i];
}

hipError_t launch_block_to_maps(const float* block, int64_t n_pos, int ng, const int64_t* dst_off,
                                float* out, hipStream_t st) {
    const int64_t n = n_pos * ng;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(block_to_maps_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       block, n_pos, ng, dst_off, out);
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

}  // namespace dpmt
