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
//                      every root position; exact windowed search
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

template <int PB>
struct AFrag;  // 16-byte fragment load from LDS with the alignment PB allows

__device__ __forceinline__ uint4 lds_load16(const char* p, int pb) {
    if (pb >= 16) return *reinterpret_cast<const uint4*>(p);
    const uint2 a = *reinterpret_cast<const uint2*>(p);
    const uint2 b = *reinterpret_cast<const uint2*>(p + 8);
    return make_uint4(a.x, a.y, b.x, b.y);
}

template <CorrKind KIND>
__device__ __forceinline__ v16f mfma_step(const uint4& a, const uint4& b, v16f c) {
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

template <CorrKind KIND, int PB, int TY, int BB, int WY>
__global__ __launch_bounds__(64 * WY) void corr_kernel(const CorrTile* __restrict__ tiles,
                                                       const GroupDesc* __restrict__ groups,
                                                       const char* __restrict__ Z,
                                                       const char* __restrict__ G,
                                                       float* __restrict__ out, int cell_bytes,
                                                       int Q, int win_bytes) {
    extern __shared__ __align__(16) char smem[];
    constexpr int NT = 64 * WY;
    constexpr int TYWG = TY * WY;
    constexpr int CH = PB >= 16 ? 16 : 8;          // window copy granule
    constexpr int PFMAX = (BB * CORR_MAX_H + WY - 1) / WY;   // prefetch uint4 per thread

    const CorrTile t = tiles[blockIdx.x];
    const GroupDesc g = groups[t.group];
    const int h = g.h, S = g.S;
    const int WC = 31 + (32 * S) / PB;             // window cells per row
    const int pitch = WC * PB;
    const int nrows = TYWG + h - 1;
    char* win = smem;
    uint4* gbuf0 = reinterpret_cast<uint4*>(smem + win_bytes);
    uint4* gbuf1 = gbuf0 + BB * h * 64;

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

    const int n_chunk = BB * h * 64;               // uint4 per G chunk
    const int total = Q * S;
    auto chunk_src = [&](int step, int i) -> const uint4* {
        const int q = step / S, s = step - q * S;
        const int l = i & 63;
        const int n = (i >> 6) % h;
        const int b = i / (64 * h);
        const int64_t blk = t.fb0 + b;
        return reinterpret_cast<const uint4*>(
                   G + g.g_off + ((((blk * Q + q) * S + s) * (int64_t)h + n) << 10)) + l;
    };

    // prologue: chunk 0 straight into buffer 0
    for (int i = tid; i < n_chunk; i += NT) gbuf0[i] = *chunk_src(0, i);

    for (int step = 0; step < total; ++step) {
        const int q = step / S, s = step - q * S;
        if (s == 0) {
            __syncthreads();                       // previous plane fully consumed
            const int cpc = PB / CH;
            const int nch = nrows * WC * cpc;
            for (int i = tid; i < nch; i += NT) {
                const int k = i % cpc;
                const int cc = (i / cpc) % WC;
                const int r = i / (cpc * WC);
                const int y = t.y0 + r, x = t.x0 + cc;
                char* dst = win + r * pitch + cc * PB + k * CH;
                const bool in = (y < t.H) && (x < t.W);
                const char* src = Z + ((t.z_cell + (int64_t)y * t.W + x) * cell_bytes + q * PB + k * CH);
                if constexpr (CH == 16) {
                    *reinterpret_cast<uint4*>(dst) = in ? *reinterpret_cast<const uint4*>(src)
                                                        : make_uint4(0, 0, 0, 0);
                } else {
                    *reinterpret_cast<uint2*>(dst) = in ? *reinterpret_cast<const uint2*>(src)
                                                        : make_uint2(0, 0);
                }
            }
        }
        __syncthreads();                           // window and chunk `step` visible

        uint4 pf[PFMAX];
        const bool more = step + 1 < total;
        if (more) {
#pragma unroll
            for (int k = 0; k < PFMAX; ++k) {
                const int i = tid + k * NT;
                if (i < n_chunk) pf[k] = *chunk_src(step + 1, i);
            }
        }

        const uint4* gb = (step & 1) ? gbuf1 : gbuf0;
        const char* abase = win + (wv * TY) * pitch + p * PB + 32 * s + 16 * j;
        uint4 A[TY];
#pragma unroll
        for (int i = 0; i < TY; ++i) A[i] = lds_load16(abase + i * pitch, PB);
        for (int n = 0; n < h; ++n) {
            uint4 B[BB];
#pragma unroll
            for (int b = 0; b < BB; ++b) B[b] = gb[(b * h + n) * 64 + lane];
#pragma unroll
            for (int i = 0; i < TY; ++i)
#pragma unroll
                for (int b = 0; b < BB; ++b) acc[i][b] = mfma_step<KIND>(A[i], B[b], acc[i][b]);
            if (n + 1 < h) {
#pragma unroll
                for (int i = 0; i + 1 < TY; ++i) A[i] = A[i + 1];
                A[TY - 1] = lds_load16(abase + (n + TY) * pitch, PB);
            }
        }

        if (more) {
            uint4* nb = (step & 1) ? gbuf0 : gbuf1;
#pragma unroll
            for (int k = 0; k < PFMAX; ++k) {
                const int i = tid + k * NT;
                if (i < n_chunk) nb[i] = pf[k];
            }
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

template <CorrKind KIND, int PB, int TY, int BB, int WY>
static hipError_t launch_corr_t(const CorrTile* tiles, int n_tiles, const GroupDesc* groups,
                                const void* Z, const void* G, float* out, int cell_bytes, int Q,
                                int max_h, int max_S, hipStream_t st) {
    CorrLaunch cfg{KIND, Packing{0, 0, PB, Q}, TY, BB, WY};
    const size_t lds = corr_lds_bytes(cfg, max_h, max_S);
    const int WC = 31 + (32 * max_S) / PB;
    const size_t win = (size_t)(TY * WY + max_h - 1) * WC * PB;
    const int win_bytes = (int)((win + 15) & ~size_t(15));
    auto kern = corr_kernel<KIND, PB, TY, BB, WY>;
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
// distance transform helpers
//
// For a target t on a line with values v[0..n) and cost c(u) = b*u + a*u^2
// (u = position - t, a > 0), a position u can only beat the target itself if
// c(u - t) <= v[u] - v[t] <= M - v[t], M the line maximum.  Solving the
// quadratic gives a window [t + lo, t + hi] that holds every possible
// maximiser; scanning any superset of it in ascending order with a strict >
// returns the exact maximum and its smallest maximiser.  Lanes of a wave scan
// the union of their windows so that the loads stay coalesced.
// ---------------------------------------------------------------------------
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

__device__ __forceinline__ void dt_window(float M, float vt, float a, float b, int t, int n, int& lo,
                                          int& hi) {
    const float delta = fmaxf(M - vt, 0.f);
    const float s = sqrtf(fmaf(4.f * a, delta, b * b));
    const float inv = 0.5f / a;
    const float ulo = floorf((-b - s) * inv) - 1.f;
    const float uhi = ceilf((-b + s) * inv) + 1.f;
    // clamp in float first: a huge window (tiny a, large range) must not overflow int
    lo = t + (int)fmaxf(ulo, -(float)n);
    hi = t + (int)fminf(uhi, (float)n);
    lo = max(lo, 0);
    hi = min(hi, n - 1);
}

__device__ __forceinline__ int find_item(const int32_t* __restrict__ prefix, int n, int b) {
    int lo = 0, hi = n - 1;                        // last item with prefix <= b
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Row pass: thread = (pair, part row y').  For every root column x0 of the
// pair's component the target is x_t = 2*x0 + v_x; writes the row maximum of
// resp[y'][x'] - (d_x (x'-x_t) + d_xx (x'-x_t)^2) and its argmax x'.
__global__ __launch_bounds__(256) void dt_row_kernel(const DTItem* __restrict__ items,
                                                     const int32_t* __restrict__ prefix,
                                                     int n_items,
                                                     const PairDesc* __restrict__ pairs,
                                                     const float* __restrict__ resp,
                                                     float* __restrict__ r1v,
                                                     int32_t* __restrict__ r1a) {
    const int it = find_item(prefix, n_items, blockIdx.x);
    const DTItem I = items[it];
    const int local = blockIdx.x - prefix[it];
    const int pc = (I.np + 63) >> 6;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int pidx = (local % pc) * 64 + lane;
    const int yp = (local / pc) * DT_ROWS_PER_BLOCK + wv;
    if (yp >= I.Hp) return;                        // wave-uniform
    const bool active = pidx < I.np;
    const PairDesc P = pairs[I.pair_base + (active ? pidx : 0)];
    const int64_t rs = I.ng;                       // element stride along x'
    const float* row = resp + I.resp_off + (int64_t)yp * I.Wp * rs + P.fcol;
    const int Wp = I.Wp;

    float M = -FLT_MAX;
    if (active)
        for (int x = 0; x < Wp; ++x) M = fmaxf(M, row[x * rs]);

    const int Wo_c = I.Wr - P.w0 + 1;
    const float b = P.d[0], a = P.d[1];
    float* ov = r1v + I.r1_off + (int64_t)yp * I.Wt * I.np;
    int32_t* oa = r1a + I.r1_off + (int64_t)yp * I.Wt * I.np;
    for (int x0 = 0; x0 < I.Wt; ++x0) {
        const int xt = 2 * x0 + P.vx;
        const bool ok = active && x0 < Wo_c && xt >= 0 && xt < Wp;
        int lo = INT_MAX, hi = INT_MIN;
        if (ok) dt_window(M, row[xt * rs], a, b, xt, Wp, lo, hi);
        const int LO = wave_min_i(lo), HI = wave_max_i(hi);
        float best = -INFINITY;
        int arg = -1;
        if (ok) {
            for (int x = LO; x <= HI; ++x) {
                const float u = (float)(x - xt);
                const float val = row[x * rs] - u * fmaf(a, u, b);
                if (val > best) { best = val; arg = x; }
            }
        }
        if (active) {
            ov[(int64_t)x0 * I.np + pidx] = best;
            oa[(int64_t)x0 * I.np + pidx] = arg;
        }
    }
}

// Column pass + placement: thread = (pair, root column x0).  For every root
// row y0 the target is y_t = 2*y0 + v_y; maximises the row-pass value minus
// (d_y (y'-y_t) + d_yy (y'-y_t)^2) over y', then writes the deformed part score
// D and the (dy, dx) placement offset of the component's map.
__global__ __launch_bounds__(256) void dt_col_kernel(const DTItem* __restrict__ items,
                                                     const int32_t* __restrict__ prefix,
                                                     int n_items,
                                                     const PairDesc* __restrict__ pairs,
                                                     const MapDesc* __restrict__ maps,
                                                     const float* __restrict__ r1v,
                                                     const int32_t* __restrict__ r1a,
                                                     float* __restrict__ dbuf,
                                                     int16_t* __restrict__ offs) {
    const int it = find_item(prefix, n_items, blockIdx.x);
    const DTItem I = items[it];
    const int local = blockIdx.x - prefix[it];
    const int pc = (I.np + 63) >> 6;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int pidx = (local % pc) * 64 + lane;
    const int x0 = (local / pc) * DT_COLS_PER_BLOCK + wv;
    if (x0 >= I.Wt) return;                        // wave-uniform
    const bool active = pidx < I.np;
    const PairDesc P = pairs[I.pair_base + (active ? pidx : 0)];
    const MapDesc Md = maps[I.map_base + P.comp];
    const int Ho_c = Md.Ho, Wo_c = Md.Wo;
    const int xt = 2 * x0 + P.vx;
    const bool colok = active && x0 < Wo_c && xt >= 0 && xt < I.Wp;
    const int64_t cs = (int64_t)I.Wt * I.np;       // element stride along y'
    const float* col = r1v + I.r1_off + (int64_t)x0 * I.np + pidx;
    const int32_t* cola = r1a + I.r1_off + (int64_t)x0 * I.np + pidx;
    const int Hp = I.Hp;

    float M = -FLT_MAX;
    if (colok)
        for (int y = 0; y < Hp; ++y) M = fmaxf(M, col[y * cs]);

    const float b = P.d[2], a = P.d[3];
    const int64_t plane = (int64_t)Ho_c * Wo_c;
    for (int y0 = 0; y0 < I.Ht; ++y0) {
        const int yt = 2 * y0 + P.vy;
        const bool ok = colok && y0 < Ho_c && yt >= 0 && yt < Hp;
        int lo = INT_MAX, hi = INT_MIN;
        if (ok) dt_window(M, col[yt * cs], a, b, yt, Hp, lo, hi);
        const int LO = wave_min_i(lo), HI = wave_max_i(hi);
        float best = -INFINITY;
        int argy = -1;
        if (ok) {
            for (int y = LO; y <= HI; ++y) {
                const float u = (float)(y - yt);
                const float val = col[y * cs] - u * fmaf(a, u, b);
                if (val > best) { best = val; argy = y; }
            }
        }
        if (active && x0 < Wo_c && y0 < Ho_c) {
            const int64_t pos = (int64_t)y0 * Wo_c + x0;
            dbuf[Md.dbuf_off + P.slot * plane + pos] = ok ? best : -INFINITY;
            if (offs) {
                int dy = 0, dx = 0;
                if (ok) {
                    dy = argy - yt;
                    dx = cola[argy * cs] - xt;
                }
                int16_t* o = offs + Md.offs_off + (P.slot * plane + pos) * 2;
                o[0] = (int16_t)dy;
                o[1] = (int16_t)dx;
            }
        }
    }
}

// Assembly: thread = (map, root position).
__global__ __launch_bounds__(ASM_BLOCK) void assemble_kernel(const MapDesc* __restrict__ maps,
                                                             const int32_t* __restrict__ prefix,
                                                             int n_maps,
                                                             const float* __restrict__ rresp,
                                                             const float* __restrict__ dbuf,
                                                             float* __restrict__ scores) {
    const int m = find_item(prefix, n_maps, blockIdx.x);
    const MapDesc Md = maps[m];
    const int64_t pos = (int64_t)(blockIdx.x - prefix[m]) * ASM_BLOCK + threadIdx.x;
    const int64_t plane = (int64_t)Md.Ho * Md.Wo;
    if (pos >= plane) return;
    float s = rresp[Md.rresp_off + pos * Md.rng + Md.rcol];
    for (int i = 0; i < Md.n_parts; ++i) s += dbuf[Md.dbuf_off + i * plane + pos];
    scores[Md.score_off + pos] = s;
}

hipError_t launch_dt_row(const DTItem* items, const int32_t* prefix, int n_items, int n_blocks,
                         const PairDesc* pairs, const float* resp, float* r1v, int32_t* r1a,
                         hipStream_t st) {
    if (n_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(dt_row_kernel, dim3(n_blocks), dim3(64 * DT_ROWS_PER_BLOCK), 0, st, items,
                       prefix, n_items, pairs, resp, r1v, r1a);
    return hipGetLastError();
}

hipError_t launch_dt_col(const DTItem* items, const int32_t* prefix, int n_items, int n_blocks,
                         const PairDesc* pairs, const MapDesc* maps, const float* r1v,
                         const int32_t* r1a, float* dbuf, int16_t* offs, hipStream_t st) {
    if (n_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(dt_col_kernel, dim3(n_blocks), dim3(64 * DT_COLS_PER_BLOCK), 0, st, items,
                       prefix, n_items, pairs, maps, r1v, r1a, dbuf, offs);
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
// single-map distance transform for every target cell
// ---------------------------------------------------------------------------
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

// thread = target (y, x), x fastest; scans along x (row pass)
__global__ void dt1_row_kernel(const float* __restrict__ v, int rows, int cols, int64_t ld,
                               const float* __restrict__ M, float a, float b,
                               float* __restrict__ ov, int32_t* __restrict__ oa) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool ok = i < (int64_t)rows * cols;
    const int y = ok ? (int)(i / cols) : 0;
    const int xt = ok ? (int)(i - (int64_t)y * cols) : 0;
    const float* row = v + y * ld;
    int lo = INT_MAX, hi = INT_MIN;
    if (ok) dt_window(M[y], row[xt], a, b, xt, cols, lo, hi);
    const int LO = wave_min_i(lo), HI = wave_max_i(hi);
    if (!ok) return;
    float best = -INFINITY;
    int arg = -1;
    for (int x = max(LO, 0); x <= min(HI, cols - 1); ++x) {
        const float u = (float)(x - xt);
        const float val = row[x] - u * fmaf(a, u, b);
        if (val > best) { best = val; arg = x; }
    }
    ov[i] = best;
    oa[i] = arg;
}

// thread = target (y, x), x fastest; scans along y (column pass)
__global__ void dt1_col_kernel(const float* __restrict__ r1v, const int32_t* __restrict__ r1a,
                               int rows, int cols, const float* __restrict__ M, float a, float b,
                               float* __restrict__ out, int32_t* __restrict__ ay,
                               int32_t* __restrict__ ax) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool ok = i < (int64_t)rows * cols;
    const int yt = ok ? (int)(i / cols) : 0;
    const int x = ok ? (int)(i - (int64_t)yt * cols) : 0;
    int lo = INT_MAX, hi = INT_MIN;
    if (ok) dt_window(M[x], r1v[(int64_t)yt * cols + x], a, b, yt, rows, lo, hi);
    const int LO = wave_min_i(lo), HI = wave_max_i(hi);
    if (!ok) return;
    float best = -INFINITY;
    int arg = -1;
    for (int y = max(LO, 0); y <= min(HI, rows - 1); ++y) {
        const float u = (float)(y - yt);
        const float val = r1v[(int64_t)y * cols + x] - u * fmaf(a, u, b);
        if (val > best) { best = val; arg = y; }
    }
    out[i] = best;
    if (ay) ay[i] = arg;
    if (ax) ax[i] = r1a[(int64_t)arg * cols + x];
}

hipError_t launch_dt_single(const float* resp, int rows, int cols, int ld, const float* d,
                            float* rowmax, float* r1v, int32_t* r1a, float* out, int32_t* ay,
                            int32_t* ax, hipStream_t st) {
    const int64_t n = (int64_t)rows * cols;
    if (n <= 0) return hipSuccess;
    const unsigned nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(dt1_rowmax_kernel, dim3((rows + 255) / 256), dim3(256), 0, st, resp, rows,
                       cols, (int64_t)ld, rowmax);
    hipLaunchKernelGGL(dt1_row_kernel, dim3(nb), dim3(256), 0, st, resp, rows, cols, (int64_t)ld,
                       rowmax, d[1], d[0], r1v, r1a);
    hipLaunchKernelGGL(dt1_colmax_kernel, dim3((cols + 255) / 256), dim3(256), 0, st, r1v, rows,
                       cols, rowmax);
    hipLaunchKernelGGL(dt1_col_kernel, dim3(nb), dim3(256), 0, st, r1v, r1a, rows, cols, rowmax,
                       d[3], d[2], out, ay, ax);
    return hipGetLastError();
}

}  // namespace dpmt
